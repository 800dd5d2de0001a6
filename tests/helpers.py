"""Small test-side utilities (no method arithmetic): marker coordinates and the
paper's error metrics (Sec. 3.2, Eqs. Eq_error_surface and Eq_error_shape)."""
import numpy as np


def markers_xy(st):
    """Index-space coordinates of every marker of a host State."""
    hp = st.h_present()
    jj, ii = np.nonzero(hp)
    xs = ii + st.hoff[jj, ii]
    ys = jj.astype(np.float64)
    vp = st.v_present()
    jj2, ii2 = np.nonzero(vp)
    xs2 = ii2.astype(np.float64)
    ys2 = jj2 + st.voff[jj2, ii2]
    return np.concatenate([xs, xs2]), np.concatenate([ys, ys2])


def e_area(C0, C1):
    a0 = float(np.sum(C0))
    return abs(float(np.sum(C1)) - a0) / a0


def e_shape(st, cx, cy, r):
    """max_i |dist(x_i) - R| in index units."""
    X, Y = markers_xy(st)
    return float(np.max(np.abs(np.hypot(X - cx, Y - cy) - r)))


def cell_marker_count(c):
    """Markers per cell from a node-colour array (ny+1, nx+1)."""
    bl = c[:-1, :-1]
    br = c[:-1, 1:]
    tr = c[1:, 1:]
    tl = c[1:, :-1]
    return ((bl != br).astype(int) + (br != tr) + (tl != tr) + (bl != tl))


def circle_cell_fractions(nx, ny, cx, cy, r):
    """Exact area fraction of the disc in every cell (index units), by
    integrating the clipped chord height over each cell column."""
    from scipy.integrate import quad
    C = np.zeros((ny, nx))
    for i in range(max(int(np.floor(cx - r)), 0), min(int(np.ceil(cx + r)), nx)):
        x0, x1 = max(i, cx - r), min(i + 1, cx + r)
        if x1 <= x0:
            continue
        for j in range(max(int(np.floor(cy - r)), 0), min(int(np.ceil(cy + r)), ny)):
            def seg(x, j=j):
                w = np.sqrt(max(r * r - (x - cx) ** 2, 0.0))
                lo, hi = max(j, cy - w), min(j + 1, cy + w)
                return max(hi - lo, 0.0)
            pts = [x for x in (cx - np.sqrt(max(r * r - (j - cy) ** 2, 0)), cx + np.sqrt(max(r * r - (j - cy) ** 2, 0)),
                               cx - np.sqrt(max(r * r - (j + 1 - cy) ** 2, 0)),
                               cx + np.sqrt(max(r * r - (j + 1 - cy) ** 2, 0))) if x0 < x < x1]
            val, _ = quad(seg, x0, x1, points=pts or None, epsabs=1e-14, epsrel=1e-13, limit=200)
            C[j, i] = val
    return C
