"""A 50-digit reference of one EBIT sweep, for pinning the FP64 oracle's
rounding on tiny grids (test infrastructure; tests only).

It evaluates the same definitions as the oracle, written independently and
organised per output (each new marker gathers what it needs) rather than as
the oracle's global passes, in mpmath arithmetic with 50 significant digits:

  Sec. 2.1, Eq. (Eq_marker_dis): aligned markers move along their line by the
      bilinear face velocity times dt (interpolated along the line, then
      across it), unaligned ones to their gray points;
  Sec. 2.3 / 2.4: a node changes colour when an aligned marker passes it;
      the landers of an edge pair off and one survives (the middle one by
      position when three arrive);
  Sec. 2.2: a new unaligned marker is where the circle through the advected
      chain P1-P2-P3 (and the one through P2-P3-P4) meets the grid line,
      averaged, the straight chord P2-P3 as the fallback; roots by the plain
      quadratic formula (no cancellation matters at 50 digits);
  Sec. 2.3 rules (1)-(5): the centre colour of a cell follows the aligned
      candidate kept on its bottom or top edge, left line first.

Inputs are FP64 numpy arrays, converted exactly; the result is returned as
numpy arrays (offsets rounded to FP64 at the end).
"""
import mpmath as mp
import numpy as np

mp.mp.dps = 50


def _lerp(a, b, t):
    return a + t * (b - a)


def sweep_x(c, cc, hoff, voff, u, lam, line=False):
    """One x sweep. c (ny+1, nx+1), cc (ny, nx), hoff (ny+1, nx), voff
    (ny, nx+1), u (ny, nx+1). Returns the new (c, cc, hoff, voff)."""
    ny, nx = cc.shape
    lam = mp.mpf(lam)

    def U(i, r):
        r = min(max(r, 0), ny - 1)
        return mp.mpf(float(u[r, i]))

    def hpres(i, j):
        return c[j, i] != c[j, i + 1]

    def vpres(i, j):
        return c[j, i] != c[j + 1, i]

    # advected positions: aligned H(i, j) -> x = i + s + d (y = j)
    sp = {}
    for j in range(ny + 1):
        for i in range(nx):
            if hpres(i, j):
                s = mp.mpf(float(hoff[j, i]))
                ub = _lerp(_lerp(U(i, j - 1), U(i + 1, j - 1), s), _lerp(U(i, j), U(i + 1, j), s), mp.mpf("0.5"))
                sp[(i, j)] = s + ub * lam
    # gray points: V(i, j) -> (i + d, j + t); walls hold
    gray = {}
    for j in range(ny):
        for i in range(nx + 1):
            if vpres(i, j):
                t = mp.mpf(float(voff[j, i]))
                if t < mp.mpf("0.5"):
                    ub = _lerp(U(i, j - 1), U(i, j), t + mp.mpf("0.5"))
                else:
                    ub = _lerp(U(i, j), U(i, j + 1), t - mp.mpf("0.5"))
                d = mp.mpf(0) if i in (0, nx) else ub * lam
                gray[(i, j)] = (d, t)

    # new colours: a node flips when an aligned marker passes it
    nc = c.copy()
    for (i, j), s in sp.items():
        if s >= 1:
            nc[j, i + 1] ^= 1
        elif s < 0:
            nc[j, i] ^= 1

    # landers: positions (absolute x) of the markers landing on H(i, j)
    def landers(i, j):
        out = []
        for k in (i - 1, i, i + 1):
            if 0 <= k < nx and (k, j) in sp:
                s = sp[(k, j)]
                tgt = k + 1 if s >= 1 else (k - 1 if s < 0 else k)
                if tgt == i:
                    out.append((k + s, k))
        out.sort()
        return out

    nh = hoff.copy()
    kept = {}  # source edge (k, j) -> the edge it survives on
    for j in range(ny + 1):
        for i in range(nx):
            L = landers(i, j)
            if len(L) % 2 == 1:
                x, k = L[len(L) // 2]
                nh[j, i] = float(x - i)
                kept[(k, j)] = i

    # old segments of a cell: list of pairs of edge ids (0 bottom, 1 right, 2 top, 3 left)
    def segs(p, q):
        bl, br, tr, tl = c[q, p], c[q, p + 1], c[q + 1, p + 1], c[q + 1, p]
        on = [bl != br, br != tr, tl != tr, bl != tl]
        m = [e for e in range(4) if on[e]]
        if len(m) == 2:
            return [tuple(m)]
        if len(m) == 4:
            # pair around the corners whose colour differs from the centre
            if bl != cc[q, p]:
                return [(3, 0), (1, 2)]
            return [(0, 1), (2, 3)]
        return []

    def marker(p, q, e):
        return {0: ("H", p, q), 1: ("V", p + 1, q), 2: ("H", p, q + 1), 3: ("V", p, q)}[e]

    def pos(m):
        kind, i, j = m
        if kind == "H":
            return (i + sp[(i, j)], mp.mpf(j))
        d, t = gray[(i, j)]
        return (i + d, j + t)

    def neighbour(p, q, e):
        """Partner, in the cell across edge e of cell (p, q), of that edge's marker."""
        pp, qq = {0: (p, q - 1), 1: (p + 1, q), 2: (p, q + 1), 3: (p - 1, q)}[e]
        if not (0 <= pp < nx and 0 <= qq < ny):
            return None
        eo = (e + 2) % 4
        for a, b in segs(pp, qq):
            if a == eo:
                return marker(pp, qq, b)
            if b == eo:
                return marker(pp, qq, a)
        return None

    def circle_root(P, Q, R, outer, P2, P3, ysl):
        """Where the circle (or line) through P, Q, R meets X = 0, on the far
        side of chord P2-P3 from `outer`; None when it does not exist or leaves
        the edge."""
        M = mp.matrix([[P[0] ** 2 + P[1] ** 2, P[0], P[1], 1], [Q[0] ** 2 + Q[1] ** 2, Q[0], Q[1], 1],
                       [R[0] ** 2 + R[1] ** 2, R[0], R[1], 1]])
        # a (X^2 + Y^2) + b X + c Y + e = 0 through the three points
        a = mp.det(mp.matrix([[M[r, 1], M[r, 2], M[r, 3]] for r in range(3)]))
        cc_ = mp.det(mp.matrix([[M[r, 0], M[r, 1], M[r, 3]] for r in range(3)]))
        e = -mp.det(mp.matrix([[M[r, 0], M[r, 1], M[r, 2]] for r in range(3)]))
        # on X = 0: a Y^2 + c Y + e = 0 (the minors' cofactor signs: +, -, +, -)
        cY = cc_
        if a == 0:
            if cY == 0:
                return None
            roots = [-e / cY]
        else:
            disc = cY * cY - 4 * a * e
            if disc < 0:
                disc = mp.mpf(0)
            roots = [(-cY + mp.sqrt(disc)) / (2 * a), (-cY - mp.sqrt(disc)) / (2 * a)]

        def side(X, Y):
            return (P3[0] - P2[0]) * (Y - P2[1]) - (P3[1] - P2[1]) * (X - P2[0])

        so = side(*outer)
        if len(roots) == 1:
            r = roots[0]
        else:
            across = [r for r in roots if side(0, r) * so < 0]
            r = across[0] if len(across) == 1 else min(roots, key=lambda y: abs(y - ysl))
        return r if 0 <= r <= 1 else None

    nv = voff.copy()
    res = {}  # (line, row) -> (result for the cell on the right, for the cell on the left)
    for j in range(ny):
        for i in range(1, nx):
            if nc[j, i] == nc[j + 1, i]:
                continue
            cross = []
            for p in (i - 1, i):
                for ea, eb in segs(p, j):
                    ma, mb = marker(p, j, ea), marker(p, j, eb)
                    A, B = pos(ma), pos(mb)
                    la, lb = A[0] < i, B[0] < i
                    if la == lb:
                        continue
                    if not la:
                        (ea, ma, A), (eb, mb, B) = (eb, mb, B), (ea, ma, A)
                    X2, Y2, X3, Y3 = A[0] - i, A[1] - j, B[0] - i, B[1] - j
                    ysl = Y2 + (Y3 - Y2) * (0 - X2) / (X3 - X2)
                    ysl = min(max(ysl, mp.mpf(0)), mp.mpf(1))
                    cross.append((ysl, p, ea, eb, ma, mb, (X2, Y2), (X3, Y3)))
            assert len(cross) % 2 == 1, "crossing parity differs from the colours"
            cross.sort(key=lambda z: z[0])
            ysl, p, e2, e3, m2, m3, P2, P3 = cross[len(cross) // 2]
            m1 = neighbour(p, j, e2)
            m4 = neighbour(p, j, e3)
            if P3[0] == 0:
                y = P3[1]
            elif line:
                y = ysl
            else:
                got = []
                if m1 is not None:
                    X1 = pos(m1)
                    P1 = (X1[0] - i, X1[1] - j)
                    r = circle_root(P1, P2, P3, P1, P2, P3, ysl)
                    if r is not None:
                        got.append(r)
                if m4 is not None:
                    X4 = pos(m4)
                    P4 = (X4[0] - i, X4[1] - j)
                    r = circle_root(P2, P3, P4, P4, P2, P3, ysl)
                    if r is not None:
                        got.append(r)
                y = sum(got) / len(got) if got else ysl
            nv[j, i] = float(y)

            # centre rules: a candidate is an aligned marker kept on the cell's
            # bottom or top edge; it isolates the corner it shares with line i
            def rule(first, second, cell):
                for m in ([first] + ([second] if first[0] == "V" and second is not None else [])):
                    kind, k, r = m
                    if kind == "H" and r in (j, j + 1) and kept.get((k, r)) == cell:
                        return 1 - int(nc[r, i])
                return -1

            right = rule(m3, m4, i) if i < nx else -1
            left = rule(m2, m1, i - 1)
            res[(i, j)] = (right, left)

    ncc = cc.copy()
    for j in range(ny):
        for i in range(nx):
            r_left_line = res.get((i, j), (-1, -1))[0]
            r_right_line = res.get((i + 1, j), (-1, -1))[1]
            if r_left_line >= 0:
                ncc[j, i] = r_left_line
            elif r_right_line >= 0:
                ncc[j, i] = r_right_line
    return nc, ncc, nh, nv


def sweep(st, u, v, dt, direction, line=False):
    """One sweep of a State (direction 0: x with u; 1: y with v, by
    transposing the grid). Returns a new State."""
    lam = dt / st.h
    if direction == 0:
        c, cc, h, vv = sweep_x(st.c, st.cc, st.hoff, st.voff, u, lam, line)
    else:
        c, cc, vv_t, h_t = sweep_x(st.c.T.copy(), st.cc.T.copy(), st.voff.T.copy(), st.hoff.T.copy(),
                                   v.T.copy(), lam, line)
        c, cc, h, vv = c.T.copy(), cc.T.copy(), h_t.T.copy(), vv_t.T.copy()
    out = st.copy()
    out.c, out.cc, out.hoff, out.voff = c, cc, h, vv
    return out
