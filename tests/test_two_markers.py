"""Pins of the two-markers-per-edge oracle (oracle/two_markers.py), the
kinematic extension Sec. 2.4 and Sec. 4 propose for thin films.

  - With films forbidden (rupture gap delta = inf) it reduces exactly to the
    one-marker oracle: colours, centre colours and offsets bit-identical, C
    within rounding, on smooth, dense random and checkerboard states; so its
    boundary pairing, crossing rule, centre rule and fraction generalise the
    pinned one-marker ones rather than replacing them.
  - A film squeezed by a linear converging flow u = -k (x - xm) (bilinear
    interpolation is exact for it) has walls that follow the explicit Euler
    map x' = xm + (1 - k)(x - xm) exactly; when both walls reach one cell
    column the film is kept as a pair of markers on every crossed edge, its
    area equals its width times its height, and it ruptures in exactly the
    step its width falls below delta. The one-marker method loses the same
    film the moment it becomes sub-cell (Sec. 2.4: structures below the grid
    size are removed).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import two_markers as T
from paper_2309_00338_amd import inputs as I


def _cases():
    out = []
    for n, kind, seed in ((24, "smooth", 0), (20, "dense", 1), (16, "dense", 3), (12, "checker", 4)):
        if kind == "smooth":
            st = I.init_state(n, n, [I.Circle(n * 0.4, n * 0.5, n * 0.2), I.Ellipse(n * 0.72, n * 0.45, n * 0.14,
                                                                                       n * 0.08, 0.7)], h=1.0 / n)
            u, v = I.vortex_faces(n)
            dt = 0.45 * st.h / max(abs(u).max(), abs(v).max())
        elif kind == "dense":
            st = I.random_colouring(n, n, seed=seed)
            u, v = I.shear_faces(n, n, seed + 9)
            dt = 0.45 * st.h / max(abs(u).max(), abs(v).max())
        else:
            st = I.checkerboard(n, n, seed=seed)
            u, v = I.shear_faces(n, n, seed + 9)
            dt = 0.2 * st.h / max(abs(u).max(), abs(v).max())
        out.append((kind, n, st, u, v, dt))
    return out


@pytest.mark.parametrize("case", range(4))
def test_without_films_it_is_the_one_marker_method(case):
    kind, n, st, u, v, dt = _cases()[case]
    f, o = T.Film.from_state(st), st.copy()
    for k in range(4):
        f = T.step(f, u, v, dt, math.inf)
        f.check()
        assert oracle.step(o, u, v, dt)[0] == oracle.OK
        assert np.array_equal(f.c, o.c) and np.array_equal(f.cc, o.cc), (kind, k)
        h1, h2, v1, v2 = T.to_arrays(f)
        hp, vp = o.h_present(), o.v_present()
        assert np.isnan(h2).all() and np.isnan(v2).all()
        assert np.array_equal(h1[hp], o.hoff[hp]) and np.array_equal(v1[vp], o.voff[vp]), (kind, k)
    assert np.abs(T.fraction(f) - oracle.fraction(o)).max() < 1e-15


def _film(n=16, x1=7.2, x2=8.9):
    """A vertical film x1 < x < x2 (cell units) over the whole height, colour 1,
    one marker per crossed horizontal edge at each wall."""
    c = np.zeros((n + 1, n + 1), np.uint8)
    for i in range(n + 1):
        c[:, i] = 1 if x1 < i < x2 else 0
    cc = np.zeros((n, n), np.uint8)
    for i in range(n):
        cc[:, i] = 1 if x1 < i + 0.5 < x2 else 0
    H = [[[] for _ in range(n)] for _ in range(n + 1)]
    for j in range(n + 1):
        for x in (x1, x2):
            H[j][int(math.floor(x))].append(x - math.floor(x))
    V = [[[] for _ in range(n + 1)] for _ in range(n)]
    return T.Film(n, n, 1.0 / n, c, cc, H, V)


def test_squeezed_film_survives_as_pairs_and_ruptures_at_the_gap():
    n, k, xm, delta = 16, 0.25, 8.05, 0.05
    f = _film(n)
    lam = 1.0  # dt = h
    u = np.zeros((n, n + 1))
    for i in range(n + 1):
        u[:, i] = -k * (i - xm) / lam
    v = np.zeros((n + 1, n))
    w0 = 1.7
    one = f.copy()
    rupture = None
    for s in range(1, 16):
        stats = T.new_stats()
        f = T.step(f, u, v, f.h * lam, delta, stats)
        f.check()
        one = T.step(one, u, v, one.h * lam, math.inf)
        w = w0 * (1.0 - k) ** s
        C = T.fraction(f)
        if w >= delta:
            # every crossed edge holds the walls at the Euler map's positions
            for j in range(n + 1):
                xs = sorted(i + o for i in range(n) for o in f.H[j][i])
                assert len(xs) == 2
                assert abs(xs[0] - (xm - 0.85 * (1 - k) ** s)) < 1e-12 and abs(xs[1] - (xm + 0.85 * (1 - k) ** s)) < 1e-12
            assert abs(C.sum() - w * n) < 1e-11, (s, C.sum(), w * n)
            if int(math.floor(xs[0])) == int(math.floor(xs[1])):
                # sub-cell: one pair per edge, every node outside the film's colour
                assert all(len(f.H[j][int(xs[0])]) == 2 for j in range(n + 1)) and f.c.sum() == 0
        else:
            rupture = s
            assert stats["annihilated"] == 2 * (n + 1) and C.sum() == 0.0
            break
    assert rupture == 13  # 1.7 * 0.75**13 = 0.040 < 0.05 <= 1.7 * 0.75**12
    # the one-marker method removes the film in the step both walls first share an edge
    g = _film(n)
    lost = None
    for s in range(1, 16):
        g = T.step(g, u, v, g.h * lam, math.inf)
        if T.fraction(g).sum() == 0.0:
            lost = s
            break
    assert lost == 10  # 8.05 - 0.85 * 0.75**10 >= 8: the left wall crosses node 8
    assert one.c.sum() == 0


def test_fraction_of_a_film_cell_is_its_width():
    """A cell crossed by a vertical film between x = 0.3 and 0.55 (pairs on its
    bottom and top edges, centre colour 1): C = 0.25; a slanted film gives the
    trapezoid of its two walls."""
    c = np.zeros((5, 5), np.uint8)
    H = [[[] for _ in range(4)] for _ in range(5)]
    V = [[[] for _ in range(5)] for _ in range(4)]
    H[1][1] = [0.3, 0.55]
    H[2][1] = [0.3, 0.55]
    cc = np.zeros((4, 4), np.uint8)
    cc[1, 1] = 1
    C = T.fraction(T.Film(4, 4, 0.25, c, cc, H, V))
    assert abs(C[1, 1] - 0.25) < 1e-15
    H[2][1] = [0.1, 0.45]
    C = T.fraction(T.Film(4, 4, 0.25, c, cc, H, V))
    assert abs(C[1, 1] - 0.5 * ((0.55 - 0.3) + (0.45 - 0.1))) < 1e-15
