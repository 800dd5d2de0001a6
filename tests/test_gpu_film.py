"""GPU parity of the two-markers-per-edge step (include/ebit_film.h) with its
CPU oracle (oracle/two_markers.py): colours, centre colours, marker counts and
offsets bit-identical after every step, C within 1e-15, counters equal.

Workloads: the states the oracle's own pins use with films forbidden (delta =
inf, where the step is the one-marker method and is also checked against the
one-marker GPU path); the squeezed film of the oracle's pin, which survives as
pairs and ruptures at the gap; two circles driven into each other, whose
meeting edges keep pairs; random colourings under sheared faces (films,
three crossings and ruptures together) on square and ragged grids; and a CFL
violation reported like the oracle's."""
import math

import numpy as np
import pytest

from oracle import two_markers as T
from paper_2309_00338_amd import inputs as I

pytestmark = pytest.mark.gpu


def _to_oracle(fs):
    H = [[[float(fs.ho[j, i, k]) for k in range(fs.hn[j, i])] for i in range(fs.nx)] for j in range(fs.ny + 1)]
    V = [[[float(fs.vo[j, i, k]) for k in range(fs.vn[j, i])] for i in range(fs.nx + 1)] for j in range(fs.ny)]
    return T.Film(fs.nx, fs.ny, fs.h, fs.c, fs.cc, H, V, fs.step)


def _of_oracle(f):
    from paper_2309_00338_amd.film import FilmState

    hn = np.array([[len(f.H[j][i]) for i in range(f.nx)] for j in range(f.ny + 1)], np.uint8)
    vn = np.array([[len(f.V[j][i]) for i in range(f.nx + 1)] for j in range(f.ny)], np.uint8)
    ho = np.zeros((f.ny + 1, f.nx, 2))
    vo = np.zeros((f.ny, f.nx + 1, 2))
    for j in range(f.ny + 1):
        for i in range(f.nx):
            for k, o in enumerate(f.H[j][i]):
                ho[j, i, k] = o
    for j in range(f.ny):
        for i in range(f.nx + 1):
            for k, o in enumerate(f.V[j][i]):
                vo[j, i, k] = o
    return FilmState(f.nx, f.ny, f.h, np.array(f.c, np.uint8), np.array(f.cc, np.uint8), hn, ho, vn, vo, f.step)


def _compare(gs, f, where):
    o = _of_oracle(f)
    assert np.array_equal(gs.c, o.c), f"{where}: node colours"
    assert np.array_equal(gs.cc, o.cc), f"{where}: centre colours ({np.argwhere(gs.cc != o.cc)[:5]})"
    assert np.array_equal(gs.hn, o.hn), f"{where}: H counts ({np.argwhere(gs.hn != o.hn)[:5]})"
    assert np.array_equal(gs.vn, o.vn), f"{where}: V counts ({np.argwhere(gs.vn != o.vn)[:5]})"
    for k in range(2):
        mh, mv = o.hn > k, o.vn > k
        assert np.array_equal(gs.ho[..., k][mh], o.ho[..., k][mh]), f"{where}: H offsets {k}"
        assert np.array_equal(gs.vo[..., k][mv], o.vo[..., k][mv]), f"{where}: V offsets {k}"


class FilmLockstep:
    """The GPU film step and the oracle side by side, one sweep at a time on the
    oracle side so that its marker counts per sweep can be summed."""

    def __init__(self, fs, u, v, delta):
        import torch

        from paper_2309_00338_amd.film import EbitFilm

        self.g = EbitFilm(fs, delta)
        self.f = _to_oracle(fs)
        self.u_h, self.v_h, self.delta = u, v, delta
        self.u = torch.from_numpy(np.ascontiguousarray(u)).to("cuda:0")
        self.v = torch.from_numpy(np.ascontiguousarray(v)).to("cuda:0")
        self.stats = T.new_stats()
        self.markers = 0
        self.pairs = 0

    def _count(self, f):
        n = sum(len(e) for row in f.H for e in row) + sum(len(e) for row in f.V for e in row)
        self.pairs = max(self.pairs, sum(len(e) == 2 for row in f.H for e in row) +
                         sum(len(e) == 2 for row in f.V for e in row))
        return n

    def step(self, dt, where):
        self.g.advect(self.u, self.v, dt)
        first = 0 if self.f.step % 2 == 0 else 1
        g = self.f
        for d in (first, 1 - first):
            self.markers += self._count(g)
            g = T.sweep(g, self.u_h, self.v_h, dt, d, self.delta, self.stats)
        g.step = self.f.step + 1
        g.check()
        self.f = g
        self._count(g)
        _compare(self.g.get_state(), g, where)
        C = self.g.fraction().cpu().numpy()
        Co = T.fraction(g)
        assert np.abs(C - Co).max() <= 1e-15, f"{where}: C differs by {np.abs(C - Co).max()}"

    def counters(self):
        got = self.g.stats()
        assert got["parity_fail"] == 0, got
        exp = {"markers": self.markers, "annihilated": self.stats["annihilated"],
               "annihilated_unaligned": self.stats["annihilated_unaligned"],
               "three_crossings": self.stats["three_crossings"]}
        assert {k: got[k] for k in exp} == exp, (got, exp)
        return got


def _oracle_cases():
    out = []
    for n, kind, seed in ((24, "smooth", 0), (20, "dense", 1), (16, "dense", 3), (12, "checker", 4)):
        if kind == "smooth":
            st = I.init_state(n, n, [I.Circle(n * 0.4, n * 0.5, n * 0.2),
                                     I.Ellipse(n * 0.72, n * 0.45, n * 0.14, n * 0.08, 0.7)], h=1.0 / n)
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
        out.append((kind, st, u, v, dt))
    return out


@pytest.mark.parametrize("case", range(4))
def test_without_films_matches_oracle_and_one_marker_path(case):
    """delta = inf: the film step equals its oracle and the one-marker GPU step
    (colours, offsets bit for bit) on smooth, dense random and checkerboard
    states."""
    import torch

    from paper_2309_00338_amd import ebit
    from paper_2309_00338_amd.film import FilmState

    kind, st, u, v, dt = _oracle_cases()[case]
    ls = FilmLockstep(FilmState.of(st), u, v, math.inf)
    one = ebit.EbitGrid(st)
    for k in range(4):
        ls.step(dt, f"{kind} step {k}")
        one.advect(ls.u, ls.v, dt)
        gs, os_ = ls.g.get_state(), one.get_state()
        assert np.array_equal(gs.c, os_.c) and np.array_equal(gs.cc, os_.cc), (kind, k)
        assert (gs.hn <= 1).all() and (gs.vn <= 1).all()
        hp, vp = gs.hn == 1, gs.vn == 1
        assert np.array_equal(gs.ho[..., 0][hp], os_.hoff[hp]) and np.array_equal(gs.vo[..., 0][vp], os_.voff[vp])
    C1 = one.fraction()
    torch.cuda.synchronize()
    assert np.abs(ls.g.fraction().cpu().numpy() - C1.cpu().numpy()).max() < 1e-14
    ls.counters()


def _film(n=16, x1=7.2, x2=8.9):
    from paper_2309_00338_amd.film import FilmState

    c = np.zeros((n + 1, n + 1), np.uint8)
    for i in range(n + 1):
        c[:, i] = 1 if x1 < i < x2 else 0
    cc = np.zeros((n, n), np.uint8)
    for i in range(n):
        cc[:, i] = 1 if x1 < i + 0.5 < x2 else 0
    hn = np.zeros((n + 1, n), np.uint8)
    ho = np.zeros((n + 1, n, 2))
    for x in (x1, x2):
        i = int(math.floor(x))
        ho[:, i, hn[0, i]] = x - i
        hn[:, i] += 1
    return FilmState(n, n, 1.0 / n, c, cc, hn, ho, np.zeros((n, n + 1), np.uint8), np.zeros((n, n + 1, 2)))


def test_squeezed_film_matches_oracle_and_ruptures_at_the_gap():
    """The oracle's squeezed film (u = -k (x - xm), k = 0.25, width 1.7,
    delta = 0.05): every step equal to the oracle; the walls reach one cell
    column as a pair on every crossed edge with C summing to width x height,
    and the film ruptures in step 13."""
    n, k, xm, delta = 16, 0.25, 8.05, 0.05
    u = np.zeros((n, n + 1))
    for i in range(n + 1):
        u[:, i] = -k * (i - xm)
    v = np.zeros((n + 1, n))
    ls = FilmLockstep(_film(n), u, v, delta)
    h = 1.0 / n
    rupture = None
    pairs_seen = False
    for s in range(1, 16):
        before = ls.stats["annihilated"]
        ls.step(h, f"film step {s}")
        w = 1.7 * (1.0 - k) ** s
        gs = ls.g.get_state()
        C = ls.g.fraction().cpu().numpy()
        pairs_seen |= bool((gs.hn == 2).any())
        if w >= delta:
            assert abs(C.sum() - w * n) < 1e-11, (s, C.sum(), w * n)
        else:
            rupture = s
            assert ls.stats["annihilated"] - before == 2 * (n + 1) and C.sum() == 0.0
            break
    assert rupture == 13 and pairs_seen
    ls.counters()


def test_colliding_circles_keep_pairs_where_they_meet():
    """Two circles driven into each other along x (faces left of the middle
    push right, the others left): with a rupture gap of 0.02 cell the edges
    where their fronts meet hold pairs instead of annihilating."""
    n, mid, r, gap = 40, 20, 6.0, 1.3
    st = I.init_state(n, n, [I.Circle(mid + 0.5 - gap / 2 - r, 19.4, r), I.Circle(mid + 0.5 + gap / 2 + r, 20.3, r)])
    u = np.zeros((n, n + 1))
    ii = np.arange(n + 1)
    u[:, :] = np.where(ii <= mid, 0.5, -0.5)[None, :]
    v = np.zeros((n + 1, n))
    from paper_2309_00338_amd.film import FilmState

    ls = FilmLockstep(FilmState.of(st), u, v, 0.02)
    for s in range(8):
        ls.step(0.3 * st.h / 0.5, f"collide step {s}")
    assert ls.pairs > 0
    ls.counters()


@pytest.mark.parametrize("nx,ny,seed,delta", [(32, 32, 34, 0.02), (37, 23, 42, 0.05), (24, 29, 32, 0.0)])
def test_random_colouring_under_sheared_faces(nx, ny, seed, delta):
    """Random colourings under faces whose sign alternates between rows: films
    form and rupture, three-crossing edges occur, on square and ragged grids
    (delta = 0 keeps every even landing)."""
    from paper_2309_00338_amd.film import FilmState

    st = I.random_colouring(nx, ny, seed=seed)
    u, v = I.shear_faces(nx, ny, seed + 500)
    dt = 0.45 * st.h / max(np.abs(u).max(), np.abs(v).max())
    ls = FilmLockstep(FilmState.of(st), u, v, delta)
    for s in range(5):
        ls.step(dt, f"random {nx}x{ny} step {s}")
    got = ls.counters()
    assert ls.pairs > 0 and got["annihilated"] > 0 and got["three_crossings"] > 0, (got, ls.pairs)


def test_cfl_violation_is_reported_like_the_oracle():
    from paper_2309_00338_amd import ebit
    from paper_2309_00338_amd.film import EbitFilm, FilmState

    import torch

    n = 16
    st = I.init_state(n, n, [I.Circle(8.0, 8.0, 4.0)])
    u, v = I.uniform_faces(n, n, 1.0, 0.0)
    dt = 0.6 * st.h  # 0.6 cells per sweep
    with pytest.raises(ValueError, match="CFL"):
        T.step(_to_oracle(FilmState.of(st)), u, v, dt, 0.05)
    g = EbitFilm(FilmState.of(st), 0.05)
    g.advect(torch.from_numpy(u).to("cuda:0"), torch.from_numpy(v).to("cuda:0"), dt)
    assert g.sync() == ebit.EBIT_ERR_CFL
