"""GPU parity: the HIP library against the CPU oracle, step by step, through
the C-ABI (via the thin Python binding), on seeded inputs that span several
tiles, ragged tails, walls, merges and 4-marker cells."""
import math

import numpy as np
import pytest

import oracle
from paper_2309_00338_amd import inputs as I
from tests.parity import Lockstep, compare_fields, compare_state, tie_points

pytestmark = pytest.mark.gpu


def _run(ls, dts, every=1, fields_every=1):
    for k, dt in enumerate(dts):
        ls.step(dt, check_state=(k % every == 0 or k == len(dts) - 1),
                check_fields=(k % fields_every == 0 or k == len(dts) - 1), where=f"step {k}")
    return ls.compare_counters()


def test_config1_vortex_full_trajectory():
    """64x64, R = 0.15 at (0.5, 0.75), vortex T = 2, CFL 0.5: all 256 steps."""
    w = I.single_vortex(64, period=2.0, cfl=0.5)
    ls = Lockstep(w.state, w.u, w.v)
    ls.fields("initial")
    cnt = _run(ls, w.dts)
    assert cnt["markers"] > 0 and cnt["cv_set"] > 0
    print("worst", ls.worst, cnt)


def test_vortex_T8_topology_changes():
    w = I.single_vortex(64, period=8.0, cfl=0.5)
    ls = Lockstep(w.state, w.u, w.v)
    cnt = _run(ls, w.dts, every=4, fields_every=8)
    assert cnt["annihilated"] > 0
    print("worst", ls.worst, cnt)


def test_merging_pairs_small():
    w = I.merging_pairs(n=256, pairs=12, rmin=6.0, rmax=14.0, nsteps=48)
    ls = Lockstep(w.state, w.u, w.v)
    cnt = _run(ls, w.dts)
    assert cnt["annihilated"] > 0
    print("worst", ls.worst, cnt)


def test_cosine_interface_touching_walls():
    w = I.cosine_interface(n=128, nsteps=48)
    ls = Lockstep(w.state, w.u, w.v)
    cnt = _run(ls, w.dts)
    print("worst", ls.worst, cnt)


def test_many_circles_small():
    w = I.many_circles(n=512, count=150, rmin=3.0, rmax=16.0, period=4.0, nsteps=24)
    ls = Lockstep(w.state, w.u, w.v)
    _run(ls, w.dts, every=3, fields_every=3)


@pytest.mark.parametrize("rmin,rmax", [(0.6, 1.6), (1.5, 3.5)])
def test_small_circles_parabola_fallback(rmin, rmax):
    """Circles of one to a few cells: most interfacial cells have no valid
    height (Sec. 2.5), so curvature comes from the parabola fit; kappa, its
    NaN cells and the hf_fail / ghf_fit counts match the oracle every step."""
    w = I.many_circles(n=256, count=200, rmin=rmin, rmax=rmax, period=4.0, nsteps=6, seed=78)
    ls = Lockstep(w.state, w.u, w.v)
    ls.fields("initial")
    cnt = _run(ls, w.dts)
    assert cnt["hf_fail"] > 1000 and cnt["ghf_fit"] > 1000, cnt


@pytest.mark.parametrize("nx,ny", [(64, 64), (53, 37)])
def test_dense_random_colouring(nx, ny):
    """Random node and centre colours with markers on about half of all edges:
    hundreds of listed markers per tile (several rounds per thread in the
    sweep), job-queue flushes, four-marker cells, heavy annihilation and many
    parabola fits, all against the oracle every step."""
    st = I.random_colouring(nx, ny, seed=7)
    x = np.arange(nx + 1) / nx
    y = np.arange(ny + 1) / ny
    psi = (np.sin(np.pi * x)[None, :] ** 2) * (np.sin(np.pi * y)[:, None] ** 2) / np.pi
    psi[0, :] = psi[-1, :] = 0.0
    psi[:, 0] = psi[:, -1] = 0.0
    u, v = I.faces_from_psi(psi, st.h)
    dt = 0.45 * st.h / max(np.abs(u).max(), np.abs(v).max())
    ls = Lockstep(st, u, v)
    ls.fields("initial")
    cnt = _run(ls, [dt] * 6)
    assert cnt["annihilated"] > 100 and cnt["ghf_fit"] > 100, cnt


# (64, 37) and (37, 48): the last node column (row) alone in its block of the
# colour bit plane on one axis, a ragged last tile on the other
@pytest.mark.parametrize("nx,ny", [(37, 53), (53, 19), (16, 16), (4, 4), (17, 33), (64, 37), (37, 48)])
def test_ragged_rectangular_grids(nx, ny):
    rng = np.random.Generator(np.random.PCG64(nx * 1000 + ny))
    shapes = []
    if min(nx, ny) >= 12:
        r = 0.3 * min(nx, ny)
        shapes.append(I.Ellipse(nx / 2 + rng.uniform(-1, 1), ny / 2 + rng.uniform(-1, 1), r, 0.7 * r, 0.4))
    else:
        shapes.append(I.Circle(nx / 2 + 0.13, ny / 2 - 0.21, 1.3))
    st = I.init_state(nx, ny, shapes, h=1.0 / max(nx, ny))
    n = max(nx, ny)
    # vortex-like divergence-free field on the rectangle from a node stream function
    x = np.arange(nx + 1) / nx
    y = np.arange(ny + 1) / ny
    psi = (np.sin(np.pi * x)[None, :] ** 2) * (np.sin(np.pi * y)[:, None] ** 2) / np.pi
    psi[0, :] = psi[-1, :] = 0.0
    psi[:, 0] = psi[:, -1] = 0.0
    u, v = I.faces_from_psi(psi, st.h)
    umax = max(np.abs(u).max(), np.abs(v).max(), 1e-30)
    dt = 0.45 * st.h / umax
    ls = Lockstep(st, u, v)
    ls.fields("initial")
    _run(ls, [dt * math.cos(0.05 * k) for k in range(40)])


def test_ellipses_instance():
    rng = np.random.Generator(np.random.PCG64(44))
    st, u, v, dts = I.random_instance(rng, 96, 6, steps=60)
    ls = Lockstep(st, u, v)
    _run(ls, dts, every=2, fields_every=2)


def test_empty_grid_and_full_grid():
    for fill in (0, 1):
        st = I.init_state(40, 24, [])
        st.c[:] = fill
        st.cc[:] = fill
        w_u, w_v = I.uniform_faces(40, 24, 0.3, -0.2)
        ls = Lockstep(st, w_u, w_v)
        ls.fields("initial")
        _run(ls, [0.01] * 4)


def test_xy_flag_fixed_sweep_order():
    w = I.single_vortex(48, period=2.0, cfl=0.5)
    ls = Lockstep(w.state, w.u, w.v, flags=1)
    _run(ls, w.dts[:60])


def test_fraction_and_curvature_calls_match_fused():
    w = I.single_vortex(64, period=2.0, cfl=0.5)
    ls = Lockstep(w.state, w.u, w.v)
    for dt in w.dts[:40]:
        ls.g.advect(ls.u, ls.v, dt)
    C1, K1 = ls.g.fraction_curvature()
    C2 = ls.g.fraction()
    K2 = ls.g.curvature(C2)
    assert ls.torch.equal(C1, C2)
    assert ls.torch.equal(K1.nan_to_num(7.0), K2.nan_to_num(7.0))
    ls.g.advect(ls.u, ls.v, w.dts[40])
    from paper_2309_00338_amd import ebit

    with pytest.raises(ebit.EbitError) as e:
        ls.g.curvature(C2)
    assert e.value.code == ebit.EBIT_ERR_STATE


def test_checkpoint_resume_is_exact():
    w = I.single_vortex(64, period=2.0, cfl=0.5)
    from paper_2309_00338_amd import ebit

    import torch

    u = torch.from_numpy(w.u).cuda()
    v = torch.from_numpy(w.v).cuda()
    a = ebit.EbitGrid(w.state)
    for dt in w.dts[:30]:
        a.advect(u, v, dt)
    snap = a.get_state()
    for dt in w.dts[30:60]:
        a.advect(u, v, dt)
    end_a = a.get_state()
    b = ebit.EbitGrid(w.state)
    b.set_state(snap)
    for dt in w.dts[30:60]:
        b.advect(u, v, dt)
    end_b = b.get_state()
    assert end_a.step == end_b.step == 60
    assert np.array_equal(end_a.c, end_b.c) and np.array_equal(end_a.cc, end_b.cc)
    hp, vp = end_a.h_present(), end_a.v_present()
    assert np.array_equal(end_a.hoff[hp], end_b.hoff[hp]) and np.array_equal(end_a.voff[vp], end_b.voff[vp])


def test_cfl_and_domain_errors_latch():
    from paper_2309_00338_amd import ebit

    import torch

    w = I.single_vortex(32)
    g = ebit.EbitGrid(w.state)
    u = torch.from_numpy(w.u).cuda()
    v = torch.from_numpy(w.v).cuda()
    g.advect(u, v, 1.2 / 32)  # |d| up to 1.2 cells: latched, kernels finish
    with pytest.raises(ebit.EbitError) as e:
        g.sync()
    assert e.value.code == ebit.EBIT_ERR_CFL
    g.set_state(w.state)
    g.sync()
    st = I.init_state(16, 16, [I.Circle(1.9, 8.2, 1.5)])
    g2 = ebit.EbitGrid(st, flags=1)
    uu, vv = I.uniform_faces(16, 16, -0.45, 0.0)  # 0.45 cells per sweep
    uu = torch.from_numpy(uu).cuda()
    vv = torch.from_numpy(vv).cuda()
    code = 0
    for _ in range(6):
        g2.advect(uu, vv, 1.0 / 16)
        try:
            g2.sync()
        except ebit.EbitError as ex:
            code = ex.code
            break
    assert code == ebit.EBIT_ERR_DOMAIN


def test_straight_line_mode_config1():
    """EBIT-SL (flag EBIT_FIT_LINE) on the config-1 vortex, all 256 steps."""
    from paper_2309_00338_amd import ebit

    w = I.single_vortex(64, period=2.0, cfl=0.5)
    ls = Lockstep(w.state, w.u, w.v, flags=ebit.EBIT_FIT_LINE)
    cnt = _run(ls, w.dts, every=2, fields_every=4)
    assert cnt["fit_reject"] == 0 and cnt["fit_fallback"] == 0
    print("worst", ls.worst, cnt)


@pytest.mark.parametrize("line", [False, True])
def test_zalesak_disk_64(line):
    """Zalesak's disk (Sec. 3.4), one full revolution (1024 steps), both modes."""
    from paper_2309_00338_amd import ebit

    w = I.zalesak(64)
    ls = Lockstep(w.state, w.u, w.v, flags=ebit.EBIT_FIT_LINE if line else 0)
    _run(ls, w.dts, every=32, fields_every=128)


def _ns_compare(got, want, where, kappa=None, sigma=0.0, h=1.0, n=1):
    """rho and mu within 1e-12 relative. The face forces are linear in the
    face curvature, which each side takes from its own kappa (within K_REL of
    each other, relative to max(|kappa|, 1 / (n h)): the field tolerance), so
    they get that error's bound on top: 2 K_REL sigma / h max(|kappa|, 1 / (n h))."""
    from tests.parity import K_REL

    kf = 0.0
    if kappa is not None:
        fin = np.isfinite(kappa)
        kf = 2.0 * K_REL * sigma / h * max(np.abs(kappa[fin]).max(initial=0.0), 1.0 / (n * h))
    for name, g, o in zip(("rho", "mu", "fx", "fy"), got, want):
        g = g.cpu().numpy() if hasattr(g, "cpu") else g
        d = np.abs(g - o)
        tol = 1e-12 * np.maximum(np.abs(o), 1.0) + (kf if name in ("fx", "fy") else 0.0)
        assert (d <= tol).all(), f"{where}: {name} max diff {d.max()} (tolerance there {tol.flat[d.argmax()]})"


def _wide_state(nx, ny):
    """Ellipses spread along a wide, short grid (several per tile row, some
    crossing tile-row boundaries), in cell units of h = 1 / nx."""
    rng = np.random.Generator(np.random.PCG64(nx * 7 + ny))
    shapes = []
    for k in range(max(2, nx // 120)):
        cx = (k + 0.5) * nx / max(2, nx // 120) + rng.uniform(-3, 3)
        cy = rng.uniform(0.3, 0.7) * ny
        a = rng.uniform(3.0, min(10.0, 0.3 * ny))
        shapes.append(I.Ellipse(cx, cy, a, rng.uniform(0.5, 0.9) * a, rng.uniform(0, 1)))
    return I.init_state(nx, ny, shapes, h=1.0 / nx)


@pytest.mark.parametrize("nx,ny", [(1030, 40), (2050, 20), (1023, 19)])
def test_wide_rows_fraction_and_curvature(nx, ny):
    """Rows at least as long as a wavefront run of the uniform fill, not a
    multiple of 16 cells: the linear fill's runs inside a row, across a row's
    end and across a tile row (and, at 1023, the element-wise walk)."""
    st = _wide_state(nx, ny)
    u, v = I.uniform_faces(nx, ny, 0.3, -0.2)
    ls = Lockstep(st, u, v)
    ls.fields("initial")
    _run(ls, [0.4 / nx] * 4)


def _narrow_state(nx, ny=160):
    """A grid narrower than 8 cells holding a band of colour 1 across its whole
    width (an ellipse cut by both side walls): uniform tiles of colour 0 below
    and above, of colour 1 inside, near tiles only at the band's two ends."""
    return I.init_state(nx, ny, [I.Ellipse(nx / 2 + 0.07, 80.3, 9.0, 40.0, 0.0)], h=1.0 / ny)


@pytest.mark.parametrize("nx", [4, 5, 6, 7])
def test_narrow_grids_uniform_fill(nx):
    """Rows narrower than 8 cells: one 16-element virtual row of the uniform
    fill spans several grid rows (a lane's step wraps more than one row). The
    outputs start as NaN so that a cell the fill skips shows too."""
    import torch

    st = _narrow_state(nx)
    u, v = I.uniform_faces(nx, st.ny, 0.0, 0.3)
    ls = Lockstep(st, u, v)
    for k in range(4):
        ls.step(0.4 / st.ny, check_state=True, check_fields=False, where=f"step {k}")
        C = torch.full((st.ny, nx), float("nan"), dtype=torch.float64, device="cuda:0")
        K = torch.full((st.ny, nx), float("nan"), dtype=torch.float64, device="cuda:0")
        ls.g.fraction_curvature(C, K)
        Co = oracle.fraction(ls.o)
        Ko, _ = oracle.curvature(ls.o, Co)
        assert (Co[:32] == 0).all() and (Co[48:112] == 1).all() and (Co[128:] == 0).all()
        compare_fields(C.cpu().numpy(), K.cpu().numpy(), Co, Ko, nx, st.h, f"{nx}x{st.ny} step {k}")


@pytest.mark.parametrize("case", ["vortex64", "circles512", "ragged37x53", "narrow5x40", "wide300x6",
                                  "wide1030x40", "wide1024x24", "wide2050x20", "band4x160", "band7x160"])
def test_ns_fields_match_oracle(case):
    """rho, mu and the surface-tension face forces from the GPU C and kappa,
    against the oracle from the oracle's C and kappa, after a few steps."""
    from paper_2309_00338_amd import ebit

    if case == "vortex64":
        w = I.single_vortex(64, period=2.0, cfl=0.5)
        st, u, v, dts = w.state, w.u, w.v, w.dts[:20]
    elif case == "circles512":
        w = I.many_circles(n=512, count=150, rmin=3.0, rmax=16.0, period=4.0, nsteps=6)
        st, u, v, dts = w.state, w.u, w.v, w.dts
    elif case == "ragged37x53":
        st = I.init_state(37, 53, [I.Ellipse(18.3, 26.1, 11.0, 7.0, 0.4)], h=1.0 / 53)
        u, v = I.uniform_faces(37, 53, 0.3, -0.2)
        dts = [0.5 / 53] * 6
    elif case.startswith("band"):
        # uniform tiles of both colours in rows narrower than 8 cells
        st = _narrow_state(int(case[4:].split("x")[0]))
        u, v = I.uniform_faces(st.nx, st.ny, 0.0, 0.3)
        dts = [0.4 / st.ny] * 4
    elif case.startswith("wide") and int(case[4:].split("x")[0]) >= 1024:
        # rows of at least one wavefront run of the uniform pass: runs inside
        # a row and runs across a row end (and a tile row), face rows nx + 1
        nx, ny = (int(t) for t in case[4:].split("x"))
        st = _wide_state(nx, ny)
        u, v = I.uniform_faces(nx, ny, 0.3, -0.2)
        dts = [0.4 / max(nx, ny)] * 4
    else:
        # rows shorter than a wavefront's stride of the uniform pass, or one
        # tile row only: the linear passes wrap rows many times or never
        nx, ny, sh = ((5, 40, I.Ellipse(2.6, 20.3, 1.7, 7.0, 0.1)) if case == "narrow5x40"
                      else (300, 6, I.Ellipse(150.2, 3.1, 60.0, 1.8, 0.0)))
        st = I.init_state(nx, ny, [sh], h=1.0 / max(nx, ny))
        u, v = I.uniform_faces(nx, ny, 0.3, -0.2)
        dts = [0.4 / max(nx, ny)] * 4
    ls = Lockstep(st, u, v)
    for k, dt in enumerate(dts):
        ls.step(dt, check_state=False, check_fields=False, where=f"step {k}")
    C, K = ls.g.fraction_curvature()
    fl = (1000.0, 1.2, 1e-3, 1.8e-5, 0.07)
    got = ls.g.ns_fields(C, K, *fl)
    Co = oracle.fraction(ls.o)
    Ko, _ = oracle.curvature(ls.o, Co)
    want = oracle.ns_fields(ls.o, Co, Ko, *fl)
    _ns_compare(got, want, case, kappa=Ko, sigma=fl[4], h=st.h, n=max(st.nx, st.ny))


def test_ns_fields_require_current_fraction():
    from paper_2309_00338_amd import ebit

    w = I.single_vortex(64, period=2.0, cfl=0.5)
    ls = Lockstep(w.state, w.u, w.v)
    C, K = ls.g.fraction_curvature()
    ls.g.advect(ls.u, ls.v, w.dts[0])
    with pytest.raises(ebit.EbitError) as e:
        ls.g.ns_fields(C, K, 1, 1, 1, 1, 1)
    assert e.value.code == ebit.EBIT_ERR_STATE


def test_checkerboard_both_sweeps_queue_more_jobs_than_one_grid_edge_count():
    """Alternating node colours: every edge carries a marker and every cell
    four. The first sweep's fit jobs stay listed until the second sweep's
    launch has applied their centre rules, so both sweeps' jobs are alive at
    once; here they outnumber (nx+1)(ny+1), the list length that once held
    them. States, fields and counters match the oracle every step."""
    n = 64
    st = I.checkerboard(n, n, seed=11)
    x = np.arange(n + 1) / n
    psi = (np.sin(np.pi * x)[None, :] ** 2) * (np.sin(np.pi * x)[:, None] ** 2) / np.pi
    psi[0, :] = psi[-1, :] = psi[:, 0] = psi[:, -1] = 0.0
    u, v = I.faces_from_psi(psi, st.h)
    dt = 0.2 * st.h / max(np.abs(u).max(), np.abs(v).max())
    o = st.copy()
    assert oracle.sweep(o, u, v, dt, 0)[0] == oracle.OK
    jobs_x = int(o.v_present()[:, 1:-1].sum())
    assert oracle.sweep(o, u, v, dt, 1)[0] == oracle.OK
    jobs_y = int(o.h_present()[1:-1, :].sum())
    assert jobs_x + jobs_y > (n + 1) * (n + 1), (jobs_x, jobs_y)
    ls = Lockstep(st, u, v)
    ls.fields("initial")
    cnt = _run(ls, [dt] * 4)
    assert cnt["cv_set"] > 1000, cnt


@pytest.mark.parametrize("nx,ny,seed", [(64, 64, 33), (53, 37, 38), (160, 96, 35)])
def test_rare_branches_under_sheared_random_faces(nx, ny, seed):
    """Random colouring under a field whose sign alternates between rows
    (columns for v): markers of neighbouring rows converge and pass each other,
    which reaches the branches smooth flows never do: three aligned markers
    landing on one edge (the middle kept), a new unaligned edge crossed by three
    advected segments (the median taken) and four-marker cells that no
    centre rule settles. Each count is nonzero and equal to the oracle's, and
    the states and fields match every step."""
    st = I.random_colouring(nx, ny, seed=seed)
    u, v = I.shear_faces(nx, ny, seed + 500)
    dt = 0.49 * st.h / max(np.abs(u).max(), np.abs(v).max())
    ls = Lockstep(st, u, v)
    ls.fields("initial")
    cnt = _run(ls, [dt] * 6)
    assert cnt["three_landers"] > 0 and cnt["three_crossings"] > 0 and cnt["cv_unresolved"] > 0, cnt
    print(cnt)


def test_wall_markers_hold_under_wall_normal_motion():
    """A nearly flat interface touching both side walls, translated by a
    uniform field whose wall faces are not zero: the wall-line markers keep
    their offsets in the x sweep (counted as wall violations) and slide along
    the walls in the y sweep; no marker leaves the grid."""
    n = 96
    st = I.init_state(n, n, [I.CosineBelow(n, 0.5, 0.004)])
    u, v = I.uniform_faces(n, n, 0.6, 0.4)
    dt = 0.5 * st.h  # 0.3 and 0.2 cells per sweep
    ls = Lockstep(st, u, v)
    ls.fields("initial")
    cnt = _run(ls, [dt] * 8)
    assert cnt["wall_violation"] >= 16, cnt


def test_mismatch_at_a_tie_resyncs_and_elsewhere_fails():
    """The harness's tie rule, exercised by editing the oracle's state after its
    step (on the CPU): an offset difference on an edge where the oracle logged a
    tie is recorded and the GPU is re-set from the oracle, after which both
    sides agree again; the same difference far from every tie fails."""
    w = I.merging_pairs(n=256, pairs=12, rmin=6.0, rmax=14.0, nsteps=40)
    ls = Lockstep(w.state, w.u, w.v)
    planted = []

    def at_tie(o, ties):
        if planted or not ties:
            return
        kind, i, j = ties[0]["edge"]
        if kind == "H" and o.h_present()[j, i]:
            o.hoff[j, i] = min(1.0, o.hoff[j, i] + 1e-9)
            planted.append((kind, i, j))
        elif kind == "V" and o.v_present()[j, i]:
            o.voff[j, i] = min(1.0, o.voff[j, i] + 1e-9)
            planted.append((kind, i, j))

    for k in range(40):
        ls.step(w.dts[k], check_fields=(k % 4 == 3), where=f"step {k}", plant=at_tie)
        if planted and k > 8:
            break
    assert planted and len(ls.resyncs) == 1, (planted, ls.resyncs)
    ls.compare_counters()

    ls2 = Lockstep(w.state, w.u, w.v)

    def far(o, ties):
        tp = tie_points(ties)
        jj, ii = np.nonzero(o.h_present())
        for j, i in zip(jj, ii):
            if all(max(abs(i + 0.5 - a), abs(j - b)) > 10 for a, b in tp):
                o.hoff[j, i] = min(1.0, o.hoff[j, i] + 1e-9) if o.hoff[j, i] < 0.5 else o.hoff[j, i] - 1e-9
                return

    with pytest.raises(AssertionError):
        ls2.step(w.dts[0], plant=far)
