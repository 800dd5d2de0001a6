"""GPU parity of the batched and served forms: every grid of a batch or a pool
against its own oracle run, step by step, through the C-ABI."""
import numpy as np
import pytest

import oracle
from paper_2309_00338_amd import ebit
from paper_2309_00338_amd import inputs as I
from tests.parity import compare_fields, compare_state

pytestmark = pytest.mark.gpu


def _instances():
    """Grids of several sizes, ragged tails and one fixed sweep order."""
    rng = np.random.Generator(np.random.PCG64(4242))
    out = []
    for n, k in ((20, 1), (33, 3), (48, 4), (64, 2), (71, 5), (96, 6)):
        st, u, v, dts = I.random_instance(rng, n, k, ellipses=True, steps=16)
        out.append((st, u, v, dts))
    # a rectangular grid with a ragged tail in both directions
    st = I.init_state(37, 53, [I.Ellipse(18.3, 26.1, 11.0, 7.0, 0.4)], h=1.0 / 53)
    x = np.arange(38) / 37
    y = np.arange(54) / 53
    psi = (np.sin(np.pi * x)[None, :] ** 2) * (np.sin(np.pi * y)[:, None] ** 2) / np.pi
    psi[0, :] = psi[-1, :] = 0.0
    psi[:, 0] = psi[:, -1] = 0.0
    u, v = I.faces_from_psi(psi, st.h)
    umax = max(np.abs(u).max(), np.abs(v).max())
    out.append((st, u, v, [0.45 * st.h / umax * (1 - 0.02 * k) for k in range(16)]))
    return out


def test_batch_matches_oracle_per_grid():
    import torch

    inst = _instances()
    b = ebit.EbitBatch([s for s, _, _, _ in inst])
    U, V = b.pack_velocities([u for _, u, _, _ in inst], [v for _, _, v, _ in inst])
    nsteps = len(inst[0][3])
    dts = torch.tensor([[d[k] for _, _, _, d in inst] for k in range(nsteps)], dtype=torch.float64, device="cuda:0")
    C, K = b.new_fields()
    orc = [s.copy() for s, _, _, _ in inst]
    ocnt = oracle.new_counters()
    for k in range(nsteps):
        b.advect(U, V, dts[k])
        for g, (st, u, v, d) in enumerate(inst):
            rc, _ = oracle.step(orc[g], u, v, d[k], counters=ocnt)
            assert rc == oracle.OK
        if k % 3 == 2 or k == nsteps - 1:
            b.fraction_curvature(C, K)
            torch.cuda.synchronize()
            for g in range(len(inst)):
                gs = b.get_state(g)
                compare_state(gs, orc[g], f"grid {g} step {k}")
                Co = oracle.fraction(orc[g])
                Ko, _ = oracle.curvature(orc[g], Co, counters=ocnt)
                compare_fields(b.field(C, g).cpu().numpy(), b.field(K, g).cpu().numpy(), Co, Ko, orc[g].nx,
                               orc[g].h, f"grid {g} step {k}")
    assert b.sync() == [0] * len(inst)
    gc = {k: v for k, v in b.stats().items() if k not in ebit.SCHEDULE_COUNTERS}
    assert gc == oracle.counters_dict(ocnt)


def test_batch_equals_single_handles():
    """The batch gives bit-identical states to one handle per grid."""
    import torch

    inst = _instances()[:4]
    b = ebit.EbitBatch([s for s, _, _, _ in inst])
    U, V = b.pack_velocities([u for _, u, _, _ in inst], [v for _, _, v, _ in inst])
    singles = [ebit.EbitGrid(s) for s, _, _, _ in inst]
    us = [(torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda()) for _, u, v, _ in inst]
    for k in range(10):
        dts = torch.tensor([d[k] for _, _, _, d in inst], dtype=torch.float64, device="cuda:0")
        b.advect(U, V, dts)
        for g, h in enumerate(singles):
            h.advect(us[g][0], us[g][1], inst[g][3][k])
    for g, h in enumerate(singles):
        a, s = b.get_state(g), h.get_state()
        assert np.array_equal(a.c, s.c) and np.array_equal(a.cc, s.cc)
        assert np.array_equal(a.hoff * a.h_present(), s.hoff * s.h_present())
        assert np.array_equal(a.voff * a.v_present(), s.voff * s.v_present())


def test_batch_error_is_per_grid():
    """A CFL violation in one grid latches only that grid's status."""
    import torch

    inst = _instances()[:3]
    b = ebit.EbitBatch([s for s, _, _, _ in inst])
    U, V = b.pack_velocities([u for _, u, _, _ in inst], [v for _, _, v, _ in inst])
    dts = torch.tensor([inst[0][3][0], 3.0 / inst[1][0].nx, inst[2][3][0]], dtype=torch.float64, device="cuda:0")
    b.advect(U, V, dts)
    st = b.sync()
    assert st[0] == 0 and st[2] == 0 and st[1] == ebit.EBIT_ERR_CFL


class _Ref:
    """One grid of the pool and its oracle twin."""

    def __init__(self, st, u, v, dt):
        self.o = st.copy()
        self.o.step = 0
        self.u, self.v, self.dt = u, v, dt

    def step(self, ocnt):
        rc, _ = oracle.step(self.o, self.u, self.v, self.dt, counters=ocnt)
        assert rc == oracle.OK


def _pool_instance(n, k, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    st, u, v, dts = I.random_instance(rng, n, k, ellipses=True, steps=1, period=1e9)
    return st, u, v, dts[0]


def test_pool_admit_step_retire_matches_oracle():
    pool = ebit.EbitPool(max_grids=3, max_tiles=64, arena_bytes=64 << 20)
    ocnt = oracle.new_counters()
    live = {}

    def admit(n, k, seed):
        st, u, v, dt = _pool_instance(n, k, seed)
        slot = pool.admit(st, u, v, dt)
        if slot is not None:
            live[slot] = _Ref(st, u, v, dt)
        return slot

    def step_and_check(tag):
        pool.step()
        for s, r in live.items():
            r.step(ocnt)
        for s, r in live.items():
            C, K, steps, status = pool.read(s)
            assert status == 0 and steps == r.o.step
            compare_state(pool.get_state(s), r.o, f"{tag} slot {s}")
            Co = oracle.fraction(r.o)
            Ko, _ = oracle.curvature(r.o, Co, counters=ocnt)
            compare_fields(C, K, Co, Ko, r.o.nx, r.o.h, f"{tag} slot {s}")

    a = admit(48, 3, 11)
    for k in range(3):
        step_and_check(f"A{k}")
    b = admit(40, 2, 12)  # its step 0 runs at an odd pool step: both sweep orders in one phase
    for k in range(2):
        step_and_check(f"AB{k}")
    c = admit(33, 2, 13)
    assert admit(20, 1, 14) is None  # no free slot
    step_and_check("ABC")
    pool.retire(a)
    live.pop(a)
    d = admit(44, 4, 15)  # reuses the freed slot, tiles and arena space
    assert d == a
    for k in range(4):
        step_and_check(f"BCD{k}")
    pool.retire(b)
    live.pop(b)
    step_and_check("CD")
    assert c is not None


def test_batch_with_mixed_flags():
    """Grids with the circle fit, the straight line and the fixed x-then-y order
    in one batch, each against its own oracle run."""
    import torch

    inst = _instances()[:3]
    flags = [0, ebit.EBIT_FIT_LINE, ebit.EBIT_SWEEP_XY | ebit.EBIT_FIT_LINE]
    b = ebit.EbitBatch([s for s, _, _, _ in inst], flags=flags)
    U, V = b.pack_velocities([u for _, u, _, _ in inst], [v for _, _, v, _ in inst])
    orc = [s.copy() for s, _, _, _ in inst]
    for k in range(12):
        dts = torch.tensor([d[k] for _, _, _, d in inst], dtype=torch.float64, device="cuda:0")
        b.advect(U, V, dts)
        for g, (st, u, v, d) in enumerate(inst):
            rc, _ = oracle.step(orc[g], u, v, d[k], xy_only=bool(flags[g] & 1), line=bool(flags[g] & 2))
            assert rc == oracle.OK
        for g in range(3):
            compare_state(b.get_state(g), orc[g], f"grid {g} step {k}")


def test_batch_ns_fields_per_grid():
    import torch

    inst = _instances()
    b = ebit.EbitBatch([s for s, _, _, _ in inst])
    U, V = b.pack_velocities([u for _, u, _, _ in inst], [v for _, _, v, _ in inst])
    orc = [s.copy() for s, _, _, _ in inst]
    for k in range(5):
        dts = torch.tensor([d[k] for _, _, _, d in inst], dtype=torch.float64, device="cuda:0")
        b.advect(U, V, dts)
        for g, (st, u, v, d) in enumerate(inst):
            assert oracle.step(orc[g], u, v, d[k])[0] == oracle.OK
    C, K = b.new_fields()
    b.fraction_curvature(C, K)
    fl = (800.0, 2.0, 0.5, 0.01, 0.3)
    rho, mu, fx, fy = b.ns_fields(C, K, *fl)
    for g in range(len(inst)):
        nx, ny, _ = b.shapes[g]
        Co = oracle.fraction(orc[g])
        Ko, _ = oracle.curvature(orc[g], Co)
        want = oracle.ns_fields(orc[g], Co, Ko, *fl)
        got = (b.field(rho, g), b.field(mu, g),
               fx[b.u_off[g]:b.u_off[g] + ny * (nx + 1)].view(ny, nx + 1),
               fy[b.v_off[g]:b.v_off[g] + (ny + 1) * nx].view(ny + 1, nx))
        for name, gg, o in zip(("rho", "mu", "fx", "fy"), got, want):
            d = np.abs(gg.cpu().numpy() - o) / np.maximum(np.abs(o), 1.0)
            assert d.max(initial=0) <= 1e-12, (g, name, d.max())


def test_one_grid_batch_and_pool_match_oracle():
    """A batch of one grid and a pool of one slot run the single-grid kernels
    (the step's first centre pass inside the second sweep's launch), with a
    device dt and with the pool's own velocities; the pool also steps empty
    between a retire and the next admission."""
    import torch

    st, u, v, dts = _instances()[2]
    b = ebit.EbitBatch([st])
    U, V = b.pack_velocities([u], [v])
    o = st.copy()
    C, K = b.new_fields()
    for k in range(8):
        b.advect(U, V, torch.tensor([dts[k]], dtype=torch.float64, device="cuda:0"))
        assert oracle.step(o, u, v, dts[k])[0] == oracle.OK
        compare_state(b.get_state(0), o, f"batch step {k}")
    b.fraction_curvature(C, K)
    Co = oracle.fraction(o)
    Ko, _ = oracle.curvature(o, Co)
    compare_fields(b.field(C, 0).cpu().numpy(), b.field(K, 0).cpu().numpy(), Co, Ko, o.nx, o.h, "batch")
    assert b.sync() == [0]

    pool = ebit.EbitPool(max_grids=1, max_tiles=64, arena_bytes=64 << 20)
    for seed in (21, 22):
        pst, pu, pv, pdt = _pool_instance(44, 3, seed)
        slot = pool.admit(pst, pu, pv, pdt)
        assert slot == 0
        ref = _Ref(pst, pu, pv, pdt)
        for k in range(5):
            pool.step()
            ref.step(None)
        Cp, Kp, steps, status = pool.read(slot)
        assert status == 0 and steps == ref.o.step
        compare_state(pool.get_state(slot), ref.o, f"pool seed {seed}")
        Co = oracle.fraction(ref.o)
        Ko, _ = oracle.curvature(ref.o, Co)
        compare_fields(Cp, Kp, Co, Ko, ref.o.nx, ref.o.h, f"pool seed {seed}")
        pool.retire(slot)
        pool.step()  # nothing live: no sweep, nothing pending


@pytest.mark.parametrize("which", ["many", "one"])
def test_graph_replay_matches_eager_steps_and_oracle(which):
    """ebit_batch_capture records 4 steps (advect + fraction/curvature) as one
    graph; three replays, with the program's own eager work and
    synchronisations between them, give bit for bit the states, C and kappa of
    12 eager steps of an identical batch, and the oracle's after the last.
    "one": a batch of a single grid (the one-grid kernels, whose first centre
    pass rides with the second sweep)."""
    import torch

    inst = _instances()
    if which == "one":
        inst = inst[3:4]
    K = 4
    states = [s for s, _, _, _ in inst]
    eager, graphed = ebit.EbitBatch(states), ebit.EbitBatch(states, stream=torch.cuda.Stream())
    U, V = eager.pack_velocities([u for _, u, _, _ in inst], [v for _, _, v, _ in inst])
    dts = torch.tensor([[d[k] for _, _, _, d in inst] for k in range(K)], dtype=torch.float64, device="cuda:0")
    Ce, Ke = eager.new_fields()
    Cg, Kg = graphed.new_fields()
    graph = graphed.capture(K, U, V, dts, Cg, Kg)
    orc = [s.copy() for s in states]
    for rep in range(3):
        for k in range(K):
            eager.advect(U, V, dts[k])
            eager.fraction_curvature(Ce, Ke)
            for g, (st, u, v, d) in enumerate(inst):
                assert oracle.step(orc[g], u, v, d[k])[0] == oracle.OK
        graph.launch()
        # eager work of the program between replays
        x = torch.randn(256, 256, device="cuda:0", dtype=torch.float64)
        (x @ x).sum().item()
        torch.cuda.synchronize()
        for g in range(len(inst)):
            a, b = eager.get_state(g), graphed.get_state(g)
            assert a.step == b.step == (rep + 1) * K
            assert np.array_equal(a.c, b.c) and np.array_equal(a.cc, b.cc), (rep, g)
            assert np.array_equal(a.hoff * a.h_present(), b.hoff * b.h_present()), (rep, g)
            assert np.array_equal(a.voff * a.v_present(), b.voff * b.v_present()), (rep, g)
            fe, fg = eager.field(Ce, g).cpu().numpy(), graphed.field(Cg, g).cpu().numpy()
            assert np.array_equal(fe, fg), (rep, g)
            ke, kg = eager.field(Ke, g).cpu().numpy(), graphed.field(Kg, g).cpu().numpy()
            assert np.array_equal(np.isnan(ke), np.isnan(kg)) and np.array_equal(ke[~np.isnan(ke)], kg[~np.isnan(kg)])
    assert graphed.sync() == [0] * len(inst)
    for g in range(len(inst)):
        compare_state(graphed.get_state(g), orc[g], f"grid {g} after {3 * K} steps")
        Co = oracle.fraction(orc[g])
        Ko, _ = oracle.curvature(orc[g], Co)
        compare_fields(graphed.field(Cg, g).cpu().numpy(), graphed.field(Kg, g).cpu().numpy(), Co, Ko, orc[g].nx,
                       orc[g].h, f"grid {g}")
    # an odd number of eager steps breaks the captured schedule: refused, nothing runs
    graphed.advect(U, V, dts[0])
    with pytest.raises(ebit.EbitError) as e:
        graph.launch()
    assert e.value.code == ebit.EBIT_ERR_STATE
    graph.close()
    graphed.close()


def test_pool_isolates_failing_requests():
    """Four requests share a pool: one whose dt moves its markers more than half
    a cell per sweep (a CFL error) and one admitted with an invalid state (an
    offset outside [0, 1] on a marker edge, found by the device-side
    validation of the asynchronous admission). The bulk status call reports
    CFL and ARG for exactly those slots; they are evicted, and the other two
    requests, stepped on in the same pool, stay equal to their oracle runs
    every step."""
    import torch

    pool = ebit.EbitPool(max_grids=4, max_tiles=128, arena_bytes=128 << 20)
    good = {}
    st, u, v, dt = _pool_instance(48, 3, 21)
    good[pool.admit(st, u, v, dt)] = _Ref(st, u, v, dt)
    st, u, v, dt = _pool_instance(40, 2, 22)
    cfl = pool.admit(st, u, v, 4.0 * dt)
    st, u, v, dt = _pool_instance(36, 2, 23)
    good[pool.admit(st, u, v, dt)] = _Ref(st, u, v, dt)
    st, u, v, dt = _pool_instance(30, 2, 24)
    jj, ii = np.nonzero(st.h_present())
    bad = st.copy()
    bad.hoff[jj[0], ii[0]] = 1.5
    arg = pool.admit(bad, u, v, dt)
    pool.step()
    status = pool.status().cpu().numpy()
    assert status[cfl] == ebit.EBIT_ERR_CFL and status[arg] == ebit.EBIT_ERR_ARG, status
    assert all(status[s] == 0 for s in good), status
    pool.retire(cfl)
    pool.retire(arg)
    ocnt = oracle.new_counters()
    for r in good.values():
        r.step(ocnt)
    for k in range(5):
        if k:
            pool.step()
            for r in good.values():
                r.step(ocnt)
        for s, r in good.items():
            C, K, steps, status = pool.read(s)
            assert status == 0 and steps == r.o.step
            compare_state(pool.get_state(s), r.o, f"step {k} slot {s}")
            Co = oracle.fraction(r.o)
            Ko, _ = oracle.curvature(r.o, Co)
            compare_fields(C, K, Co, Ko, r.o.nx, r.o.h, f"step {k} slot {s}")
    torch.cuda.synchronize()


def _psi_faces(st):
    x = np.arange(st.nx + 1) / st.nx
    y = np.arange(st.ny + 1) / st.ny
    psi = (np.sin(np.pi * x)[None, :] ** 2) * (np.sin(np.pi * y)[:, None] ** 2) / np.pi
    psi[0, :] = psi[-1, :] = 0.0
    psi[:, 0] = psi[:, -1] = 0.0
    return I.faces_from_psi(psi, st.h)


def test_batch_of_checkerboards_fills_the_job_queues():
    """Alternating node colours in every grid of a batch: every interior edge
    queues a fit job each sweep, the most a tile can queue. With several grids
    the sweep's workgroups queue on 8 queues whose regions are bounded from the
    sweep's chunking; none may overflow (an overflow latches EBIT_ERR_NOMEM),
    and every grid matches its oracle run step by step."""
    import torch

    inst = []
    for k, (nx, ny) in enumerate(((64, 64), (48, 40), (33, 20), (80, 16))):
        st = I.checkerboard(nx, ny, seed=21 + k)
        u, v = _psi_faces(st)
        dt = 0.2 * st.h / max(np.abs(u).max(), np.abs(v).max())
        inst.append((st, u, v, [dt] * 4))
    b = ebit.EbitBatch([s for s, _, _, _ in inst])
    U, V = b.pack_velocities([u for _, u, _, _ in inst], [v for _, _, v, _ in inst])
    dts = torch.tensor([[d[k] for _, _, _, d in inst] for k in range(4)], dtype=torch.float64, device="cuda:0")
    C, K = b.new_fields()
    orc = [s.copy() for s, _, _, _ in inst]
    ocnt = oracle.new_counters()
    for k in range(4):
        b.advect(U, V, dts[k])
        for g, (st, u, v, d) in enumerate(inst):
            assert oracle.step(orc[g], u, v, d[k], counters=ocnt)[0] == oracle.OK
        b.fraction_curvature(C, K)
        torch.cuda.synchronize()
        for g in range(len(inst)):
            compare_state(b.get_state(g), orc[g], f"grid {g} step {k}")
            Co = oracle.fraction(orc[g])
            Ko, _ = oracle.curvature(orc[g], Co, counters=ocnt)
            compare_fields(b.field(C, g).cpu().numpy(), b.field(K, g).cpu().numpy(), Co, Ko, orc[g].nx, orc[g].h,
                           f"grid {g} step {k}")
    assert b.sync() == [0] * len(inst)
    gc = {k: v for k, v in b.stats().items() if k not in ebit.SCHEDULE_COUNTERS}
    assert gc == oracle.counters_dict(ocnt)
    assert gc["cv_set"] > 1000, gc


def test_batch_with_narrow_grids():
    """Grids narrower than 8 cells packed between ordinary ones: the uniform
    fill's virtual rows of 16 elements span several rows of a narrow grid. The
    outputs start as NaN so that a cell the fill skips shows too."""
    import torch

    grids = []
    for nx in (5, 4, 7, 6):
        grids.append(I.init_state(nx, 160, [I.Ellipse(nx / 2 + 0.07, 80.3, 9.0, 40.0, 0.0)], h=1.0 / 160))
    grids.insert(2, I.init_state(37, 53, [I.Ellipse(18.3, 26.1, 11.0, 7.0, 0.4)], h=1.0 / 53))
    faces = [I.uniform_faces(s.nx, s.ny, 0.0, 0.3) for s in grids]
    b = ebit.EbitBatch(grids)
    U, V = b.pack_velocities([u for u, _ in faces], [v for _, v in faces])
    dt = [0.4 / s.ny for s in grids]
    dts = torch.tensor(dt, dtype=torch.float64, device="cuda:0")
    orc = [s.copy() for s in grids]
    for k in range(4):
        b.advect(U, V, dts)
        for g, s in enumerate(orc):
            rc, _ = oracle.step(s, faces[g][0], faces[g][1], dt[g])
            assert rc == oracle.OK
        C, K = b.new_fields()
        C.fill_(float("nan"))
        K.fill_(float("nan"))
        b.fraction_curvature(C, K)
        torch.cuda.synchronize()
        for g, s in enumerate(orc):
            compare_state(b.get_state(g), s, f"grid {g} step {k}")
            Co = oracle.fraction(s)
            Ko, _ = oracle.curvature(s, Co)
            compare_fields(b.field(C, g).cpu().numpy(), b.field(K, g).cpu().numpy(), Co, Ko, s.nx, s.h,
                           f"grid {g} step {k}")
    assert b.sync() == [0] * len(grids)
    # the consumers' uniform part on the same grids (from the last C and kappa)
    from tests.test_gpu_parity import _ns_compare

    fl = (1000.0, 1.2, 1e-3, 1.8e-5, 0.07)
    rho, mu, fx, fy = b.ns_fields(C, K, *fl)
    for g, s in enumerate(orc):
        nx, ny = s.nx, s.ny
        Co = oracle.fraction(s)
        Ko, _ = oracle.curvature(s, Co)
        got = (b.field(rho, g), b.field(mu, g),
               fx[b.u_off[g]:b.u_off[g] + ny * (nx + 1)].view(ny, nx + 1),
               fy[b.v_off[g]:b.v_off[g] + (ny + 1) * nx].view(ny + 1, nx))
        _ns_compare(got, oracle.ns_fields(s, Co, Ko, *fl), f"grid {g}", kappa=Ko, sigma=fl[4], h=s.h, n=max(nx, ny))
