"""Schedule invariance: the launch schedule of an engine (workgroups per CU of
the sweeps, fits and fraction pass, the near/fill split, the batch's minimum
sweep chunk) decides only which workgroup handles which tile or job. States,
C, kappa and the interface consumers' fields are bit-identical under every
value the tuner can choose and under extreme settings, for one grid and for a
batch; the tuner itself leaves a valid schedule and caches it."""
import numpy as np
import pytest

from paper_2309_00338_amd import ebit
from paper_2309_00338_amd import inputs as I
from paper_2309_00338_amd import tune

pytestmark = pytest.mark.gpu

EXTREMES = [
    {"sweep_per_cu": 1, "fit_per_cu": 1, "frac_near_per_cu": 0.5, "ns_near_per_cu": 0.5, "sweep_min_chunk": 1},
    {"sweep_per_cu": 5, "fit_per_cu": 3, "frac_near_per_cu": 2.5, "ns_near_per_cu": 7.0, "sweep_min_chunk": 3},
    {"sweep_per_cu": 64, "fit_per_cu": 64, "frac_near_per_cu": 64.0, "ns_near_per_cu": 64.0, "sweep_min_chunk": 4096},
]


def _settings():
    out = [dict(s) for s in EXTREMES]
    for f, vals in tune.CANDIDATES.items():
        out += [{f: v} for v in vals]
    return out


def _one_grid_run(sched, w, steps=5):
    import torch

    g = ebit.EbitGrid(w.state)
    if sched is not None:
        g.set_schedule(sched)
    u, v = torch.from_numpy(w.u).cuda(), torch.from_numpy(w.v).cuda()
    for k in range(steps):
        g.advect(u, v, w.dts[k])
    C, K = g.fraction_curvature()
    rho, mu, fx, fy = g.ns_fields(C, K, 1000.0, 1.2, 1e-3, 1.8e-5, 0.07)
    torch.cuda.synchronize()
    st = g.get_state()
    used = g.get_schedule()
    arrs = [st.c, st.cc, st.hoff * st.h_present(), st.voff * st.v_present()] + [t.cpu().numpy() for t in
                                                                                  (C, K, rho, mu, fx, fy)]
    g.close()
    return arrs, used


def _equal(a, b):
    for x, y in zip(a, b):
        assert x.shape == y.shape
        assert np.array_equal(np.isnan(x), np.isnan(y)) if x.dtype.kind == "f" else True
        if x.dtype.kind == "f":
            assert np.array_equal(x[~np.isnan(x)], y[~np.isnan(y)])
        else:
            assert np.array_equal(x, y)


def test_one_grid_results_do_not_depend_on_the_schedule():
    w = I.many_circles(n=512, count=150, rmin=2.0, rmax=16.0, period=4.0, nsteps=6, seed=91)
    ref, used = _one_grid_run(None, w)
    assert all(used[k] > 0 for k in ebit.SCHEDULE_FIELDS)
    for s in _settings():
        got, used = _one_grid_run(s, w)
        _equal(ref, got)
        for k, v in s.items():
            assert 0 < used[k] <= v or k == "sweep_min_chunk" and used[k] == v, (s, used)


def test_batch_results_do_not_depend_on_the_schedule():
    import torch

    inst = I.batched_instances(count=10, nmin=40, nmax=200, steps=5, seed=77)

    def run(sched):
        b = ebit.EbitBatch([s for s, _, _, _ in inst])
        if sched is not None:
            b.set_schedule(sched)
        U, V = b.pack_velocities([u for _, u, _, _ in inst], [v for _, _, v, _ in inst])
        C, K = b.new_fields()
        for k in range(5):
            b.advect(U, V, torch.tensor([d[k] for _, _, _, d in inst], dtype=torch.float64, device="cuda:0"))
        b.fraction_curvature(C, K)
        torch.cuda.synchronize()
        out = []
        for g in range(len(inst)):
            st = b.get_state(g)
            out += [st.c, st.cc, st.hoff * st.h_present(), st.voff * st.v_present()]
        out += [C.cpu().numpy(), K.cpu().numpy()]
        b.close()
        return out

    ref = run(None)
    for s in _settings():
        _equal(ref, run(s))


def test_tuner_picks_a_schedule_and_caches_it(tmp_path):
    import torch

    w = I.many_circles(n=256, count=40, rmin=3.0, rmax=12.0, period=4.0, nsteps=40, seed=5)
    g = ebit.EbitGrid(w.state)
    u, v = torch.from_numpy(w.u).cuda(), torch.from_numpy(w.v).cuda()
    C, K = g.new_field(), g.new_field()
    k = [0]

    def step():
        g.advect(u, v, w.dts[k[0] % 40])
        g.fraction_curvature(C, K)
        k[0] += 1

    path = str(tmp_path / "sched.json")
    key = tune.size_key("one", 256 * 256)
    best, info = tune.tune(g, step, g.stream, steps=2, reps=1, key=key, path=path)
    assert g.get_schedule() == best and info["us_per_step"] > 0
    assert tune.schedule_for(key, path) == best
