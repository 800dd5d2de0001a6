"""The entry point for callers that cannot allocate device memory
(ebit_step_static, include/ebit.h) against the handle path it varies
(ebit_create + ebit_advect + ebit_fraction_curvature): the same state, C and
kappa, bit for bit, on two calls in a row, the second on a smaller grid (the
scratch keeps the first call's contents), and a grid beyond the scratch
rejected before any device work."""
import ctypes

import numpy as np
import pytest

from paper_2309_00338_amd import inputs as I

pytestmark = pytest.mark.gpu


def _case(n, m, seed):
    st = I.init_state(n, m, [I.Circle(0.5 * n + 0.31, 0.55 * m - 0.17, 0.3 * min(n, m)),
                             I.Ellipse(0.2 * n + 0.4, 0.25 * m, 0.12 * min(n, m), 0.07 * min(n, m), 0.6)],
                      h=1.0 / max(n, m))
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y = np.arange(n + 1) / n, np.arange(m + 1) / m
    psi = (np.sin(np.pi * x)[None, :] ** 2) * (np.sin(np.pi * y)[:, None] ** 2) / np.pi * rng.uniform(0.5, 1.5)
    psi[0, :] = psi[-1, :] = psi[:, 0] = psi[:, -1] = 0.0
    u, v = I.faces_from_psi(psi, st.h)
    dt = 0.45 * st.h / max(np.abs(u).max(), np.abs(v).max())
    return st, u, v, dt


def _static_step(st, u, v, dt, step):
    import torch

    from paper_2309_00338_amd import ebit

    d = "cuda:0"
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(d)  # noqa: E731
    node, cell, hoff, voff = T(st.c), T(st.cc), T(st.hoff), T(st.voff)
    C = torch.full((st.ny, st.nx), -7.0, dtype=torch.float64, device=d)
    K = torch.full((st.ny, st.nx), -7.0, dtype=torch.float64, device=d)
    status = torch.full((1,), -1, dtype=torch.int32, device=d)
    g = ebit.ebit_grid(st.nx, st.ny, st.h, 0)
    rc = ebit.step_static(g, node, cell, hoff, voff, T(u), T(v), dt, step, C, K, status)
    assert rc == ebit.EBIT_OK, ebit.strerror(rc)
    torch.cuda.synchronize()
    out = I.State(st.nx, st.ny, st.h, node.cpu().numpy(), cell.cpu().numpy(), hoff.cpu().numpy(),
                  voff.cpu().numpy(), st.step + 1)
    return out, C.cpu().numpy(), K.cpu().numpy(), int(status.item())


def _handle_step(st, u, v, dt, step):
    import torch

    from paper_2309_00338_amd import ebit

    s = st.copy()
    s.step = step
    g = ebit.EbitGrid(s, device="cuda:0")
    g.advect(torch.from_numpy(u).to("cuda:0"), torch.from_numpy(v).to("cuda:0"), dt)
    C, K = g.fraction_curvature()
    torch.cuda.synchronize()
    return g.get_state(), C.cpu().numpy(), K.cpu().numpy()


def _same(a, b):
    sa, Ca, Ka = a
    sb, Cb, Kb = b
    assert np.array_equal(sa.c, sb.c) and np.array_equal(sa.cc, sb.cc)
    hp, vp = sb.h_present(), sb.v_present()
    assert np.array_equal(sa.hoff[hp], sb.hoff[hp]) and np.array_equal(sa.voff[vp], sb.voff[vp])
    assert np.array_equal(Ca, Cb)
    assert np.array_equal(np.isnan(Ka), np.isnan(Kb))
    fin = ~np.isnan(Kb)
    assert np.array_equal(Ka[fin], Kb[fin])


def test_static_scratch_step_matches_the_handle_path_twice_in_a_row():
    for (n, m, seed, step) in ((200, 170, 3, 0), (72, 60, 4, 1)):
        st, u, v, dt = _case(n, m, seed)
        print(f"static step {n}x{m} seed {seed} step {step}", flush=True)
        s_out, Cs, Ks, status = _static_step(st, u, v, dt, step)
        assert status == 0
        _same((s_out, Cs, Ks), _handle_step(st, u, v, dt, step))
        assert st.n_markers() > 50 and s_out.n_markers() > 50


def test_static_scratch_rejects_a_grid_beyond_it():
    import torch

    from paper_2309_00338_amd import ebit

    n = 1400
    assert ebit.workspace_bytes(n, n, 1.0 / n) > ebit.STATIC_SCRATCH_BYTES
    g = ebit.ebit_grid(n, n, 1.0 / n, 0)
    z = ctypes.c_void_p(16)  # never dereferenced: the size check comes first
    rc = ebit.lib().ebit_step_static(ctypes.byref(g), z, z, z, z, z, z, 1e-3, 0, z, z, z,
                                     torch.cuda.current_stream().cuda_stream)
    assert rc == ebit.EBIT_ERR_NOMEM
