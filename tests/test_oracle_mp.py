"""Pin P10: the FP64 oracle against a 50-digit reference of the same sweep
(tests/mp_reference.py, written independently and organised per output) on
tiny grids: identical colours, centre colours and marker presence, and marker
offsets within 1e-13 cell widths, sweep by sweep, except in a sweep where the
oracle counted a near-degenerate decision (a tie, within 1e-12), where FP64
rounding may legitimately decide the other way."""
import numpy as np
import pytest

import oracle
from paper_2309_00338_amd import inputs as I
from tests import mp_reference as MP


def _smooth_case(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = [I.Circle(n * rng.uniform(0.3, 0.45), n * rng.uniform(0.3, 0.7), n * rng.uniform(0.12, 0.2)),
              I.Ellipse(n * rng.uniform(0.65, 0.72), n * rng.uniform(0.3, 0.7), n * 0.14, n * 0.08,
                        rng.uniform(0, np.pi))]
    st = I.init_state(n, n, shapes, h=1.0 / n)
    x = np.arange(n + 1) / n
    psi = np.zeros((n + 1, n + 1))
    for _ in range(3):
        k, l = rng.integers(1, 4, 2)
        psi += rng.normal(0, 0.1) * np.sin(k * np.pi * x)[None, :] * np.sin(l * np.pi * x)[:, None]
    u, v = I.faces_from_psi(psi, st.h)
    dt = 0.45 * st.h / max(np.abs(u).max(), np.abs(v).max())
    return st, u, v, dt


def _dense_case(n, seed):
    st = I.random_colouring(n, n, seed=seed)
    u, v = I.shear_faces(n, n, seed + 7)
    dt = 0.45 * st.h / max(np.abs(u).max(), np.abs(v).max())
    return st, u, v, dt


def _compare(a, b, where):
    assert np.array_equal(a.c, b.c), where
    assert np.array_equal(a.cc, b.cc), where
    hp, vp = a.h_present(), a.v_present()
    dh = np.abs(a.hoff - b.hoff)[hp].max(initial=0.0)
    dv = np.abs(a.voff - b.voff)[vp].max(initial=0.0)
    assert dh <= 1e-13 and dv <= 1e-13, (where, dh, dv)
    return max(dh, dv)


@pytest.mark.parametrize("kind,n,seed", [("smooth", 12, 1), ("smooth", 16, 2), ("smooth", 16, 3),
                                         ("dense", 10, 4), ("dense", 12, 5), ("dense", 12, 6)])
def test_oracle_sweeps_equal_the_50_digit_reference(kind, n, seed):
    st, u, v, dt = (_smooth_case if kind == "smooth" else _dense_case)(n, seed)
    compared, worst, events = 0, 0.0, 0
    for s in range(6):
        d = s % 2 if kind == "smooth" else (s + seed) % 2
        ref = MP.sweep(st, u, v, dt, d)
        o = st.copy()
        rc, cnt = oracle.sweep(o, u, v, dt, d)
        assert rc == oracle.OK
        c = oracle.counters_dict(cnt)
        if c["ties"] == 0:
            worst = max(worst, _compare(o, ref, f"{kind} {n} seed {seed} sweep {s}"))
            compared += 1
        events += c["annihilated"] + c["cv_set"] + c["three_landers"] + c["three_crossings"]
        st = o  # continue from the oracle's state
    assert compared >= 4 and events > 0, (compared, events)
