"""GPU parity at the full benchmark sizes, in the launch configuration the
benchmark times (same library calls, same tiles and persistent grids): two
steps of each large workload, every node, edge, centre colour, C and kappa
compared with the oracle."""
import pytest

from paper_2309_00338_amd import inputs as I
from tests.parity import Lockstep

pytestmark = pytest.mark.gpu


def _two_steps(w):
    print(f"[full] {w.name}: {w.state.n_markers()} markers", flush=True)
    ls = Lockstep(w.state, w.u, w.v)
    for k in range(2):
        ls.step(w.dts[k], where=f"{w.name} step {k}")
        print(f"[full] {w.name} step {k} ok {ls.worst}", flush=True)
    cnt = ls.compare_counters()
    assert cnt["markers"] > 0
    return cnt


def test_config2_large_grid_8192():
    _two_steps(I.many_circles(n=8192, count=2000, nsteps=2))


def test_config3a_merging_pairs_4096():
    _two_steps(I.merging_pairs(n=4096, pairs=500, nsteps=2))


def test_config3b_cosine_4096():
    _two_steps(I.cosine_interface(n=4096, nsteps=2))
