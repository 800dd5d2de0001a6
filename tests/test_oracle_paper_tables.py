"""Soft reproduction of the paper's kinematic tables by the oracle.

Single vortex (Sec. 3.3, Tables 3 and 4) at CFL 0.125: the area and shape
errors of the returned circle must lie within a factor 3 of the published EBIT
values and fall with resolution (the paper reports about first order). The
paper's numbers come from its Basilisk implementation, whose unpublished
details (centre-CV figures, tie rules) differ from this oracle's readings, so
this is a loose gate, not parity.
"""
import json
import os

import pytest

import oracle
from paper_2309_00338_amd import inputs as I
from tests.helpers import e_area, e_shape

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def _run(n, period):
    w = I.single_vortex(n, period=period, cfl=0.125)
    st = w.state
    C0 = oracle.fraction(st)
    for dt in w.dts:
        assert oracle.step(st, w.u, w.v, dt)[0] == oracle.OK
    return e_area(C0, oracle.fraction(st)), e_shape(st, 0.5 * n, 0.75 * n, 0.15 * n) / n


def test_vortex_T2_within_factor_3_of_table_3():
    tab = GOLD["vortex_T2"]
    prev = None
    for n in (32, 64):
        ea, es = _run(n, 2.0)
        k = tab["N"].index(n)
        assert tab["E_area"][k] / 3 <= ea <= tab["E_area"][k] * 3, (n, ea)
        assert tab["E_shape"][k] / 3 <= es <= tab["E_shape"][k] * 3, (n, es)
        if prev:
            assert ea < prev[0] and es < prev[1]
        prev = (ea, es)


def test_vortex_T8_within_factor_3_of_table_4():
    tab = GOLD["vortex_T8"]
    for n in (32, 64):
        ea, es = _run(n, 8.0)
        k = tab["N"].index(n)
        assert tab["E_area"][k] / 3 <= ea <= tab["E_area"][k] * 3, (n, ea)
        assert tab["E_shape"][k] / 3 <= es <= tab["E_shape"][k] * 3, (n, es)
