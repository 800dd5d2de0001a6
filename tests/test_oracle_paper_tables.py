"""Reproduction of the paper's kinematic tables by the oracle.

Single vortex (Sec. 3.3, Tables 3 and 4), translation (Sec. 3.2, Table 1) and
Zalesak's disk (Sec. 3.4, Table 5), circle fit (EBIT) and straight line
(EBIT-SL, the method's first version). The EBIT-SL rows and the Zalesak E_sym
of the circle fit are matched within a few percent, which pins the advection,
landing, annihilation and centre-CV readings over hundreds of steps. The
circle-fit area and shape errors depend on unpublished details of the paper's
implementation (centre-CV figures, tie rules) and are held to a factor 3 and to
falling with resolution.

E_sym is estimated as sum |C(T) - C(0)| h^2, a lower bound of the area of the
symmetric difference of the two reconstructions (equal to it where, cell by
cell, one region contains the other).
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2309_00338_amd import inputs as I
from tests.helpers import e_area, e_shape

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
TIGHT = 0.06  # relative tolerance on the matched rows


def _errors(st, C0, cx, cy, r, n):
    C1 = oracle.fraction(st)
    if C1.sum() == 0.0:
        return None
    return {"E_area": e_area(C0, C1), "E_shape": e_shape(st, cx, cy, r) / n,
            "E_sym": float(np.abs(C1 - C0).sum()) / (n * n)}


def _vortex(n, period, line=False):
    w = I.single_vortex(n, period=period, cfl=0.125)
    st = w.state
    C0 = oracle.fraction(st)
    for dt in w.dts:
        assert oracle.step(st, w.u, w.v, dt, line=line)[0] == oracle.OK
    return _errors(st, C0, 0.5 * n, 0.75 * n, 0.15 * n, n)


def _translation(n, line=False):
    w = I.translation(n)
    st = w.state
    C0 = oracle.fraction(st)
    for k, dt in enumerate(w.dts):
        s = 1.0 if k < w.meta["reverse_at"] else -1.0
        assert oracle.step(st, s * w.u, s * w.v, dt, line=line)[0] == oracle.OK
    return _errors(st, C0, 0.25 * n, 0.75 * n, 0.15 * n, n)


def _zalesak(n, line=False):
    w = I.zalesak(n)
    st = w.state
    C0 = oracle.fraction(st)
    for dt in w.dts:
        assert oracle.step(st, w.u, w.v, dt, line=line)[0] == oracle.OK
    return _errors(st, C0, 0.5 * n, 0.75 * n, 0.15 * n, n)


def _close(ours, paper, rel):
    return abs(ours - paper) <= rel * paper


# ours / paper for the T = 2 circle-fit rows at N = 32, 64 (time factor at t_n):
# E_area 0.70, 0.66; E_shape 0.60, 0.54; E_sym 0.79, 0.82
T2_BOUNDS = {"E_area": (0.6, 1.25), "E_shape": (0.45, 1.25), "E_sym": (0.6, 1.25)}


def test_vortex_T2_close_to_table_3():
    tab = GOLD["vortex_T2"]
    prev = None
    for n in (32, 64):
        e = _vortex(n, 2.0)
        k = tab["N"].index(n)
        for key, (lo, hi) in T2_BOUNDS.items():
            assert lo * tab[key][k] <= e[key] <= hi * tab[key][k], (n, key, e[key], tab[key][k])
        if prev:
            assert e["E_area"] < prev["E_area"] and e["E_shape"] < prev["E_shape"]
        prev = e


def test_vortex_T8_within_factor_3_of_table_4():
    tab = GOLD["vortex_T8"]
    for n in (32, 64):
        e = _vortex(n, 8.0)
        k = tab["N"].index(n)
        assert tab["E_area"][k] / 3 <= e["E_area"] <= tab["E_area"][k] * 3, (n, e)
        assert tab["E_shape"][k] / 3 <= e["E_shape"] <= tab["E_shape"][k] * 3, (n, e)


def test_translation_circle_fit_is_exact_table_1():
    """Table 1 EBIT row: errors of 1e-9 and below, which the paper attributes to
    its root-finding initialisation; with analytic initial markers the round
    trip is exact to rounding."""
    for n in (32, 64):
        e = _translation(n)
        assert e["E_area"] < 1e-12 and e["E_shape"] < 1e-12 and e["E_sym"] < 1e-12, (n, e)


def test_translation_straight_line_matches_table_1():
    tab = GOLD["translation_SL"]
    assert _translation(32, line=True) is None  # NA: the whole reference phase is lost
    for n in (64, 128):
        e = _translation(n, line=True)
        k = tab["N"].index(n)
        for key in ("E_area", "E_shape", "E_sym"):
            assert _close(e[key], tab[key][k], TIGHT), (n, key, e[key], tab[key][k])


def test_vortex_T2_straight_line_matches_table_3():
    tab = GOLD["vortex_T2_SL"]
    for n in (32, 64):
        e = _vortex(n, 2.0, line=True)
        k = tab["N"].index(n)
        for key in ("E_area", "E_shape", "E_sym"):
            assert _close(e[key], tab[key][k], TIGHT), (n, key, e[key], tab[key][k])


def test_vortex_T8_straight_line_loses_the_phase_table_4():
    """Table 4 EBIT-SL: NA at N = 32 and 64."""
    for n in (32, 64):
        assert _vortex(n, 8.0, line=True) is None


def test_zalesak_matches_table_5():
    cf, sl = GOLD["zalesak"], GOLD["zalesak_SL"]
    assert _zalesak(32, line=True) is None
    for n in (32, 64, 128):
        k = cf["N"].index(n)
        e = _zalesak(n)
        assert _close(e["E_sym"], cf["E_sym"][k], TIGHT), (n, e, cf["E_sym"][k])
        assert cf["E_area"][k] / 3 <= e["E_area"] <= cf["E_area"][k] * 3, (n, e)
        if n > 32:
            s = _zalesak(n, line=True)
            for key in ("E_area", "E_sym"):
                assert _close(s[key], sl[key][k], TIGHT), (n, key, s[key], sl[key][k])


def test_straight_line_never_places_a_marker_outside_a_convex_shape():
    """EBIT-SL chords lie inside a convex interface, so under translation every
    marker stays within the exact circle and the area only shrinks."""
    n = 64
    w = I.translation(n)
    st = w.state
    from tests.helpers import markers_xy

    areas = [oracle.fraction(st).sum()]
    cx, cy = 0.25 * n, 0.75 * n
    for k in range(40):
        assert oracle.step(st, w.u, w.v, w.dts[k], line=True)[0] == oracle.OK
        cx += w.u[0, 0] * w.dts[k] * n
        cy += w.v[0, 0] * w.dts[k] * n
        X, Y = markers_xy(st)
        assert np.all(np.hypot(X - cx, Y - cy) <= 0.15 * n + 1e-9), k
        areas.append(oracle.fraction(st).sum())
    assert all(b <= a + 1e-9 for a, b in zip(areas, areas[1:]))
    assert areas[-1] < areas[0]
