"""CPU oracle for the EBIT interface step (TEST INFRASTRUCTURE ONLY).

A plain, slow, single-threaded FP64 implementation of what the GPU path
computes, written from Pan et al., arXiv 2309.00338 (Sec. 2.1-2.5). Only the
tests, the smoke check and the benchmark's CPU-baseline leg may import it; the
product library never does, and it shares no source with the product.

Every function below updates or reads numpy arrays laid out exactly as the
library's host state (row-major, x fastest). Parity unpinned parts are listed
in the test-suite docstrings where each pin lives.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB, build_oracle

COUNTERS = (
    "markers", "annihilated", "three_landers", "ties", "fit_fallback", "fit_reject",
    "parity_fallback", "three_crossings", "cv_set", "cv_conflict", "cv_unresolved",
    "wall_violation", "invariant_fail", "hf_fail", "interfacial", "ghf_fit",
)

OK, ERR_ARG, ERR_CFL, ERR_DOMAIN = 0, 1, 3, 4

_lib = None
_u8p = ctypes.POINTER(ctypes.c_uint8)
_f64p = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_oracle()
        lib = ctypes.CDLL(LIB)
        lib.or_sweep.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _u8p, _u8p, _f64p, _f64p, _f64p,
                                 _f64p, ctypes.c_double, ctypes.c_int, ctypes.c_int, _i64p]
        lib.or_step.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _u8p, _u8p, _f64p, _f64p, _f64p,
                                _f64p, ctypes.c_double, ctypes.c_int64, ctypes.c_int, _i64p]
        lib.or_fraction.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _u8p, _f64p, _f64p, _f64p]
        lib.or_curvature.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _u8p, _f64p, _f64p, _f64p, _f64p,
                                     _i64p]
        d = ctypes.c_double
        lib.or_ns_fields.argtypes = [ctypes.c_int, ctypes.c_int, d, _u8p, _f64p, _f64p, d, d, d, d, d, _f64p,
                                     _f64p, _f64p, _f64p]
        lib.or_parabola_fit.argtypes = [ctypes.c_int, _f64p, _f64p, d, d, ctypes.c_int, ctypes.c_int, d, _f64p]
        for f in (lib.or_sweep, lib.or_step, lib.or_fraction, lib.or_curvature, lib.or_ns_fields,
                  lib.or_parabola_fit):
            f.restype = ctypes.c_int
        lib.or_tie_log.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.c_int64]
        lib.or_tie_log.restype = None
        lib.or_tie_count.argtypes = []
        lib.or_tie_count.restype = ctypes.c_int64
        assert lib.or_counter_count() == len(COUNTERS)
        _lib = lib
    return _lib


def _p(a, t):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(t)


def _check(st):
    assert st.c.dtype == np.uint8 and st.c.shape == (st.ny + 1, st.nx + 1)
    assert st.cc.dtype == np.uint8 and st.cc.shape == (st.ny, st.nx)
    assert st.hoff.dtype == np.float64 and st.hoff.shape == (st.ny + 1, st.nx)
    assert st.voff.dtype == np.float64 and st.voff.shape == (st.ny, st.nx + 1)


def new_counters():
    return np.zeros(len(COUNTERS), np.int64)


def counters_dict(arr):
    return {k: int(v) for k, v in zip(COUNTERS, arr)}


TIE_KINDS = {1: "landed offset at a node", 2: "crossing endpoint on the line", 3: "equal crossing heights",
             4: "root on the chord", 5: "new offset at a node"}


class _TieLog:
    """Collects the oracle's tie locations during one call, as dicts with the
    kind, the sweep direction and the edge in grid coordinates: ("H", i, j) or
    ("V", i, j). Kind 1 concerns the sweep's aligned edge, kinds 2-5 its new
    unaligned edge."""

    def __init__(self, out, cap=1 << 16):
        self.out, self.cap = out, cap

    def __enter__(self):
        if self.out is not None:
            self.buf = np.zeros(4 * self.cap, np.int32)
            _load().or_tie_log(self.buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), self.cap)
        return self

    def __exit__(self, *exc):
        if self.out is None:
            return False
        lib = _load()
        n = min(int(lib.or_tie_count()), self.cap)
        lib.or_tie_log(None, 0)
        for k in range(n):
            kind, d, a, b = (int(x) for x in self.buf[4 * k:4 * k + 4])
            aligned = kind == 1
            if d == 0:
                edge = ("H", a, b) if aligned else ("V", a, b)
            else:
                edge = ("V", b, a) if aligned else ("H", b, a)
            self.out.append({"kind": kind, "what": TIE_KINDS[kind], "dir": d, "edge": edge})
        return False


def sweep(st, u, v, dt, direction, counters=None, line=False, ties=None):
    """One 1D sweep in place (direction 0 = x with u, 1 = y with v); line:
    EBIT-SL placement of the new unaligned markers instead of the circle fit."""
    _check(st)
    cnt = new_counters() if counters is None else counters
    u = np.ascontiguousarray(u, np.float64)
    v = np.ascontiguousarray(v, np.float64)
    with _TieLog(ties):
        rc = _load().or_sweep(st.nx, st.ny, st.h, _p(st.c, _u8p), _p(st.cc, _u8p), _p(st.hoff, _f64p),
                              _p(st.voff, _f64p), _p(u, _f64p), _p(v, _f64p), float(dt), int(direction),
                              2 if line else 0, _p(cnt, _i64p))
    return rc, cnt


def step(st, u, v, dt, xy_only=False, counters=None, line=False, ties=None):
    """One time step (two sweeps) in place; advances st.step. line: EBIT-SL.
    ties: a list that receives the locations of the step's ties."""
    _check(st)
    cnt = new_counters() if counters is None else counters
    u = np.ascontiguousarray(u, np.float64)
    v = np.ascontiguousarray(v, np.float64)
    with _TieLog(ties):
        rc = _load().or_step(st.nx, st.ny, st.h, _p(st.c, _u8p), _p(st.cc, _u8p), _p(st.hoff, _f64p),
                             _p(st.voff, _f64p), _p(u, _f64p), _p(v, _f64p), float(dt), int(st.step),
                             (1 if xy_only else 0) | (2 if line else 0), _p(cnt, _i64p))
    st.step += 1
    return rc, cnt


def fraction(st):
    _check(st)
    C = np.empty((st.ny, st.nx), np.float64)
    _load().or_fraction(st.nx, st.ny, _p(st.c, _u8p), _p(st.cc, _u8p), _p(st.hoff, _f64p), _p(st.voff, _f64p),
                        _p(C, _f64p))
    return C


def curvature(st, C, counters=None):
    _check(st)
    cnt = new_counters() if counters is None else counters
    C = np.ascontiguousarray(C, np.float64)
    K = np.empty((st.ny, st.nx), np.float64)
    _load().or_curvature(st.nx, st.ny, st.h, _p(st.c, _u8p), _p(st.hoff, _f64p), _p(st.voff, _f64p), _p(C, _f64p),
                         _p(K, _f64p), _p(cnt, _i64p))
    return K, cnt


def ns_fields(st, C, K, rho1, rho2, mu1, mu2, sigma):
    """Density and viscosity per cell (Eq. physical with H = C) and the
    surface-tension face forces sigma kappa_f grad C on the x- and y-faces."""
    _check(st)
    C = np.ascontiguousarray(C, np.float64)
    K = np.ascontiguousarray(K, np.float64)
    rho = np.empty((st.ny, st.nx))
    mu = np.empty((st.ny, st.nx))
    fx = np.empty((st.ny, st.nx + 1))
    fy = np.empty((st.ny + 1, st.nx))
    rc = _load().or_ns_fields(st.nx, st.ny, st.h, _p(st.c, _u8p), _p(C, _f64p), _p(K, _f64p), rho1, rho2, mu1, mu2,
                              sigma, _p(rho, _f64p), _p(mu, _f64p), _p(fx, _f64p), _p(fy, _f64p))
    assert rc == OK
    return rho, mu, fx, fy


def parabola_fit(px, py, xc, yc, gx, gy, h):
    """Curvature of the least-squares parabola through points (px, py) in the
    frame of the normal (gx, gy) at (xc, yc), the curvature fallback; None when
    the fit is not defined."""
    px = np.ascontiguousarray(px, np.float64)
    py = np.ascontiguousarray(py, np.float64)
    k = np.zeros(1)
    ok = _load().or_parabola_fit(len(px), _p(px, _f64p), _p(py, _f64p), float(xc), float(yc), int(gx), int(gy),
                                 float(h), _p(k, _f64p))
    return float(k[0]) if ok else None
