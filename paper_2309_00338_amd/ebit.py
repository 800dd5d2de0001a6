"""Python binding of libebit.so (the MI355X EBIT interface step).

Argument marshalling only: torch tensors supply device memory and the stream,
every step of the path runs in the library's HIP kernels. The names follow the
C-ABI in include/ebit.h. Importing this module fails loudly when the built
library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from .inputs import State

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libebit.so")

EBIT_OK, EBIT_ERR_ARG, EBIT_ERR_STATE, EBIT_ERR_CFL, EBIT_ERR_DOMAIN, EBIT_ERR_DEVICE, EBIT_ERR_NOMEM = range(7)
EBIT_SWEEP_ALTERNATE, EBIT_SWEEP_XY = 0, 1

COUNTERS = (
    "markers", "annihilated", "three_landers", "ties", "fit_fallback", "fit_reject",
    "parity_fallback", "three_crossings", "cv_set", "cv_conflict", "cv_unresolved",
    "wall_violation", "invariant_fail", "hf_fail", "interfacial",
    "tiles_swept", "tiles_empty", "tiles_near",
)
# counters that describe the GPU schedule and have no oracle counterpart
SCHEDULE_COUNTERS = ("tiles_swept", "tiles_empty", "tiles_near")


class ebit_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("h", ctypes.c_double), ("flags", ctypes.c_uint32)]


class ebit_state(ctypes.Structure):
    _fields_ = [("node_color", ctypes.c_void_p), ("cell_color", ctypes.c_void_p), ("hoff", ctypes.c_void_p),
                ("voff", ctypes.c_void_p)]


class ebit_counters(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in COUNTERS]


class EbitError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} (code {code})")


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libebit.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    G, S = ctypes.POINTER(ebit_grid), ctypes.POINTER(ebit_state)
    sigs = {
        "ebit_workspace_bytes": [G, ctypes.POINTER(sz)],
        "ebit_create": [G, S, vp, sz, vp, ctypes.POINTER(vp)],
        "ebit_advect": [vp, vp, vp, ctypes.c_double],
        "ebit_fraction": [vp, vp],
        "ebit_curvature": [vp, vp, vp],
        "ebit_fraction_curvature": [vp, vp, vp],
        "ebit_get_state": [vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int64)],
        "ebit_set_state": [vp, S, ctypes.c_int64],
        "ebit_stats": [vp, ctypes.POINTER(ebit_counters)],
        "ebit_stats_reset": [vp],
        "ebit_sync": [vp],
        "ebit_destroy": [vp],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.ebit_strerror.argtypes = [ctypes.c_int]
    lib.ebit_strerror.restype = ctypes.c_char_p
    return lib


_lib = _load()


def lib() -> ctypes.CDLL:
    return _lib


def strerror(code: int) -> str:
    return _lib.ebit_strerror(int(code)).decode()


def _chk(rc: int, where: str):
    if rc != EBIT_OK:
        raise EbitError(rc, where)


def workspace_bytes(nx: int, ny: int, h: float, flags: int = 0) -> int:
    g = ebit_grid(nx, ny, h, flags)
    n = ctypes.c_size_t(0)
    _chk(_lib.ebit_workspace_bytes(ctypes.byref(g), ctypes.byref(n)), "ebit_workspace_bytes")
    return n.value


def _host_state(st: State):
    arrs = (np.ascontiguousarray(st.c, np.uint8), np.ascontiguousarray(st.cc, np.uint8),
            np.ascontiguousarray(st.hoff, np.float64), np.ascontiguousarray(st.voff, np.float64))
    s = ebit_state(*(a.ctypes.data for a in arrs))
    return s, arrs


class EbitGrid:
    """One EBIT interface on one uniform grid, resident on the GPU."""

    def __init__(self, state: State, flags: int = EBIT_SWEEP_ALTERNATE, device: str = "cuda:0", stream=None):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.nx, self.ny, self.h = state.nx, state.ny, state.h
        self.grid = ebit_grid(state.nx, state.ny, state.h, flags)
        nbytes = workspace_bytes(state.nx, state.ny, state.h, flags)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        s, keep = _host_state(state)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _chk(_lib.ebit_create(ctypes.byref(self.grid), ctypes.byref(s), self.ws.data_ptr(), nbytes,
                                  self.stream.cuda_stream, ctypes.byref(handle)), "ebit_create")
        self._h = handle
        self.step = state.step

    # -- checks ---------------------------------------------------------
    def _dev(self, t, shape, name):
        torch = self.torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != self.device:
            raise TypeError(f"{name} must be a float64 tensor on {self.device}")
        if tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {shape}, got {tuple(t.shape)}")
        return t.data_ptr()

    def new_field(self):
        return self.torch.empty((self.ny, self.nx), dtype=self.torch.float64, device=self.device)

    # -- the four calls ----------------------------------------------------
    def advect(self, u, v, dt: float):
        pu = self._dev(u, (self.ny, self.nx + 1), "u")
        pv = self._dev(v, (self.ny + 1, self.nx), "v")
        _chk(_lib.ebit_advect(self._h, pu, pv, float(dt)), "ebit_advect")
        self.step += 1

    def fraction(self, C=None):
        C = self.new_field() if C is None else C
        _chk(_lib.ebit_fraction(self._h, self._dev(C, (self.ny, self.nx), "C")), "ebit_fraction")
        return C

    def curvature(self, C, K=None):
        K = self.new_field() if K is None else K
        _chk(_lib.ebit_curvature(self._h, self._dev(C, (self.ny, self.nx), "C"),
                                 self._dev(K, (self.ny, self.nx), "K")), "ebit_curvature")
        return K

    def fraction_curvature(self, C=None, K=None):
        C = self.new_field() if C is None else C
        K = self.new_field() if K is None else K
        _chk(_lib.ebit_fraction_curvature(self._h, self._dev(C, (self.ny, self.nx), "C"),
                                          self._dev(K, (self.ny, self.nx), "K")), "ebit_fraction_curvature")
        return C, K

    # -- state, counters ---------------------------------------------------
    def get_state(self) -> State:
        c = np.empty((self.ny + 1, self.nx + 1), np.uint8)
        cc = np.empty((self.ny, self.nx), np.uint8)
        hoff = np.empty((self.ny + 1, self.nx), np.float64)
        voff = np.empty((self.ny, self.nx + 1), np.float64)
        step = ctypes.c_int64(0)
        _chk(_lib.ebit_get_state(self._h, c.ctypes.data, cc.ctypes.data, hoff.ctypes.data, voff.ctypes.data,
                                 ctypes.byref(step)), "ebit_get_state")
        return State(self.nx, self.ny, self.h, c, cc, hoff, voff, int(step.value))

    def set_state(self, state: State):
        s, keep = _host_state(state)
        _chk(_lib.ebit_set_state(self._h, ctypes.byref(s), int(state.step)), "ebit_set_state")
        self.step = state.step

    def stats(self) -> dict:
        out = ebit_counters()
        _chk(_lib.ebit_stats(self._h, ctypes.byref(out)), "ebit_stats")
        return {k: int(getattr(out, k)) for k in COUNTERS}

    def stats_reset(self):
        _chk(_lib.ebit_stats_reset(self._h), "ebit_stats_reset")

    def sync(self):
        _chk(_lib.ebit_sync(self._h), "ebit_sync")

    def close(self):
        if getattr(self, "_h", None):
            _lib.ebit_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
