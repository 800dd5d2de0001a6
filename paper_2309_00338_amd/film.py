"""Python binding of the two-markers-per-edge step (include/ebit_film.h).

Argument marshalling only: every pass runs in the library's HIP kernels. A
film state is a set of numpy arrays in the header's layout; `FilmState.of`
turns a one-marker state (inputs.State) into one.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import ebit
from .ebit import _chk, ebit_grid
from .inputs import State


class ebit_film_state(ctypes.Structure):
    _fields_ = [("node_color", ctypes.c_void_p), ("cell_color", ctypes.c_void_p), ("hcount", ctypes.c_void_p),
                ("hoff", ctypes.c_void_p), ("vcount", ctypes.c_void_p), ("voff", ctypes.c_void_p)]


ebit_film_out = ebit_film_state  # same fields, written by the library

FILM_COUNTERS = ("markers", "annihilated", "annihilated_unaligned", "three_crossings", "parity_fail")


class ebit_film_counters(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in FILM_COUNTERS]


def _declare(lib):
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    G = ctypes.POINTER(ebit_grid)
    sigs = {
        "ebit_film_workspace_bytes": [G, ctypes.POINTER(sz)],
        "ebit_film_create": [G, ctypes.c_double, ctypes.POINTER(ebit_film_state), ctypes.c_int64, vp, sz, vp,
                             ctypes.POINTER(vp)],
        "ebit_film_advect": [vp, vp, vp, ctypes.c_double],
        "ebit_film_fraction": [vp, vp],
        "ebit_film_get_state": [vp, ctypes.POINTER(ebit_film_out)],
        "ebit_film_set_state": [vp, ctypes.POINTER(ebit_film_state), ctypes.c_int64],
        "ebit_film_stats": [vp, ctypes.POINTER(ebit_film_counters)],
        "ebit_film_sync": [vp],
        "ebit_film_destroy": [vp],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    return lib


_lib = _declare(ebit.lib())


@dataclass
class FilmState:
    """Node and centre colours, marker counts (0, 1, 2) and offset pairs."""
    nx: int
    ny: int
    h: float
    c: np.ndarray   # (ny+1, nx+1) uint8
    cc: np.ndarray  # (ny, nx) uint8
    hn: np.ndarray  # (ny+1, nx) uint8
    ho: np.ndarray  # (ny+1, nx, 2) float64, ascending, the first hn meaningful
    vn: np.ndarray  # (ny, nx+1) uint8
    vo: np.ndarray  # (ny, nx+1, 2) float64
    step: int = 0

    @classmethod
    def of(cls, st: State) -> "FilmState":
        """A one-marker state: one marker on every edge whose end colours differ."""
        c = np.ascontiguousarray(st.c, np.uint8)
        hn = (c[:, :-1] != c[:, 1:]).astype(np.uint8)
        vn = (c[:-1, :] != c[1:, :]).astype(np.uint8)
        ho = np.zeros((st.ny + 1, st.nx, 2))
        vo = np.zeros((st.ny, st.nx + 1, 2))
        ho[..., 0] = np.where(hn == 1, st.hoff, 0.0)
        vo[..., 0] = np.where(vn == 1, st.voff, 0.0)
        return cls(st.nx, st.ny, st.h, c, np.ascontiguousarray(st.cc, np.uint8), hn, ho, vn, vo, st.step)

    def copy(self) -> "FilmState":
        return FilmState(self.nx, self.ny, self.h, self.c.copy(), self.cc.copy(), self.hn.copy(), self.ho.copy(),
                         self.vn.copy(), self.vo.copy(), self.step)

    def _arrays(self):
        return [np.ascontiguousarray(a, dt) for a, dt in ((self.c, np.uint8), (self.cc, np.uint8),
                                                          (self.hn, np.uint8), (self.ho, np.float64),
                                                          (self.vn, np.uint8), (self.vo, np.float64))]

    def _host(self):
        arrs = self._arrays()
        return ebit_film_state(*[a.ctypes.data for a in arrs]), arrs


def workspace_bytes(nx: int, ny: int, h: float) -> int:
    n = ctypes.c_size_t()
    _chk(_lib.ebit_film_workspace_bytes(ctypes.byref(ebit_grid(nx, ny, h, 0)), ctypes.byref(n)),
         "ebit_film_workspace_bytes")
    return n.value


class EbitFilm:
    """A two-markers-per-edge interface on one grid, resident on the GPU.
    delta is the rupture gap in cell widths (math.inf: no films)."""

    def __init__(self, state: FilmState, delta: float, device: str = "cuda:0", stream=None):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.nx, self.ny, self.h = state.nx, state.ny, state.h
        self.grid = ebit_grid(state.nx, state.ny, state.h, 0)
        nbytes = workspace_bytes(state.nx, state.ny, state.h)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        s, keep = state._host()
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _chk(_lib.ebit_film_create(ctypes.byref(self.grid), float(delta), ctypes.byref(s), int(state.step),
                                       self.ws.data_ptr(), nbytes, self.stream.cuda_stream, ctypes.byref(handle)),
                 "ebit_film_create")
        self._h = handle
        self.step = int(state.step)

    def _dev(self, t, shape, name):
        torch = self.torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != self.device:
            raise TypeError(f"{name} must be a float64 tensor on {self.device}")
        if tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {shape}, got {tuple(t.shape)}")
        return t.data_ptr()

    def advect(self, u, v, dt: float):
        pu = self._dev(u, (self.ny, self.nx + 1), "u")
        pv = self._dev(v, (self.ny + 1, self.nx), "v")
        _chk(_lib.ebit_film_advect(self._h, pu, pv, float(dt)), "ebit_film_advect")
        self.step += 1

    def fraction(self, C=None):
        C = self.torch.empty((self.ny, self.nx), dtype=self.torch.float64, device=self.device) if C is None else C
        _chk(_lib.ebit_film_fraction(self._h, self._dev(C, (self.ny, self.nx), "C")), "ebit_film_fraction")
        return C

    def get_state(self) -> FilmState:
        nx, ny = self.nx, self.ny
        st = FilmState(nx, ny, self.h, np.empty((ny + 1, nx + 1), np.uint8), np.empty((ny, nx), np.uint8),
                       np.empty((ny + 1, nx), np.uint8), np.empty((ny + 1, nx, 2)), np.empty((ny, nx + 1), np.uint8),
                       np.empty((ny, nx + 1, 2)), self.step)
        out = ebit_film_out(*[a.ctypes.data for a in (st.c, st.cc, st.hn, st.ho, st.vn, st.vo)])
        _chk(_lib.ebit_film_get_state(self._h, ctypes.byref(out)), "ebit_film_get_state")
        return st

    def set_state(self, state: FilmState):
        s, keep = state._host()
        _chk(_lib.ebit_film_set_state(self._h, ctypes.byref(s), int(state.step)), "ebit_film_set_state")
        self.step = int(state.step)

    def stats(self) -> dict:
        out = ebit_film_counters()
        _chk(_lib.ebit_film_stats(self._h, ctypes.byref(out)), "ebit_film_stats")
        return {k: getattr(out, k) for k in FILM_COUNTERS}

    def sync(self) -> int:
        return _lib.ebit_film_sync(self._h)

    def close(self):
        if getattr(self, "_h", None):
            _lib.ebit_film_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
