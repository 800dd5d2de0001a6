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
EBIT_SWEEP_ALTERNATE, EBIT_SWEEP_XY, EBIT_FIT_LINE = 0, 1, 2

COUNTERS = (
    "markers", "annihilated", "three_landers", "ties", "fit_fallback", "fit_reject",
    "parity_fallback", "three_crossings", "cv_set", "cv_conflict", "cv_unresolved",
    "wall_violation", "invariant_fail", "hf_fail", "interfacial", "ghf_fit",
    "tiles_swept", "tiles_empty", "tiles_near",
)
# counters that describe the GPU schedule and have no oracle counterpart
SCHEDULE_COUNTERS = ("tiles_swept", "tiles_empty", "tiles_near")


class ebit_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("h", ctypes.c_double), ("flags", ctypes.c_uint32)]


class ebit_state(ctypes.Structure):
    _fields_ = [("node_color", ctypes.c_void_p), ("cell_color", ctypes.c_void_p), ("hoff", ctypes.c_void_p),
                ("voff", ctypes.c_void_p)]


class ebit_fluid(ctypes.Structure):
    _fields_ = [("rho1", ctypes.c_double), ("rho2", ctypes.c_double), ("mu1", ctypes.c_double),
                ("mu2", ctypes.c_double), ("sigma", ctypes.c_double)]


class ebit_schedule(ctypes.Structure):
    _fields_ = [("sweep_per_cu", ctypes.c_uint32), ("fit_per_cu", ctypes.c_uint32),
                ("sweep_min_chunk", ctypes.c_uint32), ("frac_near_per_cu", ctypes.c_double),
                ("ns_near_per_cu", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


SCHEDULE_FIELDS = tuple(k for k, _ in ebit_schedule._fields_)


class ebit_counters(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in COUNTERS]


class EbitError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        detail = ""
        if code == EBIT_ERR_DEVICE:
            detail = ": " + _lib.ebit_device_error().decode()
        super().__init__(f"{where}: {strerror(code)} (code {code}){detail}")


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libebit.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    # torch first: it brings its own HIP and HSA runtimes, and the library must
    # bind to those (one HSA runtime per process) rather than load a second copy
    import torch  # noqa: F401

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
        "ebit_ns_fields": [vp, vp, vp, ctypes.POINTER(ebit_fluid), vp, vp, vp, vp],
        "ebit_get_state": [vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int64)],
        "ebit_set_state": [vp, S, ctypes.c_int64],
        "ebit_stats": [vp, ctypes.POINTER(ebit_counters)],
        "ebit_stats_reset": [vp],
        "ebit_get_schedule": [vp, ctypes.POINTER(ebit_schedule)],
        "ebit_set_schedule": [vp, ctypes.POINTER(ebit_schedule)],
        "ebit_batch_get_schedule": [vp, ctypes.POINTER(ebit_schedule)],
        "ebit_batch_set_schedule": [vp, ctypes.POINTER(ebit_schedule)],
        "ebit_pool_get_schedule": [vp, ctypes.POINTER(ebit_schedule)],
        "ebit_pool_set_schedule": [vp, ctypes.POINTER(ebit_schedule)],
        "ebit_sync": [vp],
        "ebit_destroy": [vp],
    }
    B, P = vp, vp
    i32, u32, szp = ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(sz)
    sigs.update({
        "ebit_batch_workspace_bytes": [i32, G, szp],
        "ebit_batch_create": [i32, G, S, vp, sz, vp, ctypes.POINTER(vp)],
        "ebit_batch_layout": [B, szp, szp, szp, szp],
        "ebit_batch_advect": [B, vp, vp, vp],
        "ebit_batch_fraction_curvature": [B, vp, vp],
        "ebit_batch_ns_fields": [B, vp, vp, ctypes.POINTER(ebit_fluid), vp, vp, vp, vp],
        "ebit_batch_get_state": [B, i32, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int64)],
        "ebit_batch_stats": [B, ctypes.POINTER(ebit_counters)],
        "ebit_batch_sync": [B, ctypes.POINTER(ctypes.c_int)],
        "ebit_batch_destroy": [B],
        "ebit_pool_workspace_bytes": [i32, u32, sz, szp],
        "ebit_pool_grid_bytes": [G, szp, ctypes.POINTER(u32)],
        "ebit_pool_create": [i32, u32, vp, sz, vp, ctypes.POINTER(vp)],
        "ebit_pool_admit": [P, G, S, vp, vp, ctypes.c_double, ctypes.POINTER(ctypes.c_int)],
        "ebit_pool_step": [P],
        "ebit_pool_read": [P, i32, vp, vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int)],
        "ebit_pool_get_state": [P, i32, vp, vp, vp, vp],
        "ebit_pool_retire": [P, i32],
        "ebit_pool_status": [P, vp],
        "ebit_pool_stats": [P, ctypes.POINTER(ebit_counters)],
        "ebit_pool_destroy": [P],
        "ebit_batch_capture": [B, i32, vp, vp, vp, vp, vp, ctypes.POINTER(vp)],
        "ebit_graph_launch": [vp],
        "ebit_graph_destroy": [vp],
        "ebit_step_static": [G, vp, vp, vp, vp, vp, vp, ctypes.c_double, ctypes.c_int64, vp, vp, vp, vp],
    })
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.ebit_strerror.argtypes = [ctypes.c_int]
    lib.ebit_strerror.restype = ctypes.c_char_p
    lib.ebit_device_error.argtypes = []
    lib.ebit_device_error.restype = ctypes.c_char_p
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


STATIC_SCRATCH_BYTES = 80 << 20  # EBIT_STATIC_SCRATCH_BYTES of include/ebit.h


def step_static(grid: ebit_grid, node, cell, hoff, voff, u, v, dt: float, step: int, C, K, status, stream=None):
    """ebit_step_static on device tensors (uint8 node/cell colours, float64
    offsets, velocities and fields, one int32 status), all on the current
    device: the state tensors are overwritten with the state after the step.
    Returns the call's status code (argument and HIP errors); the device-side
    status lands in `status`."""
    import torch

    st = stream if stream is not None else torch.cuda.current_stream()
    want = {"node": (node, torch.uint8, (grid.ny + 1, grid.nx + 1)), "cell": (cell, torch.uint8, (grid.ny, grid.nx)),
            "hoff": (hoff, torch.float64, (grid.ny + 1, grid.nx)), "voff": (voff, torch.float64, (grid.ny, grid.nx + 1)),
            "u": (u, torch.float64, (grid.ny, grid.nx + 1)), "v": (v, torch.float64, (grid.ny + 1, grid.nx)),
            "C": (C, torch.float64, (grid.ny, grid.nx)), "K": (K, torch.float64, (grid.ny, grid.nx)),
            "status": (status, torch.int32, (1,))}
    for name, (t, dt_, shape) in want.items():
        if t.dtype != dt_ or tuple(t.shape) != shape or not t.is_contiguous() or not t.is_cuda:
            raise ValueError(f"{name} must be a contiguous {dt_} device tensor of shape {shape}")
    return _lib.ebit_step_static(ctypes.byref(grid), node.data_ptr(), cell.data_ptr(), hoff.data_ptr(),
                                 voff.data_ptr(), u.data_ptr(), v.data_ptr(), float(dt), int(step), C.data_ptr(),
                                 K.data_ptr(), status.data_ptr(), st.cuda_stream)


def _get_schedule(fn, h) -> dict:
    out = ebit_schedule()
    _chk(fn(h, ctypes.byref(out)), fn.__name__)
    return out.as_dict()


def _set_schedule(fn, h, sched: dict):
    s = ebit_schedule(**{k: sched.get(k, 0) for k in SCHEDULE_FIELDS})
    _chk(fn(h, ctypes.byref(s)), fn.__name__)


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
        self.step = 0
        if state.step:
            # ebit_create starts at step 0; the step number picks the sweep order
            self.set_state(state)

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

    def ns_fields(self, C, K, rho1, rho2, mu1, mu2, sigma, rho=None, mu=None, fx=None, fy=None):
        """Density, viscosity (per cell) and surface-tension face forces from the
        current C and kappa; new tensors for any output not given."""
        t = self.torch
        rho = self.new_field() if rho is None else rho
        mu = self.new_field() if mu is None else mu
        fx = t.empty((self.ny, self.nx + 1), dtype=t.float64, device=self.device) if fx is None else fx
        fy = t.empty((self.ny + 1, self.nx), dtype=t.float64, device=self.device) if fy is None else fy
        fl = ebit_fluid(rho1, rho2, mu1, mu2, sigma)
        _chk(_lib.ebit_ns_fields(self._h, self._dev(C, (self.ny, self.nx), "C"), self._dev(K, (self.ny, self.nx), "K"),
                                 ctypes.byref(fl), self._dev(rho, (self.ny, self.nx), "rho"),
                                 self._dev(mu, (self.ny, self.nx), "mu"), self._dev(fx, (self.ny, self.nx + 1), "fx"),
                                 self._dev(fy, (self.ny + 1, self.nx), "fy")), "ebit_ns_fields")
        return rho, mu, fx, fy

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

    def get_schedule(self) -> dict:
        return _get_schedule(_lib.ebit_get_schedule, self._h)

    def set_schedule(self, sched: dict):
        """Launch schedule (ebit_schedule fields; missing or 0 = device default)."""
        _set_schedule(_lib.ebit_set_schedule, self._h, sched)

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


def _empty_state(nx: int, ny: int, h: float, step: int = 0) -> State:
    return State(nx, ny, h, np.empty((ny + 1, nx + 1), np.uint8), np.empty((ny, nx), np.uint8),
                 np.empty((ny + 1, nx), np.float64), np.empty((ny, nx + 1), np.float64), step)


class EbitBatch:
    """A fixed set of independent grids advanced together (one launch per
    phase for all of them). Velocities, C and K live in packed device buffers;
    grid k's arrays start at the element offsets of the layout."""

    def __init__(self, states, flags=EBIT_SWEEP_ALTERNATE, device: str = "cuda:0", stream=None):
        """flags: one value for every grid or one per grid."""
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.n = n = len(states)
        if n < 1:
            raise ValueError("a batch needs at least one grid")
        self.shapes = [(st.nx, st.ny, st.h) for st in states]
        fl = list(flags) if hasattr(flags, "__len__") else [flags] * n
        if len(fl) != n:
            raise ValueError("one flags value per grid")
        grids = (ebit_grid * n)(*[ebit_grid(st.nx, st.ny, st.h, int(f)) for st, f in zip(states, fl)])
        hs, keep = [], []
        for st in states:
            s, k = _host_state(st)
            hs.append(s)
            keep.append(k)
        inits = (ebit_state * n)(*hs)
        nbytes = ctypes.c_size_t(0)
        _chk(_lib.ebit_batch_workspace_bytes(n, grids, ctypes.byref(nbytes)), "ebit_batch_workspace_bytes")
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _chk(_lib.ebit_batch_create(n, grids, inits, self.ws.data_ptr(), nbytes.value, self.stream.cuda_stream,
                                        ctypes.byref(handle)), "ebit_batch_create")
        self._h = handle
        uo, vo, co, tot = ((ctypes.c_size_t * n)(), (ctypes.c_size_t * n)(), (ctypes.c_size_t * n)(),
                           (ctypes.c_size_t * 3)())
        _chk(_lib.ebit_batch_layout(self._h, uo, vo, co, tot), "ebit_batch_layout")
        self.u_off, self.v_off, self.c_off = list(uo), list(vo), list(co)
        self.totals = tuple(tot)
        self.step = 0
        self._graphs = []

    def pack_velocities(self, us, vs):
        """Device buffers holding grid k's u and v (host arrays) at the layout's offsets."""
        torch = self.torch
        U = np.zeros(self.totals[0], np.float64)
        V = np.zeros(self.totals[1], np.float64)
        for k, (u, v) in enumerate(zip(us, vs)):
            nx, ny, _ = self.shapes[k]
            assert u.shape == (ny, nx + 1) and v.shape == (ny + 1, nx)
            U[self.u_off[k]:self.u_off[k] + u.size] = u.ravel()
            V[self.v_off[k]:self.v_off[k] + v.size] = v.ravel()
        return torch.from_numpy(U).to(self.device), torch.from_numpy(V).to(self.device)

    def new_fields(self):
        t = self.torch
        return (t.empty(self.totals[2], dtype=t.float64, device=self.device),
                t.empty(self.totals[2], dtype=t.float64, device=self.device))

    def field(self, F, k):
        nx, ny, _ = self.shapes[k]
        return F[self.c_off[k]:self.c_off[k] + nx * ny].view(ny, nx)

    def _buf(self, t, n, name):
        torch = self.torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != self.device:
            raise TypeError(f"{name} must be a float64 tensor on {self.device}")
        if t.numel() < n or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with at least {n} elements")
        return t.data_ptr()

    def advect(self, U, V, dts):
        pu = self._buf(U, self.totals[0], "u")
        pv = self._buf(V, self.totals[1], "v")
        pd = self._buf(dts, self.n, "dts")
        _chk(_lib.ebit_batch_advect(self._h, pu, pv, pd), "ebit_batch_advect")
        self.step += 1

    def fraction_curvature(self, C, K):
        _chk(_lib.ebit_batch_fraction_curvature(self._h, self._buf(C, self.totals[2], "C"),
                                                self._buf(K, self.totals[2], "K")), "ebit_batch_fraction_curvature")
        return C, K

    def ns_fields(self, C, K, rho1, rho2, mu1, mu2, sigma):
        """Packed rho, mu (C layout), fx (u layout), fy (v layout) of every grid."""
        t = self.torch
        rho = t.empty(self.totals[2], dtype=t.float64, device=self.device)
        mu = t.empty(self.totals[2], dtype=t.float64, device=self.device)
        fx = t.empty(self.totals[0], dtype=t.float64, device=self.device)
        fy = t.empty(self.totals[1], dtype=t.float64, device=self.device)
        fl = ebit_fluid(rho1, rho2, mu1, mu2, sigma)
        _chk(_lib.ebit_batch_ns_fields(self._h, self._buf(C, self.totals[2], "C"), self._buf(K, self.totals[2], "K"),
                                       ctypes.byref(fl), rho.data_ptr(), mu.data_ptr(), fx.data_ptr(), fy.data_ptr()),
             "ebit_batch_ns_fields")
        return rho, mu, fx, fy

    def get_state(self, k) -> State:
        nx, ny, h = self.shapes[k]
        st = _empty_state(nx, ny, h)
        step = ctypes.c_int64(0)
        _chk(_lib.ebit_batch_get_state(self._h, k, st.c.ctypes.data, st.cc.ctypes.data, st.hoff.ctypes.data,
                                       st.voff.ctypes.data, ctypes.byref(step)), "ebit_batch_get_state")
        st.step = int(step.value)
        return st

    def get_schedule(self) -> dict:
        return _get_schedule(_lib.ebit_batch_get_schedule, self._h)

    def set_schedule(self, sched: dict):
        _set_schedule(_lib.ebit_batch_set_schedule, self._h, sched)

    def stats(self) -> dict:
        out = ebit_counters()
        _chk(_lib.ebit_batch_stats(self._h, ctypes.byref(out)), "ebit_batch_stats")
        return {k: int(getattr(out, k)) for k in COUNTERS}

    def sync(self):
        """Per-grid status codes (0 = ok)."""
        st = (ctypes.c_int * self.n)()
        _lib.ebit_batch_sync(self._h, st)
        return list(st)

    def capture(self, ksteps: int, U, V, dts, C, K):
        """ebit_batch_capture: the next ksteps (even) steps of every grid,
        step k with the dts[k] row (device tensor of ksteps x n), then fraction
        and curvature into C, K, recorded as one graph (EbitGraph)."""
        pd = self._buf(dts, ksteps * self.n, "dts")
        out = ctypes.c_void_p()
        _chk(_lib.ebit_batch_capture(self._h, int(ksteps), self._buf(U, self.totals[0], "u"),
                                     self._buf(V, self.totals[1], "v"), pd, self._buf(C, self.totals[2], "C"),
                                     self._buf(K, self.totals[2], "K"), ctypes.byref(out)), "ebit_batch_capture")
        g = EbitGraph(self, out, int(ksteps), (U, V, dts, C, K))
        self._graphs.append(g)
        return g

    def close(self):
        for g in getattr(self, "_graphs", []):
            g.close()
        if getattr(self, "_h", None):
            _lib.ebit_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class EbitGraph:
    """K captured steps of a batch; launch() replays them on the batch's stream."""

    def __init__(self, batch, handle, ksteps, buffers):
        self.batch, self._h, self.ksteps = batch, handle, ksteps
        self._keep = buffers  # the graph reads these at every replay

    def launch(self):
        _chk(_lib.ebit_graph_launch(self._h), "ebit_graph_launch")
        self.batch.step += self.ksteps

    def close(self):
        if getattr(self, "_h", None):
            _lib.ebit_graph_destroy(self._h)
            self._h = None


class EbitPool:
    """Served form: grids admitted and retired between steps; every admitted
    grid takes one step (advection, fraction, curvature) per step() call."""

    def __init__(self, max_grids: int, max_tiles: int, arena_bytes: int, device: str = "cuda:0", stream=None):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        nbytes = ctypes.c_size_t(0)
        _chk(_lib.ebit_pool_workspace_bytes(max_grids, max_tiles, arena_bytes, ctypes.byref(nbytes)),
             "ebit_pool_workspace_bytes")
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _chk(_lib.ebit_pool_create(max_grids, max_tiles, self.ws.data_ptr(), nbytes.value,
                                       self.stream.cuda_stream, ctypes.byref(handle)), "ebit_pool_create")
        self._h = handle
        self.shapes = {}
        self.max_grids = max_grids
        self._inflight = []  # host arrays of admissions the stream may not have read yet

    @staticmethod
    def grid_bytes(nx: int, ny: int, h: float):
        g = ebit_grid(nx, ny, h, 0)
        b, t = ctypes.c_size_t(0), ctypes.c_uint32(0)
        _chk(_lib.ebit_pool_grid_bytes(ctypes.byref(g), ctypes.byref(b), ctypes.byref(t)), "ebit_pool_grid_bytes")
        return b.value, t.value

    def admit(self, state, u, v, dt: float, flags: int = EBIT_SWEEP_ALTERNATE):
        """Slot of the admitted grid, or None when the pool is full. The state
        arrays (a State, or a dict with nx, ny, h, c, cc, hoff, voff) and u, v
        may be numpy arrays or CPU torch tensors (pinned ones keep the upload
        asynchronous); they are referenced here until the stream has passed
        the admission (a later read() or sync())."""
        get = (lambda k: state[k]) if isinstance(state, dict) else (lambda k: getattr(state, k))
        nx, ny, h = int(get("nx")), int(get("ny")), float(get("h"))
        arrs = {}
        want = {"c": ((ny + 1, nx + 1), np.uint8), "cc": ((ny, nx), np.uint8), "hoff": ((ny + 1, nx), np.float64),
                "voff": ((ny, nx + 1), np.float64), "u": ((ny, nx + 1), np.float64), "v": ((ny + 1, nx), np.float64)}
        src = {"c": get("c"), "cc": get("cc"), "hoff": get("hoff"), "voff": get("voff"), "u": u, "v": v}
        ptrs = {}
        for k, (shape, dt_) in want.items():
            a = src[k]
            if isinstance(a, self.torch.Tensor):
                if a.is_cuda or tuple(a.shape) != shape or not a.is_contiguous() or \
                        a.dtype != {np.uint8: self.torch.uint8, np.float64: self.torch.float64}[dt_]:
                    raise ValueError(f"{k}: a contiguous CPU tensor of shape {shape} and dtype {dt_} is required")
                ptrs[k] = a.data_ptr()
            else:
                a = np.ascontiguousarray(a, dt_)
                if a.shape != shape:
                    raise ValueError(f"{k}: shape {a.shape}, expected {shape}")
                ptrs[k] = a.ctypes.data
            arrs[k] = a
        g = ebit_grid(nx, ny, h, flags)
        s = ebit_state(ptrs["c"], ptrs["cc"], ptrs["hoff"], ptrs["voff"])
        slot = ctypes.c_int(-1)
        rc = _lib.ebit_pool_admit(self._h, ctypes.byref(g), ctypes.byref(s), ptrs["u"], ptrs["v"], float(dt),
                                  ctypes.byref(slot))
        if rc == EBIT_ERR_NOMEM:
            return None
        _chk(rc, "ebit_pool_admit")
        self.shapes[slot.value] = (nx, ny, h)
        self._inflight.append(arrs)
        return slot.value

    def step(self):
        _chk(_lib.ebit_pool_step(self._h), "ebit_pool_step")

    def status(self, out=None):
        """Every slot's status into a device int32 tensor (asynchronous)."""
        out = self.torch.empty(self.max_grids, dtype=self.torch.int32, device=self.device) if out is None else out
        _chk(_lib.ebit_pool_status(self._h, out.data_ptr()), "ebit_pool_status")
        return out

    def sync(self):
        self.stream.synchronize()
        self._inflight = []

    def read(self, slot: int, fields: bool = True):
        nx, ny, _ = self.shapes[slot]
        C = np.empty((ny, nx), np.float64) if fields else None
        K = np.empty((ny, nx), np.float64) if fields else None
        steps, status = ctypes.c_int64(0), ctypes.c_int(0)
        _chk(_lib.ebit_pool_read(self._h, slot, C.ctypes.data if fields else None, K.ctypes.data if fields else None,
                                 ctypes.byref(steps), ctypes.byref(status)), "ebit_pool_read")
        self._inflight = []  # the read waited on the stream
        return C, K, int(steps.value), int(status.value)

    def get_state(self, slot: int) -> State:
        nx, ny, h = self.shapes[slot]
        st = _empty_state(nx, ny, h)
        _chk(_lib.ebit_pool_get_state(self._h, slot, st.c.ctypes.data, st.cc.ctypes.data, st.hoff.ctypes.data,
                                      st.voff.ctypes.data), "ebit_pool_get_state")
        return st

    def retire(self, slot: int):
        _chk(_lib.ebit_pool_retire(self._h, slot), "ebit_pool_retire")
        self.shapes.pop(slot, None)

    def get_schedule(self) -> dict:
        return _get_schedule(_lib.ebit_pool_get_schedule, self._h)

    def set_schedule(self, sched: dict):
        _set_schedule(_lib.ebit_pool_set_schedule, self._h, sched)

    def stats(self) -> dict:
        out = ebit_counters()
        _chk(_lib.ebit_pool_stats(self._h, ctypes.byref(out)), "ebit_pool_stats")
        return {k: int(getattr(out, k)) for k in COUNTERS}

    def close(self):
        if getattr(self, "_h", None):
            _lib.ebit_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
