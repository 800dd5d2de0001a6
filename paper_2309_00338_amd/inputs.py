"""Seeded synthetic inputs for the EBIT interface step.

This module only *generates* data: initial interfaces (node colours, centre
colours and exact edge crossings), MAC face velocities and time-step schedules.
It holds none of the method's arithmetic, and both the GPU library and the CPU
oracle consume what it produces.

Conventions (index space, as in the library header): node (i, j) sits at the
integer point (i, j); cell (i, j) is [i, i+1] x [j, j+1]; H(i, j) is the edge
from node (i, j) to (i+1, j) and its marker is at (i + hoff, j); V(i, j) joins
(i, j) and (i, j+1) with the marker at (i, j + voff). u[j][i] is the x-face
velocity at (i, j + 1/2) and v[j][i] the y-face velocity at (i + 1/2, j), both
in physical units on the unit square (cell size h = 1/N).

Shapes are given in index units (cell widths). The reference phase (colour 1)
is the inside of the shapes; the initial centre colour is the phase at the cell
centre, and every edge whose end colours differ carries the analytic crossing
(the paper initialises markers by root finding on the signed distance,
Sec. 3.2; closed forms are used here where they exist).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class State:
    """Host copy of an EBIT interface state (row-major, x fastest)."""

    nx: int
    ny: int
    h: float
    c: np.ndarray  # uint8 (ny+1, nx+1) node colours
    cc: np.ndarray  # uint8 (ny, nx) centre colours
    hoff: np.ndarray  # float64 (ny+1, nx)
    voff: np.ndarray  # float64 (ny, nx+1)
    step: int = 0

    def copy(self) -> "State":
        return State(self.nx, self.ny, self.h, self.c.copy(), self.cc.copy(), self.hoff.copy(),
                     self.voff.copy(), self.step)

    def h_present(self) -> np.ndarray:
        return self.c[:, :-1] != self.c[:, 1:]

    def v_present(self) -> np.ndarray:
        return self.c[:-1, :] != self.c[1:, :]

    def n_markers(self) -> int:
        return int(self.h_present().sum() + self.v_present().sum())


# --------------------------------------------------------------------------
# shapes (index units)
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Circle:
    cx: float
    cy: float
    r: float

    def bbox(self):
        return self.cx - self.r, self.cx + self.r, self.cy - self.r, self.cy + self.r

    def inside(self, X, Y):
        dx = X - self.cx
        dy = Y - self.cy
        return dx * dx + dy * dy < self.r * self.r

    def cross_h(self, i, j, left_inside):
        """x of the boundary on y = j between x = i and i + 1."""
        dy = j - self.cy
        w = np.sqrt(np.maximum(self.r * self.r - dy * dy, 0.0))
        return np.where(left_inside, self.cx + w, self.cx - w)

    def cross_v(self, i, j, low_inside):
        dx = i - self.cx
        w = np.sqrt(np.maximum(self.r * self.r - dx * dx, 0.0))
        return np.where(low_inside, self.cy + w, self.cy - w)


@dataclasses.dataclass
class NotchedDisk:
    """Zalesak's disk (Sec. 3.4): a disk with a rectangular slot of width w and
    length l cut from its bottom, centred on the disk's vertical axis (reading:
    the notch opens towards the rotation centre below the disk). Crossings by
    bisection on the inside test."""
    cx: float
    cy: float
    r: float
    w: float
    l: float

    def bbox(self):
        return self.cx - self.r, self.cx + self.r, self.cy - self.r, self.cy + self.r

    def inside(self, X, Y):
        dx = X - self.cx
        dy = Y - self.cy
        disk = dx * dx + dy * dy < self.r * self.r
        slot = (np.abs(dx) < 0.5 * self.w) & (Y < self.cy - self.r + self.l)
        return disk & ~slot

    def _bisect(self, lo, hi, fixed, along_x, lo_inside):
        lo = np.array(lo, np.float64)
        hi = np.array(hi, np.float64)
        for _ in range(64):
            mid = 0.5 * (lo + hi)
            m = self.inside(mid, fixed) if along_x else self.inside(fixed, mid)
            same = m == lo_inside
            lo = np.where(same, mid, lo)
            hi = np.where(same, hi, mid)
        return 0.5 * (lo + hi)

    def cross_h(self, i, j, left_inside):
        return self._bisect(i, i + 1.0, j, True, left_inside)

    def cross_v(self, i, j, low_inside):
        return self._bisect(j, j + 1.0, i, False, low_inside)


@dataclasses.dataclass
class Ellipse:
    cx: float
    cy: float
    a: float  # semi-axis along the rotated x'
    b: float
    theta: float

    def bbox(self):
        r = max(self.a, self.b)
        return self.cx - r, self.cx + r, self.cy - r, self.cy + r

    def _q(self, X, Y):
        ct, st = math.cos(self.theta), math.sin(self.theta)
        xp = (X - self.cx) * ct + (Y - self.cy) * st
        yp = -(X - self.cx) * st + (Y - self.cy) * ct
        return (xp / self.a) ** 2 + (yp / self.b) ** 2

    def inside(self, X, Y):
        return self._q(X, Y) < 1.0

    def _roots(self, P0x, P0y, Dx, Dy):
        """Roots t of q(P0 + t D) = 1 (quadratic), returned as (t_minus, t_plus)."""
        ct, st = math.cos(self.theta), math.sin(self.theta)
        x0 = P0x - self.cx
        y0 = P0y - self.cy
        px = (x0 * ct + y0 * st) / self.a
        py = (-x0 * st + y0 * ct) / self.b
        dx = (Dx * ct + Dy * st) / self.a
        dy = (-Dx * st + Dy * ct) / self.b
        A = dx * dx + dy * dy
        B = 2.0 * (px * dx + py * dy)
        Cq = px * px + py * py - 1.0
        disc = np.sqrt(np.maximum(B * B - 4 * A * Cq, 0.0))
        return (-B - disc) / (2 * A), (-B + disc) / (2 * A)

    def cross_h(self, i, j, left_inside):
        i = np.asarray(i, dtype=np.float64)
        tm, tp = self._roots(i, np.asarray(j, np.float64), np.ones_like(i), np.zeros_like(i))
        return i + np.where(left_inside, tp, tm)

    def cross_v(self, i, j, low_inside):
        j = np.asarray(j, dtype=np.float64)
        tm, tp = self._roots(np.asarray(i, np.float64), j, np.zeros_like(j), np.ones_like(j))
        return j + np.where(low_inside, tp, tm)


@dataclasses.dataclass
class CosineBelow:
    """Colour 1 below y = N (y0 + amp cos(2 pi x / N)) on an N x N grid (index units)."""

    n: int
    y0: float
    amp: float

    def yif(self, X):
        return self.n * (self.y0 + self.amp * np.cos(2.0 * np.pi * np.asarray(X, np.float64) / self.n))

    def bbox(self):
        return 0.0, float(self.n), 0.0, float(self.n)

    def inside(self, X, Y):
        return Y < self.yif(X)

    def cross_v(self, i, j, low_inside):
        return self.yif(np.asarray(i, np.float64) + 0 * np.asarray(j, np.float64))

    def cross_h(self, i, j, left_inside):
        i = np.asarray(i, dtype=np.float64)
        j = np.asarray(j, dtype=np.float64)
        lo = i.copy()
        hi = i + 1.0
        # bisection on g(x) = yif(x) - j, whose sign differs at the two ends
        glo = self.yif(lo) - j
        for _ in range(64):
            mid = 0.5 * (lo + hi)
            gm = self.yif(mid) - j
            same = np.sign(gm) == np.sign(glo)
            lo = np.where(same, mid, lo)
            glo = np.where(same, gm, glo)
            hi = np.where(same, hi, mid)
        return 0.5 * (lo + hi)


Shape = object


def _clip01(x):
    return np.minimum(np.maximum(x, 0.0), 1.0)


def init_state(nx: int, ny: int, shapes: Sequence[Shape], h: float | None = None) -> State:
    """Colours = inside any shape; every colour-changing edge gets its analytic
    crossing. Shapes must not overlap (each changing edge belongs to one)."""
    if h is None:
        h = 1.0 / nx
    c = np.zeros((ny + 1, nx + 1), np.uint8)
    cc = np.zeros((ny, nx), np.uint8)
    hoff = np.zeros((ny + 1, nx), np.float64)
    voff = np.zeros((ny, nx + 1), np.float64)
    boxes = []
    for s in shapes:
        x0, x1, y0, y1 = s.bbox()
        i0 = max(int(math.floor(x0)) - 1, 0)
        i1 = min(int(math.ceil(x1)) + 1, nx)
        j0 = max(int(math.floor(y0)) - 1, 0)
        j1 = min(int(math.ceil(y1)) + 1, ny)
        boxes.append((i0, i1, j0, j1))
        I, J = np.meshgrid(np.arange(i0, i1 + 1, dtype=np.float64), np.arange(j0, j1 + 1, dtype=np.float64))
        c[j0:j1 + 1, i0:i1 + 1] |= s.inside(I, J).astype(np.uint8)
        if i1 > i0 and j1 > j0:
            Ic, Jc = np.meshgrid(np.arange(i0, i1, dtype=np.float64) + 0.5, np.arange(j0, j1, dtype=np.float64) + 0.5)
            cc[j0:j1, i0:i1] |= s.inside(Ic, Jc).astype(np.uint8)
    for s, (i0, i1, j0, j1) in zip(shapes, boxes):
        I, J = np.meshgrid(np.arange(i0, i1 + 1, dtype=np.float64), np.arange(j0, j1 + 1, dtype=np.float64))
        m = s.inside(I, J)
        # H edges in the box
        dh = m[:, :-1] != m[:, 1:]
        jj, ii = np.nonzero(dh)
        if len(ii):
            gi = ii + i0
            gj = jj + j0
            x = s.cross_h(gi.astype(np.float64), gj.astype(np.float64), m[jj, ii])
            hoff[gj, gi] = _clip01(x - gi)
        dv = m[:-1, :] != m[1:, :]
        jj, ii = np.nonzero(dv)
        if len(ii):
            gi = ii + i0
            gj = jj + j0
            y = s.cross_v(gi.astype(np.float64), gj.astype(np.float64), m[jj, ii])
            voff[gj, gi] = _clip01(y - gj)
    return State(nx, ny, float(h), c, cc, hoff, voff, 0)


# --------------------------------------------------------------------------
# velocity fields (physical units on the unit square)
# --------------------------------------------------------------------------
def _sin_pi_frac(k: np.ndarray, n: int) -> np.ndarray:
    """sin(pi k / n) for integer k in [0, n], exactly 0 at both ends."""
    k = np.asarray(k)
    return np.sin(np.pi * np.minimum(k, n - k) / n)


def faces_from_psi(psi: np.ndarray, h: float) -> Tuple[np.ndarray, np.ndarray]:
    """Node-differenced MAC faces: u = dpsi/dy, v = -dpsi/dx (discretely
    divergence-free; zero wall flux where psi vanishes on the walls)."""
    u = (psi[1:, :] - psi[:-1, :]) / h
    v = -(psi[:, 1:] - psi[:, :-1]) / h
    return np.ascontiguousarray(u), np.ascontiguousarray(v)


def vortex_faces(n: int) -> Tuple[np.ndarray, np.ndarray]:
    """Single-vortex field of Sec. 3.3 at t = 0: psi = sin^2(pi x) sin^2(pi y) / pi.
    The time factor cos(pi t / T) is folded into dt by the caller."""
    h = 1.0 / n
    s = _sin_pi_frac(np.arange(n + 1), n) ** 2
    # u = dpsi/dy at (i, j+1/2); v = -dpsi/dx at (i+1/2, j), psi = s[i] s[j] / pi
    u = (s[None, :] * (s[1:, None] - s[:-1, None])) / (np.pi * h)
    v = -(s[:, None] * (s[None, 1:] - s[None, :-1])) / (np.pi * h)
    return np.ascontiguousarray(u), np.ascontiguousarray(v)


def uniform_faces(nx: int, ny: int, U: float, V: float):
    return np.full((ny, nx + 1), float(U)), np.full((ny + 1, nx), float(V))


def vortex_dt_schedule(dt: float, period: float, nsteps: int, sample: str = "start") -> List[float]:
    """dt_n = dt cos(pi t / T): the vortex time factor folded into the step.

    sample="start" takes t = t_n = n dt, the velocity of time level n that the
    explicit Euler update of Eq. (Eq_marker_dis) uses; over a full period the
    factors then sum to dt, not 0 (the discrete flow ends one start-of-period
    step short of reversing). sample="mid" takes t = t_n + dt/2, whose factors
    are antisymmetric about T/2 and sum to 0 over a whole period."""
    off = {"start": 0.0, "mid": 0.5}[sample]
    return [dt * math.cos(math.pi * ((k + off) * dt) / period) for k in range(nsteps)]


def shear_faces(nx: int, ny: int, seed: int, amp: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """Random face velocities whose sign alternates row by row for u and column
    by column for v (magnitudes uniform in [0.3, 1] amp), zero on the walls: a
    strongly sheared, converging and diverging field that drives markers of
    neighbouring rows past each other (not divergence-free; the kinematic step
    does not need it). Scale dt so that amp * dt / h <= 0.5."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sr = np.where(np.arange(ny) % 2 == 0, 1.0, -1.0)[:, None]
    sc = np.where(np.arange(nx) % 2 == 0, 1.0, -1.0)[None, :]
    u = sr * rng.uniform(0.3 * amp, amp, (ny, nx + 1))
    v = sc * rng.uniform(0.3 * amp, amp, (ny + 1, nx))
    u[:, 0] = u[:, -1] = 0.0
    v[0, :] = v[-1, :] = 0.0
    return np.ascontiguousarray(u), np.ascontiguousarray(v)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    state: State
    u: np.ndarray
    v: np.ndarray
    dts: List[float]
    meta: dict


def single_vortex(n: int = 64, period: float = 2.0, cfl: float = 0.5, radius: float = 0.15,
                  centre=(0.5, 0.75)) -> Workload:
    """One circle in the reversible vortex (Sec. 3.3); u_max = 1 analytically,
    so dt = cfl h and T / dt steps return the shape."""
    h = 1.0 / n
    st = init_state(n, n, [Circle(centre[0] * n, centre[1] * n, radius * n)])
    u, v = vortex_faces(n)
    dt = cfl * h
    nsteps = int(round(period / dt))
    return Workload(f"vortex{n}_T{period:g}", st, u, v, vortex_dt_schedule(dt, period, nsteps),
                    {"period": period, "cfl": cfl, "radius": radius, "centre": centre})


def rotation_faces(n: int) -> Tuple[np.ndarray, np.ndarray]:
    """Rigid rotation about the domain centre (Sec. 3.4): u = 2 pi (0.5 - y),
    v = 2 pi (x - 0.5) on the MAC faces (discretely divergence-free)."""
    h = 1.0 / n
    yc = (np.arange(n) + 0.5) * h
    xc = (np.arange(n) + 0.5) * h
    u = np.repeat((2.0 * np.pi * (0.5 - yc))[:, None], n + 1, axis=1)
    v = np.repeat((2.0 * np.pi * (xc - 0.5))[None, :], n + 1, axis=0)
    return np.ascontiguousarray(u), np.ascontiguousarray(v)


def zalesak(n: int = 64, cfl: float = math.pi / 16) -> Workload:
    """Zalesak's disk (Sec. 3.4): R = 0.15 at (0.5, 0.75), slot 0.05 x 0.25, one
    revolution (T = 1) at CFL = u_max dt / h with u_max = pi at t = 0."""
    st = init_state(n, n, [NotchedDisk(0.5 * n, 0.75 * n, 0.15 * n, 0.05 * n, 0.25 * n)])
    u, v = rotation_faces(n)
    h = 1.0 / n
    dt = cfl * h / math.pi
    nsteps = int(round(1.0 / dt))
    return Workload(f"zalesak{n}", st, u, v, [dt] * nsteps, {"cfl": cfl})


def translation(n: int = 64, cfl: float = 0.125):
    """Translation with uniform velocity (Sec. 3.2): R = 0.15 at (0.25, 0.75),
    u = -v = 1 until t = 0.5, then reversed; returns the workload of the first
    half and the reversed faces for the second."""
    st = init_state(n, n, [Circle(0.25 * n, 0.75 * n, 0.15 * n)])
    u, v = uniform_faces(n, n, 1.0, -1.0)
    dt = cfl / n
    nsteps = int(round(1.0 / dt))
    return Workload(f"translation{n}", st, u, v, [dt] * nsteps, {"cfl": cfl, "reverse_at": nsteps // 2})


def _place_circles(rng, n, count, rmin, rmax, gap, wall, max_tries=200000):
    """Rejection sampling: centre gap >= R1 + R2 + gap, >= R + wall from walls."""
    placed = []
    cell = max(int(2 * rmax + gap) + 1, 1)
    grid = {}
    tries = 0
    while len(placed) < count and tries < max_tries:
        tries += 1
        r = rng.uniform(rmin, rmax)
        cx = rng.uniform(r + wall, n - r - wall)
        cy = rng.uniform(r + wall, n - r - wall)
        gx, gy = int(cx // cell), int(cy // cell)
        ok = True
        for ox in (-1, 0, 1):
            for oy in (-1, 0, 1):
                for (px, py, pr) in grid.get((gx + ox, gy + oy), ()):
                    if (cx - px) ** 2 + (cy - py) ** 2 < (r + pr + gap) ** 2:
                        ok = False
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            placed.append((cx, cy, r))
            grid.setdefault((gx, gy), []).append((cx, cy, r))
    return placed


def many_circles(n: int = 8192, count: int = 2000, rmin: float = 4.0, rmax: float = 32.0, period: float = 4.0,
                 cfl: float = 0.5, nsteps: int = 64, seed: int = 1002) -> Workload:
    """Large single grid: seeded non-overlapping circles (radii in cells) in the
    vortex field with period T."""
    rng = np.random.Generator(np.random.PCG64(seed))
    circles = _place_circles(rng, n, count, rmin, rmax, gap=2.0, wall=2.0)
    st = init_state(n, n, [Circle(*c) for c in circles])
    u, v = vortex_faces(n)
    h = 1.0 / n
    dt = cfl * h
    return Workload(f"circles{n}x{len(circles)}", st, u, v, vortex_dt_schedule(dt, period, nsteps),
                    {"circles": len(circles), "period": period, "cfl": cfl, "seed": seed})


def _sin_2pi_frac(k: np.ndarray, n: int) -> np.ndarray:
    """sin(2 pi k / n) for integer k in [0, n], exactly 0 at k = 0, n/2, n."""
    m = 2 * np.asarray(k)
    return np.where(m <= n, np.sin(np.pi * np.minimum(m, n - m) / n),
                    -np.sin(np.pi * np.minimum(np.maximum(m - n, 0), 2 * n - m) / n))


def _shear_psi(n: int, amp: float = 0.05) -> np.ndarray:
    """psi' = amp/(2 pi) sin^2(pi x) sin(2 pi y), zero on all walls."""
    s2 = _sin_pi_frac(np.arange(n + 1), n) ** 2
    sy = _sin_2pi_frac(np.arange(n + 1), n)
    return (amp / (2.0 * np.pi)) * sy[:, None] * s2[None, :]


def merging_pairs(n: int = 4096, pairs: int = 500, rmin: float = 8.0, rmax: float = 24.0, nsteps: int = 128,
                  cfl: float = 0.5, seed: int = 1003) -> Workload:
    """Topology change: seeded circle pairs separated along x by a 0.5-2 cell gap,
    driven together by u = +-0.5 inside the pair's box (converging on the
    centre line of the cell column that holds the gap's midpoint), plus a weak
    shear."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / n
    psi = _shear_psi(n)
    u, v = faces_from_psi(psi, h)
    shapes = []
    boxes = []
    tries = 0
    while len(boxes) < pairs and tries < 100000:
        tries += 1
        r1 = rng.uniform(rmin, rmax)
        r2 = rng.uniform(rmin, rmax)
        g = rng.uniform(0.5, 2.0)
        w = 2 * r1 + g + 2 * r2
        x0 = rng.uniform(4.0, n - w - 4.0)
        yc = rng.uniform(max(r1, r2) + 4.0, n - max(r1, r2) - 4.0)
        bx0 = int(math.floor(x0 - 2))
        bx1 = int(math.ceil(x0 + w + 2))
        by0 = int(math.floor(yc - max(r1, r2) - 2))
        by1 = int(math.ceil(yc + max(r1, r2) + 2))
        if any(not (bx1 < b[0] or bx0 > b[1] or by1 < b[2] or by0 > b[3]) for b in boxes):
            continue
        boxes.append((bx0, bx1, by0, by1))
        c1 = Circle(x0 + r1, yc, r1)
        c2 = Circle(x0 + 2 * r1 + g + r2, yc, r2)
        shapes += [c1, c2]
        # the flow converges on the centre line of the cell column holding the
        # gap's midpoint, so the facing markers meet inside one edge
        mid = int(math.floor(x0 + 2 * r1 + g / 2))
        # faces (i, j+1/2) with bx0 <= i <= bx1, by0 <= j < by1
        ii = np.arange(bx0, bx1 + 1)
        sgn = np.where(ii <= mid, 0.5, -0.5)
        u[by0:by1, bx0:bx1 + 1] += sgn[None, :]
    st = init_state(n, n, shapes)
    umax = max(np.abs(u).max(), np.abs(v).max())
    dt = cfl * h / umax
    return Workload(f"pairs{n}x{len(boxes)}", st, u, v, [dt] * nsteps, {"pairs": len(boxes), "seed": seed})


def cosine_interface(n: int = 4096, nsteps: int = 128, cfl: float = 0.5, amp: float = 0.01) -> Workload:
    """Perturbed flat interface y = 0.5 + amp cos(2 pi x), colour 1 below, in the
    shear field psi'."""
    h = 1.0 / n
    st = init_state(n, n, [CosineBelow(n, 0.5, amp)])
    psi = _shear_psi(n)
    u, v = faces_from_psi(psi, h)
    umax = max(np.abs(u).max(), np.abs(v).max())
    dt = cfl * h / umax
    return Workload(f"cosine{n}", st, u, v, [dt] * nsteps, {"amp": amp})


def random_instance(rng, n: int, nshapes: int, ellipses: bool = True, period: float | None = None,
                    steps: int = 100, cfl: float = 0.5):
    """A small instance for the batched/served forms: circles or ellipses."""
    shapes = []
    placed = []
    tries = 0
    while len(shapes) < nshapes and tries < 20000:
        tries += 1
        a = rng.uniform(0.03, 0.12) * n
        ratio = rng.uniform(1.0, 3.0) if ellipses else 1.0
        b = max(a / ratio, 3.0)
        r = max(a, b)
        cx = rng.uniform(r + 2, n - r - 2)
        cy = rng.uniform(r + 2, n - r - 2)
        if any((cx - px) ** 2 + (cy - py) ** 2 < (r + pr + 2) ** 2 for px, py, pr in placed):
            continue
        placed.append((cx, cy, r))
        th = rng.uniform(0.0, math.pi)
        shapes.append(Ellipse(cx, cy, a, b, th) if ellipses and ratio > 1.0 else Circle(cx, cy, r))
    st = init_state(n, n, shapes)
    u, v = vortex_faces(n)
    if period is None:
        period = rng.uniform(1.0, 8.0)
    dt = cfl / n
    return st, u, v, vortex_dt_schedule(dt, period, steps)


def random_colouring(nx: int, ny: int, seed: int, p: float = 0.5) -> State:
    """A dense stress state: every node colour and centre colour drawn at
    random (probability p of colour 1), every edge offset uniform in
    [0.05, 0.95], so about half of all edges carry a marker and most cells
    carry two or four."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = (rng.random((ny + 1, nx + 1)) < p).astype(np.uint8)
    cc = (rng.random((ny, nx)) < 0.5).astype(np.uint8)
    hoff = rng.uniform(0.05, 0.95, (ny + 1, nx))
    voff = rng.uniform(0.05, 0.95, (ny, nx + 1))
    return State(nx, ny, 1.0 / max(nx, ny), c, cc, hoff, voff)


def checkerboard(nx: int, ny: int, seed: int) -> State:
    """Node colours alternating in both directions: every edge carries a
    marker and every cell has four (the densest state there is); centre colours
    random, offsets uniform in [0.05, 0.95]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = (np.add.outer(np.arange(ny + 1), np.arange(nx + 1)) & 1).astype(np.uint8)
    cc = (rng.random((ny, nx)) < 0.5).astype(np.uint8)
    hoff = rng.uniform(0.05, 0.95, (ny + 1, nx))
    voff = rng.uniform(0.05, 0.95, (ny, nx + 1))
    return State(nx, ny, 1.0 / max(nx, ny), c, cc, hoff, voff)


def batched_instances(count: int = 256, nmin: int = 64, nmax: int = 1024, steps: int = 100, seed: int = 1004,
                      max_shapes: int = 20):
    """Many independent grids for the batched form: N log-uniform in
    [nmin, nmax], 1..max_shapes circles or ellipses each (semi-major axis 3-12 %
    of the side, axis ratio 1-3, semi-minor >= 3 cells, non-overlapping
    bounding circles), single vortex with its own period T ~ U[1, 8], CFL 0.5
    with the time factor folded into each grid's dt. Returns a list of
    (state, u, v, dts)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        k = int(rng.integers(1, max_shapes + 1))
        out.append(random_instance(rng, n, k, ellipses=True, steps=steps))
    return out


def served_requests(count: int, rate: float = 200.0, nmin: int = 128, nmax: int = 2048, seed: int = 1005,
                    smin: int = 16, smax: int = 256, max_circles: int = 50, modes: int = 4):
    """Request stream for the served form: Poisson arrivals at `rate` per second;
    each request is a grid with N log-uniform in [nmin, nmax], 1..max_circles
    non-overlapping circles of radius U[max(3h, 0.01), 0.08], a steady
    divergence-free field psi = sum_m a_m sin(k_m pi x) sin(l_m pi y) with
    a_m ~ N(0, 0.1) and k_m, l_m in 1..4, dt = 0.5 h / max|face velocity|, and
    U{smin..smax} steps. Yields dicts with the arrival time and the instance,
    built lazily so a long stream never sits in memory at once."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    for r in range(count):
        t += rng.exponential(1.0 / rate)
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        ncirc = int(rng.integers(1, max_circles + 1))
        steps = int(rng.integers(smin, smax + 1))
        amps = rng.normal(0.0, 0.1, modes)
        ks = rng.integers(1, 5, modes)
        ls = rng.integers(1, 5, modes)
        circ_seed = int(rng.integers(0, 2**63 - 1))
        yield {"id": r, "arrival": t, "n": n, "circles": ncirc, "steps": steps, "amps": amps, "ks": ks, "ls": ls,
               "seed": circ_seed}


def served_instance(req):
    """The grid, velocities and dt of one served request (see served_requests)."""
    n = req["n"]
    h = 1.0 / n
    rng = np.random.Generator(np.random.PCG64(req["seed"]))
    rmin = max(3.0 * h, 0.01) * n
    rmax = max(0.08 * n, rmin)
    circles = _place_circles(rng, n, req["circles"], rmin, rmax, gap=2.0, wall=2.0, max_tries=20000)
    st = init_state(n, n, [Circle(*c) for c in circles])
    x = np.arange(n + 1) / n
    psi = np.zeros((n + 1, n + 1))
    for a, k, l in zip(req["amps"], req["ks"], req["ls"]):
        psi += a * np.sin(k * np.pi * x)[None, :] * np.sin(l * np.pi * x)[:, None]
    psi[0, :] = psi[-1, :] = 0.0
    psi[:, 0] = psi[:, -1] = 0.0
    u, v = faces_from_psi(psi, h)
    umax = max(float(np.abs(u).max()), float(np.abs(v).max()), 1e-30)
    dt = 0.5 * h / umax
    return st, u, v, dt
