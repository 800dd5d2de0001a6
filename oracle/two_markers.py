"""CPU oracle of the two-markers-per-edge extension (TEST INFRASTRUCTURE ONLY).

Sec. 2.4 allows one marker per cell edge, so two markers landing on one edge
annihilate and a film thinner than a cell disappears; the paper names the
remedy, more markers per edge (the end of Sec. 2.4, and Sec. 4, where it is
the kinematic extension proposed for thin layers of one fluid), without giving
the algorithm. This module is the reading written out for small grids, in plain
Python FP64 with the same expression orders as the one-marker oracle
(oracle/ebit_oracle.c), which it reduces to exactly when films may not form
(rupture gap delta = inf); only the tests import it.

State. Node colours c, centre colours cc, and per edge a sorted list of 0, 1
or 2 offsets: H[j][i] for the edge (i,j)-(i+1,j), V[j][i] for (i,j)-(i,j+1).
An edge carries an odd number of markers iff its end colours differ (one) and
an even number otherwise (none, or a pair: a film crossing the edge).

Readings (each stated where it is used):
  landing    the landers of an edge, ordered by position: an odd number keeps
             the middle one (as with one marker per edge); an even number
             keeps the middle two when they are at least delta apart (a film
             thicker than the rupture gap), none otherwise (rupture);
  crossings  a new unaligned edge keeps crossings by the same rule, ordered by
             the height where the advected segments cross the line;
  pairing    the markers of a cell, in counter-clockwise order round its
             boundary, cut off every boundary arc whose colour differs from
             the centre colour (two markers: one segment; four: the pairs
             around the corners that differ from the centre, as in Sec. 2.3);
  fraction   the colour-1 area of a cell is the cell (if cc = 1) minus, or the
             sum of (if cc = 0), the regions the segments cut off;
  centre     rules (1)-(5) of Sec. 2.3 as in the one-marker oracle, applied to
             the new unaligned markers of the cell's left edge (lowest first),
             then its right edge.
"""
from __future__ import annotations

import math

import numpy as np

TIE = 1e-12


def _lerp(a, b, t):
    return a + t * (b - a)


class Film:
    """A state with up to two markers per edge (lists of offsets)."""

    def __init__(self, nx, ny, h, c, cc, H, V, step=0):
        self.nx, self.ny, self.h = nx, ny, h
        self.c = np.array(c, np.uint8)
        self.cc = np.array(cc, np.uint8)
        self.H = [[sorted(H[j][i]) for i in range(nx)] for j in range(ny + 1)]
        self.V = [[sorted(V[j][i]) for i in range(nx + 1)] for j in range(ny)]
        self.step = step

    @classmethod
    def from_state(cls, st):
        """A one-marker state (inputs.State) as a film state."""
        H = [[[float(st.hoff[j, i])] if st.c[j, i] != st.c[j, i + 1] else [] for i in range(st.nx)]
             for j in range(st.ny + 1)]
        V = [[[float(st.voff[j, i])] if st.c[j, i] != st.c[j + 1, i] else [] for i in range(st.nx + 1)]
             for j in range(st.ny)]
        return cls(st.nx, st.ny, st.h, st.c, st.cc, H, V, st.step)

    def copy(self):
        return Film(self.nx, self.ny, self.h, self.c, self.cc, self.H, self.V, self.step)

    def check(self):
        for j in range(self.ny + 1):
            for i in range(self.nx):
                assert len(self.H[j][i]) % 2 == int(self.c[j, i] != self.c[j, i + 1]) and len(self.H[j][i]) <= 2
        for j in range(self.ny):
            for i in range(self.nx + 1):
                assert len(self.V[j][i]) % 2 == int(self.c[j, i] != self.c[j + 1, i]) and len(self.V[j][i]) <= 2

    def transposed(self):
        return Film(self.ny, self.nx, self.h, self.c.T, self.cc.T,
                    [[self.V[i][j] for i in range(self.ny)] for j in range(self.nx + 1)],
                    [[self.H[i][j] for i in range(self.ny + 1)] for j in range(self.nx)], self.step)


def _keep(items, order, value, delta):
    """Landing / crossing rule: items sorted by `order`; an odd count keeps the
    middle one, an even count the middle two if their `value`s are at least
    delta apart."""
    items = sorted(items, key=order)
    n = len(items)
    if n % 2 == 1:
        return [items[n // 2]]
    if n == 0:
        return []
    a, b = items[n // 2 - 1], items[n // 2]
    return [a, b] if value(b) - value(a) >= delta else []


def _boundary(c, cc, H, V, p, q):
    """Markers of cell (p, q) in counter-clockwise order from corner BL, each as
    (edge id, index in its edge's list, position along the boundary), and the
    segments as pairs of indices into that list (order: the arc around BL
    first, then counter-clockwise; each segment cuts off an arc whose colour
    differs from the centre colour)."""
    ms = []
    ms += [(0, k, o) for k, o in enumerate(H[q][p])]                       # bottom, left to right
    ms += [(1, k, o) for k, o in enumerate(V[q][p + 1])]                   # right, bottom to top
    ms += [(2, k, o) for k, o in reversed(list(enumerate(H[q + 1][p])))]   # top, right to left
    ms += [(3, k, o) for k, o in reversed(list(enumerate(V[q][p])))]       # left, top to bottom
    n = len(ms)
    if n == 0:
        return ms, []
    # colour of the arc after marker k: BL's colour flipped k + 1 times
    col0 = int(c[q, p])
    segs = []
    for idx in [n - 1] + list(range(n - 1)):
        arc_colour = col0 ^ ((idx + 1) & 1)
        if arc_colour != int(cc[q, p]):
            segs.append((idx, (idx + 1) % n))
    return ms, segs


def _circle_root(Xa, Ya, Xb, Yb, Xc, Yc, Xo, Yo, X2, Y2, X3, Y3, ysl):
    """The one-marker oracle's circle through three points met with X = 0 (same
    expressions): the root across chord P2P3 from (Xo, Yo), else the one
    nearest the chord's height; None when absent or off the edge."""
    Qa = Xa * Xa + Ya * Ya
    Qb = Xb * Xb + Yb * Yb
    Qc = Xc * Xc + Yc * Yc
    ca = Xa * (Yb - Yc) + Xb * (Yc - Ya) + Xc * (Ya - Yb)
    cc = Qa * (Xb - Xc) + Qb * (Xc - Xa) + Qc * (Xa - Xb)
    ce = -(Qa * (Xb * Yc - Xc * Yb) + Qb * (Xc * Ya - Xa * Yc) + Qc * (Xa * Yb - Xb * Ya))
    if ca == 0.0:
        if cc == 0.0:
            return None
        r = -ce / cc
    else:
        disc = cc * cc - 4.0 * ca * ce
        if disc < 0.0:
            disc = 0.0
        sq = math.sqrt(disc)
        qq = -0.5 * (cc + (sq if cc >= 0.0 else -sq))
        if qq == 0.0:
            r1 = r2 = 0.0
        else:
            r1, r2 = qq / ca, ce / qq
        DX, DY = X3 - X2, Y3 - Y2
        so = DX * (Yo - Y2) - DY * (Xo - X2)
        s1 = DX * (r1 - Y2) - DY * (0.0 - X2)
        s2 = DX * (r2 - Y2) - DY * (0.0 - X2)
        q1 = (s1 > 0.0 and so < 0.0) or (s1 < 0.0 and so > 0.0)
        q2 = (s2 > 0.0 and so < 0.0) or (s2 < 0.0 and so > 0.0)
        if q1 and not q2:
            r = r1
        elif q2 and not q1:
            r = r2
        else:
            r = r1 if abs(r1 - ysl) <= abs(r2 - ysl) else r2
    return r if 0.0 <= r <= 1.0 else None


def sweep_x(f: Film, u, lam, delta, stats):
    """One x sweep (Sec. 2.1) of a film state, returned as a new Film."""
    nx, ny = f.nx, f.ny
    c, cc, H, V = f.c, f.cc, f.H, f.V

    def U(i, r):
        return float(u[min(max(r, 0), ny - 1), i])

    # aligned markers: unnormalised advected offsets s' per (edge, index)
    sp = {}
    for j in range(ny + 1):
        for i in range(nx):
            for k, s in enumerate(H[j][i]):
                ub = _lerp(_lerp(U(i, j - 1), U(i + 1, j - 1), s), _lerp(U(i, j), U(i + 1, j), s), 0.5)
                d = ub * lam
                if abs(d) > 0.5:
                    raise ValueError("CFL")
                sp[(i, j, k)] = s + d
    # gray points of unaligned markers: displacement per (edge, index); walls hold
    dv = {}
    for j in range(ny):
        for i in range(nx + 1):
            for k, t in enumerate(V[j][i]):
                ub = _lerp(U(i, j - 1), U(i, j), t + 0.5) if t < 0.5 else _lerp(U(i, j), U(i, j + 1), t - 0.5)
                d = ub * lam
                if abs(d) > 0.5:
                    raise ValueError("CFL")
                dv[(i, j, k)] = 0.0 if i in (0, nx) else d
    # node flips: once per marker passing the node
    nc = c.copy()
    for (i, j, k), s in sp.items():
        if s >= 1.0:
            if i + 1 >= nx:
                raise ValueError("DOMAIN")
            nc[j, i + 1] ^= 1
        elif s < 0.0:
            if i == 0:
                raise ValueError("DOMAIN")
            nc[j, i] ^= 1
    # landing
    nH = [[[] for _ in range(nx)] for _ in range(ny + 1)]
    kept = {}
    for j in range(ny + 1):
        for i in range(nx):
            L = []
            for src in (i - 1, i, i + 1):
                if not 0 <= src < nx:
                    continue
                for k in range(len(H[j][src])):
                    s = sp[(src, j, k)]
                    tgt = src + 1 if s >= 1.0 else (src - 1 if s < 0.0 else src)
                    if tgt == i:
                        o = s - 1.0 if src < i else (s + 1.0 if src > i else s)
                        L.append((o, src, k))
            K = _keep(L, lambda e: e[0], lambda e: e[0], delta)
            stats["annihilated"] += len(L) - len(K)
            for o, src, k in K:
                nH[j][i].append(o)
                kept[(src, j, k)] = i
            nH[j][i].sort()

    def pos(kind, i, j, k, a0, b0):
        """Advected point of marker k of an edge (kind 0 aligned H, 1 gray V) in
        the frame of node (a0, b0), integer part first as in the one-marker
        oracle."""
        if kind == 0:
            return (float(i - a0) + sp[(i, j, k)], float(j - b0))
        return (float(i - a0) + dv[(i, j, k)], float(j - b0) + V[j][i][k])

    def ref(p, q, e, k):
        """(kind, i, j, k) of marker k on edge e of cell (p, q)."""
        return {0: (0, p, q, k), 1: (1, p + 1, q, k), 2: (0, p, q + 1, k), 3: (1, p, q, k)}[e]

    def partner(p, q, e, k):
        """Chain neighbour: the partner, in the cell across edge e of cell (p,q), of marker k of that edge."""
        pp, qq = {0: (p, q - 1), 1: (p + 1, q), 2: (p, q + 1), 3: (p - 1, q)}[e]
        if not (0 <= pp < nx and 0 <= qq < ny):
            return None
        ms, segs = _boundary(c, cc, H, V, pp, qq)
        eo = (e + 2) % 4
        for a, b in segs:
            for x, y in ((a, b), (b, a)):
                if ms[x][0] == eo and ms[x][1] == k:
                    return ref(pp, qq, ms[y][0], ms[y][1])
        return None

    nV = [[list(V[j][i]) if i in (0, nx) else [] for i in range(nx + 1)] for j in range(ny)]
    res = {}
    for j in range(ny):
        for i in range(1, nx):
            cross = []
            for p in (i - 1, i):
                ms, segs = _boundary(c, cc, H, V, p, j)
                for a, b in segs:
                    ra, rb = ref(p, j, ms[a][0], ms[a][1]), ref(p, j, ms[b][0], ms[b][1])
                    A, B = pos(*ra, i, j), pos(*rb, i, j)
                    # "left of line i" decided on the offsets, as the one-marker oracle does
                    la = (sp[ra[1:]] if ra[0] == 0 else dv[ra[1:]]) < float(i - ra[1])
                    lb = (sp[rb[1:]] if rb[0] == 0 else dv[rb[1:]]) < float(i - rb[1])
                    if la == lb:
                        continue
                    if not la:
                        ra, rb, A, B, a, b = rb, ra, B, A, b, a
                    X2, Y2, X3, Y3 = A[0], A[1], B[0], B[1]
                    y = Y2 + (Y3 - Y2) * (0.0 - X2) / (X3 - X2)
                    y = min(max(y, 0.0), 1.0)
                    cross.append((y, len(cross), p, ms[a], ms[b], ra, rb, (X2, Y2), (X3, Y3)))
            assert len(cross) % 2 == int(nc[j, i] != nc[j + 1, i]), "crossing parity"
            K = _keep(cross, lambda e: (e[0], e[1]), lambda e: e[0], delta)
            if len(cross) == 3:
                stats["three_crossings"] += 1
            stats["annihilated_unaligned"] += len(cross) - len(K)
            ys, results = [], []
            for ysl, _, p, m2, m3, r2, r3, P2, P3 in K:
                m1 = partner(p, j, m2[0], m2[1])
                m4 = partner(p, j, m3[0], m3[1])
                if P3[0] == 0.0:
                    y = P3[1]
                else:
                    got = []
                    if m1 is not None:
                        X1, Y1 = pos(*m1, i, j)
                        rA = _circle_root(X1, Y1, P2[0], P2[1], P3[0], P3[1], X1, Y1, P2[0], P2[1], P3[0], P3[1], ysl)
                        if rA is not None:
                            got.append(rA)
                    if m4 is not None:
                        X4, Y4 = pos(*m4, i, j)
                        rB = _circle_root(P2[0], P2[1], P3[0], P3[1], X4, Y4, X4, Y4, P2[0], P2[1], P3[0], P3[1], ysl)
                        if rB is not None:
                            got.append(rB)
                    y = (got[0] + got[1]) * 0.5 if len(got) == 2 else (got[0] if got else ysl)
                ys.append(y)

                def rule(first, second, cell):
                    for m in [first] + ([second] if first[0] == 1 and second is not None else []):
                        if m is None or m[0] != 0:
                            continue
                        _, mi, mj, mk = m
                        if mj in (j, j + 1) and kept.get((mi, mj, mk)) == cell:
                            return 1 - int(nc[mj, i])
                    return -1

                results.append((rule(r3, m4, i), rule(r2, m1, i - 1)))
            nV[j][i] = sorted(ys)
            res[(i, j)] = results

    ncc = cc.copy()
    for j in range(ny):
        for i in range(nx):
            left = [r for r, _ in res.get((i, j), []) if r >= 0]
            right = [r for _, r in res.get((i + 1, j), []) if r >= 0]
            if left:
                ncc[j, i] = left[0]
            elif right:
                ncc[j, i] = right[0]
    return Film(nx, ny, f.h, nc, ncc, nH, nV, f.step)


def new_stats():
    return {"annihilated": 0, "annihilated_unaligned": 0, "three_crossings": 0}


def sweep(f: Film, u, v, dt, direction, delta, stats=None):
    """One sweep of a film state: direction 0 along x with u, 1 along y with v
    (the grid transposed). Raises ValueError on a CFL or domain violation."""
    stats = new_stats() if stats is None else stats
    lam = dt / f.h
    if direction == 0:
        return sweep_x(f, u, lam, delta, stats)
    t = sweep_x(f.transposed(), np.ascontiguousarray(np.asarray(v).T), lam, delta, stats)
    return t.transposed()


def step(f: Film, u, v, dt, delta, stats=None):
    """One step: x then y on even steps, y then x on odd ones (the one-marker
    oracle's order)."""
    first = 0 if f.step % 2 == 0 else 1
    g = sweep(f, u, v, dt, first, delta, stats)
    g = sweep(g, u, v, dt, 1 - first, delta, stats)
    g.step = f.step + 1
    return g


def _polygon_area(pts):
    a = 0.0
    for k in range(len(pts)):
        x0, y0 = pts[k]
        x1, y1 = pts[(k + 1) % len(pts)]
        a += x0 * y1 - x1 * y0
    return 0.5 * a


def _tau(e, o):
    """Counter-clockwise boundary coordinate of a point on edge e at offset o
    (corners BR, TR, TL, BL at 1, 2, 3, 4 = 0)."""
    return {0: o, 1: 1.0 + o, 2: 3.0 - o, 3: 4.0 - o}[e]


def _point(tau):
    tau = tau % 4.0
    if tau <= 1.0:
        return (tau, 0.0)
    if tau <= 2.0:
        return (1.0, tau - 1.0)
    if tau <= 3.0:
        return (3.0 - tau, 1.0)
    return (0.0, 4.0 - tau)


def fraction(f: Film):
    """Colour-1 area of every cell (cell units). Each segment cuts off the
    boundary arc between two consecutive markers; that region is the polygon
    of the arc (the marker, the corners passed, the next marker) closed by the
    chord. C = 1 minus the colour-0 regions if cc = 1, the sum of the colour-1
    regions if cc = 0; marker-free cells take the corners' colour."""
    nx, ny = f.nx, f.ny
    C = np.zeros((ny, nx))
    for q in range(ny):
        for p in range(nx):
            ms, segs = _boundary(f.c, f.cc, f.H, f.V, p, q)
            if not ms:
                C[q, p] = float(f.c[q, p])
                continue
            cut = 0.0
            for a, b in segs:
                ta, tb = _tau(ms[a][0], ms[a][2]), _tau(ms[b][0], ms[b][2])
                if tb < ta:
                    tb += 4.0
                pts = [_point(ta)] + [_point(k) for k in (1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0) if ta < k < tb]
                pts.append(_point(tb))
                cut += abs(_polygon_area(pts))
            C[q, p] = 1.0 - cut if int(f.cc[q, p]) == 1 else cut
    return C


def to_arrays(f: Film):
    """Offsets as (first, second) arrays with NaN where absent, for comparisons."""
    h1 = np.full((f.ny + 1, f.nx), np.nan)
    h2 = np.full((f.ny + 1, f.nx), np.nan)
    v1 = np.full((f.ny, f.nx + 1), np.nan)
    v2 = np.full((f.ny, f.nx + 1), np.nan)
    for j in range(f.ny + 1):
        for i in range(f.nx):
            for k, o in enumerate(f.H[j][i]):
                (h1 if k == 0 else h2)[j, i] = o
    for j in range(f.ny):
        for i in range(f.nx + 1):
            for k, o in enumerate(f.V[j][i]):
                (v1 if k == 0 else v2)[j, i] = o
    return h1, h2, v1, v2
