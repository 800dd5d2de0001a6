// EBIT interface step: gfx950 kernels.
//
// Layout in HBM (one grid): node colours and centre colours as bytes, marker
// offsets as FP64 structure-of-arrays (hoff, voff), each twice (ping-pong: a
// sweep reads one copy and writes the other). The grid is cut into 16x16-cell
// tiles; a tile "has" markers if one of the edges it owns carries one, and is
// "near" if it or one of its 8 neighbours has markers. Only tiles near the
// interface (this sweep or the previous one, so both copies stay coherent) are
// swept; only near tiles do the polygon/height-function work; all other cells
// get the tile's uniform colour as C and 0 as curvature in a pure write stream.
//
// Each output (a node colour, an edge offset, a centre colour) is a function
// of the old state in a small neighbourhood, so a sweep is a gather: no
// atomics on state, no ordering between tiles, results independent of the
// schedule. Every FP64 expression is written in one fixed order and the file
// is compiled with -ffp-contract=off.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ebit_internal.h"

namespace ebit {

__device__ __forceinline__ double lerp(double a, double b, double t) { return a + t * (b - a); }

// ---------------------------------------------------------------------------
// Frame of one sweep: "a" runs along the sweep direction, "b" across it.
// DIR 0 (x sweep): (a,b) = (i,j), aligned edges are H, unaligned edges are V,
// the velocity is u. DIR 1 (y sweep): (a,b) = (j,i), aligned V, unaligned H, v.
// ---------------------------------------------------------------------------
template <int DIR>
struct Frame {
  int nx, ny, na, nb;
  double lam;
  const uint8_t *__restrict__ col;
  const uint8_t *__restrict__ cen;
  const double *__restrict__ alo;  // old aligned offsets
  const double *__restrict__ uno;  // old unaligned offsets
  const double *__restrict__ vel;

  __device__ Frame(const SweepParams &p) {
    nx = p.nx;
    ny = p.ny;
    na = DIR == 0 ? p.nx : p.ny;
    nb = DIR == 0 ? p.ny : p.nx;
    lam = p.lam;
    col = p.col;
    cen = p.cen;
    alo = DIR == 0 ? p.hoff : p.voff;
    uno = DIR == 0 ? p.voff : p.hoff;
    vel = p.vel;
  }
  __device__ size_t node(int a, int b) const {
    return DIR == 0 ? (size_t)b * (nx + 1) + a : (size_t)a * (nx + 1) + b;
  }
  __device__ size_t ale(int a, int b) const { return DIR == 0 ? (size_t)b * nx + a : (size_t)a * (nx + 1) + b; }
  __device__ size_t une(int a, int b) const { return DIR == 0 ? (size_t)b * (nx + 1) + a : (size_t)a * nx + b; }
  __device__ size_t cell(int a, int b) const { return DIR == 0 ? (size_t)b * nx + a : (size_t)a * nx + b; }

  __device__ int C(int a, int b) const { return col[node(a, b)]; }
  // aligned edge (a,b), 0 <= a < na, 0 <= b <= nb
  __device__ bool presA(int a, int b) const { return C(a, b) != C(a + 1, b); }
  // unaligned edge (a,b), 0 <= a <= na, 0 <= b < nb
  __device__ bool presU(int a, int b) const { return C(a, b) != C(a, b + 1); }

  // face velocity with ghost rows mirrored across the walls
  __device__ double V(int a, int r) const {
    r = r < 0 ? 0 : (r > nb - 1 ? nb - 1 : r);
    return vel[une(a, r)];
  }
  // explicit Euler displacement of an aligned marker, bilinear velocity
  __device__ double dispA(int a, int b, double s) const {
    double ub = lerp(lerp(V(a, b - 1), V(a + 1, b - 1), s), lerp(V(a, b), V(a + 1, b), s), 0.5);
    return ub * lam;
  }
  __device__ double sp(int a, int b) const {
    double s = alo[ale(a, b)];
    return s + dispA(a, b, s);
  }
  // displacement of an unaligned marker (gray point), before the wall rule
  __device__ double rawDispU(int a, int b) const {
    double t = uno[une(a, b)];
    double ub = t < 0.5 ? lerp(V(a, b - 1), V(a, b), t + 0.5) : lerp(V(a, b), V(a, b + 1), t - 0.5);
    return ub * lam;
  }
  __device__ double dispU(int a, int b) const { return (a == 0 || a == na) ? 0.0 : rawDispU(a, b); }

  // new corner colour: flipped by each aligned marker that crosses the node
  __device__ int newC(int a, int b) const {
    int c = C(a, b);
    if (a > 0 && a < na) {
      if (presA(a - 1, b) && sp(a - 1, b) >= 1.0) c ^= 1;
      if (presA(a, b) && sp(a, b) < 0.0) c ^= 1;
    }
    return c;
  }

  // aligned markers landing on edge (a,b); returns their number and the kept
  // source (-1 when none): one lander is kept, of three the middle source.
  __device__ int landers(int a, int b, int *keep) const {
    int src[3];
    int n = 0;
    if (a >= 1 && presA(a - 1, b) && sp(a - 1, b) >= 1.0) src[n++] = a - 1;
    if (presA(a, b)) {
      double s = sp(a, b);
      if (s >= 0.0 && s < 1.0) src[n++] = a;
    }
    if (a + 1 < na && presA(a + 1, b) && sp(a + 1, b) < 0.0) src[n++] = a + 1;
    *keep = n == 1 ? src[0] : (n == 3 ? src[1] : -1);
    return n;
  }
  // the edge an aligned marker lands on (-1 if it leaves the grid)
  __device__ int landTarget(int p, int q) const {
    double s = sp(p, q);
    int t = s >= 1.0 ? p + 1 : (s < 0.0 ? p - 1 : p);
    return (t < 0 || t >= na) ? -1 : t;
  }
  __device__ bool keptOn(int p, int q, int target) const {
    if (landTarget(p, q) != target) return false;
    int keep;
    landers(target, q, &keep);
    return keep == p;
  }

  // old segments of cell (p,q): edge pairs (0 bottom, 1 right, 2 top, 3 left)
  __device__ int segments(int p, int q, int8_t s[4]) const {
    int k0 = C(p, q), k1 = C(p + 1, q), k2 = C(p + 1, q + 1), k3 = C(p, q + 1);
    bool e0 = k0 != k1, e1 = k1 != k2, e2 = k3 != k2, e3 = k0 != k3;
    int n = (int)e0 + (int)e1 + (int)e2 + (int)e3;
    s[0] = s[1] = s[2] = s[3] = -1;
    if (n == 2) {
      int w = 0;
      if (e0) s[w++] = 0;
      if (e1) s[w++] = 1;
      if (e2) s[w++] = 2;
      if (e3) s[w++] = 3;
      return 1;
    }
    if (n == 4) {
      int cc = cen[cell(p, q)];
      int kk[4] = {k0, k1, k2, k3};
      int w = 0;
      for (int corner = 0; corner < 4; corner++)
        if (kk[corner] != cc) {
          s[w++] = (int8_t)((corner + 3) & 3);
          s[w++] = (int8_t)corner;
        }
      return 2;
    }
    return 0;
  }
};

struct MRef {
  int8_t kind;  // 0 aligned, 1 unaligned
  int a, b;
};

__device__ __forceinline__ MRef edgeMarker(int p, int q, int e) {
  MRef m;
  if (e == 0) { m.kind = 0; m.a = p; m.b = q; }
  else if (e == 1) { m.kind = 1; m.a = p + 1; m.b = q; }
  else if (e == 2) { m.kind = 0; m.a = p; m.b = q + 1; }
  else { m.kind = 1; m.a = p; m.b = q; }
  return m;
}

template <int DIR>
__device__ __forceinline__ void advPoint(const Frame<DIR> &F, MRef m, int a0, int b0, double *X, double *Y) {
  if (m.kind == 0) {
    *X = (double)(m.a - a0) + F.sp(m.a, m.b);
    *Y = (double)(m.b - b0);
  } else {
    *X = (double)(m.a - a0) + F.dispU(m.a, m.b);
    *Y = (double)(m.b - b0) + F.uno[F.une(m.a, m.b)];
  }
}

template <int DIR>
__device__ __forceinline__ bool leftOf(const Frame<DIR> &F, MRef m, int a0) {
  if (m.kind == 0) return F.sp(m.a, m.b) < (double)(a0 - m.a);
  return F.dispU(m.a, m.b) < (double)(a0 - m.a);
}

// chain neighbour of the marker on edge e of old cell (p,q), away from it
template <int DIR>
__device__ bool chainNb(const Frame<DIR> &F, int p, int q, int e, MRef *out) {
  int pp = p, qq = q;
  if (e == 0) qq = q - 1;
  else if (e == 1) pp = p + 1;
  else if (e == 2) qq = q + 1;
  else pp = p - 1;
  if (pp < 0 || pp >= F.na || qq < 0 || qq >= F.nb) return false;
  int eo = (e + 2) & 3;
  int8_t s[4];
  F.segments(pp, qq, s);
  for (int k = 0; k < 4; k += 2) {
    if (s[k] < 0) continue;
    if (s[k] == eo) { *out = edgeMarker(pp, qq, s[k + 1]); return true; }
    if (s[k + 1] == eo) { *out = edgeMarker(pp, qq, s[k]); return true; }
  }
  return false;
}

// Circle through three points as a(X^2+Y^2) + bX + cY + e = 0, intersected
// with X = 0; keeps the root across chord P2P3 from the outer point.
__device__ bool circleRoot(double Xa, double Ya, double Xb, double Yb, double Xc, double Yc, double Xo, double Yo,
                           double X2, double Y2, double X3, double Y3, double ysl, double *root, uint32_t *ties,
                           uint32_t *rejects) {
  double Qa = Xa * Xa + Ya * Ya;
  double Qb = Xb * Xb + Yb * Yb;
  double Qc = Xc * Xc + Yc * Yc;
  double ca = Xa * (Yb - Yc) + Xb * (Yc - Ya) + Xc * (Ya - Yb);
  double cc = Qa * (Xb - Xc) + Qb * (Xc - Xa) + Qc * (Xa - Xb);
  double ce = -(Qa * (Xb * Yc - Xc * Yb) + Qb * (Xc * Ya - Xa * Yc) + Qc * (Xa * Yb - Xb * Ya));
  double r;
  if (ca == 0.0) {
    if (cc == 0.0) return false;
    r = -ce / cc;
  } else {
    double disc = cc * cc - 4.0 * ca * ce;
    if (disc < 0.0) disc = 0.0;
    double sq = sqrt(disc);
    double q = -0.5 * (cc + (cc >= 0.0 ? sq : -sq));
    double r1, r2;
    if (q == 0.0) {
      r1 = 0.0;
      r2 = 0.0;
    } else {
      r1 = q / ca;
      r2 = ce / q;
    }
    double DX = X3 - X2, DY = Y3 - Y2;
    double L2 = DX * DX + DY * DY;
    double so = DX * (Yo - Y2) - DY * (Xo - X2);
    double s1 = DX * (r1 - Y2) - DY * (0.0 - X2);
    double s2 = DX * (r2 - Y2) - DY * (0.0 - X2);
    if (fabs(s1) < TIE_EPS * L2 || fabs(s2) < TIE_EPS * L2) (*ties)++;
    bool q1 = (s1 > 0.0 && so < 0.0) || (s1 < 0.0 && so > 0.0);
    bool q2 = (s2 > 0.0 && so < 0.0) || (s2 < 0.0 && so > 0.0);
    if (q1 && !q2) r = r1;
    else if (q2 && !q1) r = r2;
    else r = (fabs(r1 - ysl) <= fabs(r2 - ysl)) ? r1 : r2;
  }
  if (!(r >= 0.0 && r <= 1.0)) {
    (*rejects)++;
    return false;
  }
  *root = r;
  return true;
}

__device__ __forceinline__ double chordY(double X2, double Y2, double X3, double Y3) {
  double y = Y2 + (Y3 - Y2) * (0.0 - X2) / (X3 - X2);
  if (y < 0.0) y = 0.0;
  if (y > 1.0) y = 1.0;
  return y;
}

// Block-local counters, flushed once per block.
struct BlockCounters {
  uint32_t v[NCOUNTERS];
};

// New unaligned marker on line a (interior), row b: returns 1 and its offset
// when present; fills the centre-CV results for the cell to the right of the
// line (cell a) and to its left (cell a-1): -1 or the new centre colour.
template <int DIR>
__device__ bool newUnaligned(const Frame<DIR> &F, int a, int b, double *yout, int *resRight, int *resLeft,
                             uint32_t *cnt, bool count) {
  *resRight = -1;
  *resLeft = -1;
  uint32_t lties = 0, lrej = 0;
  int cp[4];
  int8_t cl[4], cr[4];
  double X2v[4], Y2v[4], X3v[4], Y3v[4], ysl[4];
  int nxr = 0;
  for (int p = a - 1; p <= a; p++) {
    int8_t s[4];
    F.segments(p, b, s);
    for (int k = 0; k < 4; k += 2) {
      if (s[k] < 0) continue;
      MRef m1 = edgeMarker(p, b, s[k]), m2 = edgeMarker(p, b, s[k + 1]);
      bool l1 = leftOf(F, m1, a), l2 = leftOf(F, m2, a);
      if (l1 == l2) continue;
      cp[nxr] = p;
      cl[nxr] = l1 ? s[k] : s[k + 1];
      cr[nxr] = l1 ? s[k + 1] : s[k];
      advPoint(F, edgeMarker(p, b, cl[nxr]), a, b, &X2v[nxr], &Y2v[nxr]);
      advPoint(F, edgeMarker(p, b, cr[nxr]), a, b, &X3v[nxr], &Y3v[nxr]);
      ysl[nxr] = chordY(X2v[nxr], Y2v[nxr], X3v[nxr], Y3v[nxr]);
      nxr++;
    }
  }
  int pick = -1;
  if (nxr == 1) {
    pick = 0;
  } else if (nxr == 3) {
    if (count) cnt[C_THREE_CROSSINGS]++;
    for (int x = 0; x < 3 && pick < 0; x++) {
      int below = 0;
      for (int y = 0; y < 3; y++) {
        if (y == x) continue;
        if (ysl[y] < ysl[x] || (ysl[y] == ysl[x] && y < x)) below++;
      }
      if (below == 1) pick = x;
    }
    for (int x = 0; x < 3; x++)
      for (int y = x + 1; y < 3; y++)
        if (fabs(ysl[x] - ysl[y]) < TIE_EPS) lties++;
  }
  if (pick < 0) {
    if (count) {
      cnt[C_PARITY_FALLBACK]++;
      cnt[C_TIES] += lties;
    }
    *yout = 0.5;
    return true;
  }
  double X2 = X2v[pick], Y2 = Y2v[pick], X3 = X3v[pick], Y3 = Y3v[pick];
  if (fabs(X2) < TIE_EPS || fabs(X3) < TIE_EPS) lties++;
  int p = cp[pick];
  MRef m2 = edgeMarker(p, b, cl[pick]), m3 = edgeMarker(p, b, cr[pick]), m1, m4;
  bool h1 = chainNb(F, p, b, cl[pick], &m1);
  bool h4 = chainNb(F, p, b, cr[pick], &m4);
  double y;
  uint32_t fb = 0;
  if (X3 == 0.0) {
    y = Y3;
  } else {
    double X1 = 0, Y1 = 0, X4 = 0, Y4 = 0, rA = 0, rB = 0;
    bool okA = false, okB = false;
    if (h1) {
      advPoint(F, m1, a, b, &X1, &Y1);
      okA = circleRoot(X1, Y1, X2, Y2, X3, Y3, X1, Y1, X2, Y2, X3, Y3, ysl[pick], &rA, &lties, &lrej);
    }
    if (h4) {
      advPoint(F, m4, a, b, &X4, &Y4);
      okB = circleRoot(X2, Y2, X3, Y3, X4, Y4, X4, Y4, X2, Y2, X3, Y3, ysl[pick], &rB, &lties, &lrej);
    }
    if (okA && okB) y = (rA + rB) * 0.5;
    else if (okA) y = rA;
    else if (okB) y = rB;
    else {
      y = ysl[pick];
      fb = 1;
    }
  }
  if (y < TIE_EPS || 1.0 - y < TIE_EPS) lties++;
  if (count) {
    cnt[C_TIES] += lties;
    cnt[C_FIT_REJECT] += lrej;
    cnt[C_FIT_FALLBACK] += fb;
  }
  *yout = y;

  // Centre-CV candidates: for the cell right of the line, the crossing
  // endpoint on its side (P3) and, if that is an unaligned point, its chain
  // neighbour (P4); for the cell on the left, P2 then P1. A candidate counts
  // when it is an aligned marker kept on that cell's bottom or top edge; the
  // corner it shares with this line is then isolated.
  for (int side = 0; side < 2; side++) {
    int cellA = side == 0 ? a : a - 1;
    if (cellA < 0 || cellA >= F.na) continue;
    MRef cand[2];
    int nc = 0;
    MRef first = side == 0 ? m3 : m2;
    cand[nc++] = first;
    if (first.kind == 1) {
      if (side == 0 && h4) cand[nc++] = m4;
      if (side == 1 && h1) cand[nc++] = m1;
    }
    for (int k = 0; k < nc; k++) {
      MRef m = cand[k];
      if (m.kind != 0) continue;
      if (m.b != b && m.b != b + 1) continue;
      if (!F.keptOn(m.a, m.b, cellA)) continue;
      int corner = F.newC(a, m.b);
      int res = 1 - corner;
      if (side == 0) *resRight = res;
      else *resLeft = res;
      break;
    }
  }
  return true;
}

// ---------------------------------------------------------------------------
// Sweep kernel: one workgroup per active tile (persistent over the list).
// ---------------------------------------------------------------------------
template <int DIR>
__global__ __launch_bounds__(256) void k_sweep(SweepParams P) {
  const Frame<DIR> F(P);
  __shared__ int8_t sRight[TS][TS + 1];  // [lb][la] result for cell right of line
  __shared__ int8_t sLeft[TS][TS + 1];   // result for cell left of line
  __shared__ uint32_t sCnt[NCOUNTERS];
  __shared__ int sHas;
  __shared__ uint32_t sErr;
  const int tid = threadIdx.x;
  if (tid < NCOUNTERS) sCnt[tid] = 0;
  if (tid == 0) sErr = 0;
  uint32_t cnt[NCOUNTERS];
#pragma unroll
  for (int k = 0; k < NCOUNTERS; k++) cnt[k] = 0;
  uint32_t err = 0;
  const uint32_t ntile = *P.count;
  for (uint32_t it = blockIdx.x; it < ntile; it += gridDim.x) {
    const uint32_t T = P.list[it];
    const int tx = (int)(T % (uint32_t)P.ntx), ty = (int)(T / (uint32_t)P.ntx);
    const int x0 = tx * TS, y0 = ty * TS;
    const int a0 = DIR == 0 ? x0 : y0, b0 = DIR == 0 ? y0 : x0;
    __syncthreads();
    if (tid == 0) sHas = 0;
    __syncthreads();
    int has = 0;
    // phase 1: nodes, aligned edges, unaligned edges on lines a0..a0+TS
    for (int k = tid; k < (TS + 1) * (TS + 1); k += blockDim.x) {
      const int li = k % (TS + 1), lj = k / (TS + 1);
      const int la = DIR == 0 ? li : lj, lb = DIR == 0 ? lj : li;
      const int a = a0 + la, b = b0 + lb;
      if (a > F.na || b > F.nb) continue;
      const bool ownA = la < TS || a == F.na;
      const bool ownB = lb < TS || b == F.nb;
      // node
      if (ownA && ownB) {
        int c = F.newC(a, b);
        size_t idx = F.node(a, b);
        P.ncol[idx] = (uint8_t)c;
      }
      // aligned edge (a,b)
      if (a < F.na && la < TS && ownB) {
        if (F.presA(a, b)) {
          cnt[C_MARKERS]++;
          double s = F.alo[F.ale(a, b)];
          double d = F.dispA(a, b, s);
          if (fabs(d) > 0.5) err |= ERRBIT_CFL;
          double spv = s + d;
          if ((spv >= 1.0 && a + 1 >= F.na) || (spv < 0.0 && a == 0)) err |= ERRBIT_DOMAIN;
        }
        int keep;
        int n = F.landers(a, b, &keep);
        if (n == 3) cnt[C_THREE_LANDERS]++;
        cnt[C_ANNIHILATED] += (uint32_t)(n - (n & 1));
        const int newpres = F.newC(a, b) != F.newC(a + 1, b);
        if (newpres != (n & 1)) cnt[C_INVARIANT_FAIL]++;
        if (keep >= 0) {
          double spv = F.sp(keep, b);
          double o = keep < a ? spv - 1.0 : (keep > a ? spv + 1.0 : spv);
          if (o < TIE_EPS || 1.0 - o < TIE_EPS) cnt[C_TIES]++;
          if (newpres) (DIR == 0 ? P.nhoff : P.nvoff)[F.ale(a, b)] = o;
        } else if (newpres) {
          (DIR == 0 ? P.nhoff : P.nvoff)[F.ale(a, b)] = 0.0;
        }
        if (newpres) has = 1;
      }
      // unaligned edge (a,b)
      if (b < F.nb && lb < TS) {
        const bool own = ownA;
        if (own && F.presU(a, b)) {
          cnt[C_MARKERS]++;
          double d = F.rawDispU(a, b);
          if (fabs(d) > 0.5) err |= ERRBIT_CFL;
          if ((a == 0 || a == F.na) && d != 0.0) cnt[C_WALL_VIOLATION]++;
        }
        int rR = -1, rL = -1;
        double *dst = DIR == 0 ? P.nvoff : P.nhoff;
        if (a == 0 || a == F.na) {
          // walls hold their markers (colours of wall nodes never change)
          if (own && F.presU(a, b)) {
            dst[F.une(a, b)] = F.uno[F.une(a, b)];
            has = 1;
          }
        } else if (F.newC(a, b) != F.newC(a, b + 1)) {
          double y;
          newUnaligned(F, a, b, &y, &rR, &rL, cnt, own);
          if (own) {
            dst[F.une(a, b)] = y;
            has = 1;
          }
        }
        sRight[lb][la] = (int8_t)rR;
        sLeft[lb][la] = (int8_t)rL;
      }
    }
    __syncthreads();
    // phase 2: centre colours of the tile's cells
    for (int k = tid; k < TS * TS; k += blockDim.x) {
      const int li = k % TS, lj = k / TS;
      const int la = DIR == 0 ? li : lj, lb = DIR == 0 ? lj : li;
      const int a = a0 + la, b = b0 + lb;
      if (a >= F.na || b >= F.nb) continue;
      int left = sRight[lb][la];       // line a, cell to its right
      int right = sLeft[lb][la + 1];   // line a+1, cell to its left
      int cc = F.cen[F.cell(a, b)];
      if (left >= 0) {
        cc = left;
        cnt[C_CV_SET]++;
        if (right >= 0 && right != left) cnt[C_CV_CONFLICT]++;
      } else if (right >= 0) {
        cc = right;
        cnt[C_CV_SET]++;
      } else {
        int k0 = F.newC(a, b), k1 = F.newC(a + 1, b), k2 = F.newC(a + 1, b + 1), k3 = F.newC(a, b + 1);
        if ((k0 != k1) + (k1 != k2) + (k3 != k2) + (k0 != k3) == 4) cnt[C_CV_UNRESOLVED]++;
      }
      P.ncen[F.cell(a, b)] = (uint8_t)cc;
    }
    if (has) sHas = 1;
    __syncthreads();
    if (tid == 0) P.has[T] = (uint8_t)sHas;
  }
  // flush counters
  for (int k = 0; k < NCOUNTERS; k++)
    if (cnt[k]) atomicAdd(&sCnt[k], cnt[k]);
  if (err) atomicOr(&sErr, err);
  __syncthreads();
  if (tid < NCOUNTERS && sCnt[tid]) atomicAdd(&P.ctr[tid], (unsigned long long)sCnt[tid]);
  if (tid == 0 && sErr) atomicOr(P.err, sErr);
}

// ---------------------------------------------------------------------------
// Tile bookkeeping: marker flags of the uploaded state, then per-sweep
// compaction into the active list (near now or near last sweep) and the near
// list, with wave ballots and one atomic per wave.
// ---------------------------------------------------------------------------
__global__ void k_init_has(const uint8_t *__restrict__ col, int nx, int ny, int ntx, int nty, uint8_t *has,
                           uint8_t *nearPrev) {
  const int T = blockIdx.x;
  if (T >= ntx * nty) return;
  const int tx = T % ntx, ty = T / ntx;
  const int x0 = tx * TS, y0 = ty * TS;
  __shared__ int sh;
  if (threadIdx.x == 0) sh = 0;
  __syncthreads();
  int h = 0;
  for (int k = threadIdx.x; k < (TS + 1) * (TS + 1); k += blockDim.x) {
    const int li = k % (TS + 1), lj = k / (TS + 1);
    const int i = x0 + li, j = y0 + lj;
    if (i > nx || j > ny) continue;
    const bool ownI = li < TS || i == nx;
    const bool ownJ = lj < TS || j == ny;
    const uint8_t c = col[(size_t)j * (nx + 1) + i];
    if (i < nx && li < TS && ownJ && c != col[(size_t)j * (nx + 1) + i + 1]) h = 1;
    if (j < ny && lj < TS && ownI && c != col[(size_t)(j + 1) * (nx + 1) + i]) h = 1;
  }
  if (h) sh = 1;
  __syncthreads();
  if (threadIdx.x == 0) {
    has[T] = (uint8_t)sh;
    nearPrev[T] = 0;
  }
}

__global__ void k_compact(const uint8_t *__restrict__ has, uint8_t *__restrict__ nearPrev,
                          uint8_t *__restrict__ tinfo, const uint8_t *__restrict__ col, int nx, int ntx, int nty,
                          uint32_t *actList, uint32_t *nearList, uint32_t *counts, int slot) {
  const int ntiles = ntx * nty;
  const int T = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // clear the other slot for the next compaction (nothing reads it now)
    counts[2 * (slot ^ 1)] = 0;
    counts[2 * (slot ^ 1) + 1] = 0;
  }
  bool act = false, nr = false;
  if (T < ntiles) {
    const int tx = T % ntx, ty = T / ntx;
    int n = 0;
    for (int oy = -1; oy <= 1; oy++)
      for (int ox = -1; ox <= 1; ox++) {
        const int sx = tx + ox, sy = ty + oy;
        if (sx < 0 || sy < 0 || sx >= ntx || sy >= nty) continue;
        n |= has[sy * ntx + sx];
      }
    nr = n != 0;
    act = nr || nearPrev[T] != 0;
    nearPrev[T] = (uint8_t)nr;
    tinfo[T] = (uint8_t)((nr ? 1 : 0) | (col[(size_t)(ty * TS) * (nx + 1) + tx * TS] << 1));
  }
  // wave-level compaction: ballot + popcount + mbcnt prefix
  const uint64_t ba = __ballot(act);
  const uint64_t bn = __ballot(nr);
  const int lane = threadIdx.x & 63;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  uint32_t baseA = 0, baseN = 0;
  if (lane == 0) {
    if (ba) baseA = atomicAdd(&counts[2 * slot], (uint32_t)__popcll(ba));
    if (bn) baseN = atomicAdd(&counts[2 * slot + 1], (uint32_t)__popcll(bn));
  }
  baseA = __shfl(baseA, 0);
  baseN = __shfl(baseN, 0);
  if (act) actList[baseA + __popcll(ba & below)] = (uint32_t)T;
  if (nr) nearList[baseN + __popcll(bn & below)] = (uint32_t)T;
}

// ---------------------------------------------------------------------------
// Volume fraction and height-function curvature.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int mirrorCell(int k, int n) { return k < 0 ? -1 - k : (k >= n ? 2 * n - 1 - k : k); }
// halo slots farther than one reflection (grids narrower than the halo) are
// clamped into the grid; the stencils never read them
__device__ __forceinline__ int haloCell(int k, int n) {
  k = mirrorCell(k, n);
  return k < 0 ? 0 : (k >= n ? n - 1 : k);
}
__device__ __forceinline__ int mirrorNode(int k, int n) { return k < 0 ? -k : (k > n ? 2 * n - k : k); }

// area of colour 1 in cell (i,j); also its marker count and BL colour
__device__ double cellFraction(const FracParams &P, int i, int j, int *nmark, int *cbl) {
  const size_t W1 = (size_t)P.nx + 1;
  const int kBL = P.col[(size_t)j * W1 + i], kBR = P.col[(size_t)j * W1 + i + 1];
  const int kTR = P.col[(size_t)(j + 1) * W1 + i + 1], kTL = P.col[(size_t)(j + 1) * W1 + i];
  const bool pb = kBL != kBR, pr = kBR != kTR, pt = kTL != kTR, pl = kBL != kTL;
  const int n = (int)pb + (int)pr + (int)pt + (int)pl;
  *nmark = n;
  *cbl = kBL;
  if (n == 0) return (double)kBL;
  const double hb = pb ? P.hoff[(size_t)j * P.nx + i] : 0.0;
  const double ht = pt ? P.hoff[(size_t)(j + 1) * P.nx + i] : 0.0;
  const double vl = pl ? P.voff[(size_t)j * W1 + i] : 0.0;
  const double vr = pr ? P.voff[(size_t)j * W1 + i + 1] : 0.0;
  if (n == 2) {
    // shoelace over the colour-1 corners and both markers, counter-clockwise
    double px[6], py[6];
    int m = 0;
    if (kBL) { px[m] = 0.0; py[m] = 0.0; m++; }
    if (pb) { px[m] = hb; py[m] = 0.0; m++; }
    if (kBR) { px[m] = 1.0; py[m] = 0.0; m++; }
    if (pr) { px[m] = 1.0; py[m] = vr; m++; }
    if (kTR) { px[m] = 1.0; py[m] = 1.0; m++; }
    if (pt) { px[m] = ht; py[m] = 1.0; m++; }
    if (kTL) { px[m] = 0.0; py[m] = 1.0; m++; }
    if (pl) { px[m] = 0.0; py[m] = vl; m++; }
    double acc = 0.0;
    for (int k = 0; k < m; k++) {
      const int k1 = (k + 1 == m) ? 0 : k + 1;
      acc += px[k] * py[k1] - px[k1] * py[k];
    }
    return 0.5 * acc;
  }
  // four markers: isolated corner triangles keep their corner colour, the
  // central region carries the centre colour
  const int cen = P.cen[(size_t)j * P.nx + i];
  const double tBL = 0.5 * (hb * vl), tBR = 0.5 * ((1.0 - hb) * vr);
  const double tTR = 0.5 * ((1.0 - vr) * (1.0 - ht)), tTL = 0.5 * (ht * (1.0 - vl));
  const double s = (kBL != cen) ? tBL + tTR : tBR + tTL;
  return cen ? 1.0 - s : s;
}

// Dense write of one grid row for the cells of uniform (not near) tiles:
// C = the tile's colour, K = 0. Two cells per thread; rows of even length use
// 16-byte non-temporal stores.
typedef double v2d __attribute__((ext_vector_type(2)));

template <int MODE>
__device__ __forceinline__ void fillRow(const FracParams &P, int j) {
  const uint8_t *trow = P.tinfo + (size_t)(j / TS) * P.ntx;
  const size_t rowoff = (size_t)j * P.nx;
  const int nx = P.nx;
  const bool vec = P.vec != 0;
  for (int i = 2 * (int)threadIdx.x; i < nx; i += 2 * (int)blockDim.x) {
    const uint8_t t0 = trow[i / TS];
    const bool two = i + 1 < nx;
    const uint8_t t1 = two ? trow[(i + 1) / TS] : (uint8_t)1;
    if (vec && !(t0 & 1) && !(t1 & 1)) {
      if (MODE & 1) {
        v2d c = {(double)(t0 >> 1), (double)(t1 >> 1)};
        __builtin_nontemporal_store(c, (v2d *)&P.Cout[rowoff + i]);
      }
      if (MODE & 2) {
        v2d z = {0.0, 0.0};
        __builtin_nontemporal_store(z, (v2d *)&P.Kout[rowoff + i]);
      }
      continue;
    }
    if (!(t0 & 1)) {
      if (MODE & 1) P.Cout[rowoff + i] = (double)(t0 >> 1);
      if (MODE & 2) P.Kout[rowoff + i] = 0.0;
    }
    if (two && !(t1 & 1)) {
      if (MODE & 1) P.Cout[rowoff + i + 1] = (double)(t1 >> 1);
      if (MODE & 2) P.Kout[rowoff + i + 1] = 0.0;
    }
  }
}

// Heights along columns (rows == 0) or rows (rows == 1) around cell (i,j),
// from the fraction tile in LDS; returns 1 and kappa on success.
template <class GetC, class GetN, class GetB>
__device__ bool hfTry(int i, int j, int rows, double h, GetC getC, GetN getN, GetB getB, double *kap) {
  double y[3];
  int sig = 0;
  for (int k = -1; k <= 1; k++) {
    int ei0, ej0, ei1, ej1;
    if (!rows) {
      ei0 = i + k; ej0 = j - 3;
      ei1 = i + k; ej1 = j + 3;
    } else {
      ei0 = i - 3; ej0 = j + k;
      ei1 = i + 3; ej1 = j + k;
    }
    if (getN(ei0, ej0) != 0 || getN(ei1, ej1) != 0) return false;
    const int c0 = getB(ei0, ej0), c1 = getB(ei1, ej1);
    if (c0 == c1) return false;
    const int s = c0 == 1 ? 1 : -1;
    if (sig == 0) sig = s;
    else if (sig != s) return false;
    double S = 0.0;
    for (int m = -3; m <= 3; m++) S += rows ? getC(i + m, j + k) : getC(i + k, j + m);
    y[k + 1] = sig == 1 ? S - 3.0 : 4.0 - S;
  }
  const double hx = (y[2] - y[0]) * 0.5;
  const double hxx = y[2] - 2.0 * y[1] + y[0];
  const double g = 1.0 + hx * hx;
  *kap = (-(double)sig * hxx) / (h * g * sqrt(g));
  return true;
}

// Fraction and/or curvature of the whole grid in one persistent launch.
// First the near tiles from the list: C (with marker count and BL colour) of
// the tile plus a 3-cell halo in LDS, mirrored across walls, then C and/or
// kappa of the tile's cells. Then the dense rows, where uniform tiles get
// their colour and zero curvature. MODE 1: C only; 2: kappa from the
// caller's C; 3: both.
template <int MODE>
__global__ __launch_bounds__(256) void k_frac_curv(FracParams P) {
  constexpr int W = TS + 6;
  __shared__ double sC[W][W];
  __shared__ uint8_t sN[W][W];
  __shared__ uint8_t sB[W][W];
  __shared__ uint32_t sCnt[2];
  const int tid = threadIdx.x;
  if (tid < 2) sCnt[tid] = 0;
  uint32_t interf = 0, hffail = 0;
  const uint32_t ntile = *P.count;
  for (uint32_t it = blockIdx.x; it < ntile; it += gridDim.x) {
    const uint32_t T = P.list[it];
    const int tx = (int)(T % (uint32_t)P.ntx), ty = (int)(T / (uint32_t)P.ntx);
    const int x0 = tx * TS, y0 = ty * TS;
    __syncthreads();
    for (int k = tid; k < W * W; k += blockDim.x) {
      const int li = k % W, lj = k / W;
      const int gi = haloCell(x0 - 3 + li, P.nx), gj = haloCell(y0 - 3 + lj, P.ny);
      int nm, cbl;
      double c = cellFraction(P, gi, gj, &nm, &cbl);
      if (MODE == 2) c = P.Cin[(size_t)gj * P.nx + gi];
      sC[lj][li] = c;
      sN[lj][li] = (uint8_t)nm;
      sB[lj][li] = (uint8_t)cbl;
    }
    __syncthreads();
    for (int k = tid; k < TS * TS; k += blockDim.x) {
      const int li = k % TS, lj = k / TS;
      const int i = x0 + li, j = y0 + lj;
      if (i >= P.nx || j >= P.ny) continue;
      const size_t id = (size_t)j * P.nx + i;
      if (MODE & 1) P.Cout[id] = sC[lj + 3][li + 3];
      if (MODE & 2) {
        double kap = 0.0;
        if (sN[lj + 3][li + 3] >= 2) {
          interf++;
          const uint8_t *col = P.col;
          const int nx = P.nx, ny = P.ny;
          auto nodeC = [&](int a, int b) -> int {
            return col[(size_t)mirrorNode(b, ny) * (nx + 1) + mirrorNode(a, nx)];
          };
          int ncx = 0, ncy = 0;
          for (int m = j - 1; m <= j + 2; m++)
            ncx += nodeC(i + 2, m) + nodeC(i + 1, m) - nodeC(i, m) - nodeC(i - 1, m);
          for (int l = i - 1; l <= i + 2; l++)
            ncy += nodeC(l, j + 2) + nodeC(l, j + 1) - nodeC(l, j) - nodeC(l, j - 1);
          const int firstRows = abs(ncy) >= abs(ncx) ? 0 : 1;
          auto getC = [&](int a, int b) -> double { return sC[b - y0 + 3][a - x0 + 3]; };
          auto getN = [&](int a, int b) -> int { return sN[b - y0 + 3][a - x0 + 3]; };
          auto getB = [&](int a, int b) -> int { return sB[b - y0 + 3][a - x0 + 3]; };
          if (!hfTry(i, j, firstRows, P.h, getC, getN, getB, &kap) &&
              !hfTry(i, j, 1 - firstRows, P.h, getC, getN, getB, &kap)) {
            kap = __builtin_nan("");
            hffail++;
          }
        }
        P.Kout[id] = kap;
      }
    }
  }
  for (int j = blockIdx.x; j < P.ny; j += gridDim.x) fillRow<MODE>(P, j);
  if (MODE & 2) {
    if (interf) atomicAdd(&sCnt[0], interf);
    if (hffail) atomicAdd(&sCnt[1], hffail);
    __syncthreads();
    if (tid == 0) {
      if (sCnt[0]) atomicAdd(&P.ctr[C_INTERFACIAL], (unsigned long long)sCnt[0]);
      if (sCnt[1]) atomicAdd(&P.ctr[C_HF_FAIL], (unsigned long long)sCnt[1]);
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_sweep(int dir, const SweepParams &p, int grid, hipStream_t s) {
  if (dir == 0) hipLaunchKernelGGL(k_sweep<0>, dim3(grid), dim3(256), 0, s, p);
  else hipLaunchKernelGGL(k_sweep<1>, dim3(grid), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_init_has(const uint8_t *col, int nx, int ny, int ntx, int nty, uint8_t *has, uint8_t *nearPrev,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_init_has, dim3(ntx * nty), dim3(256), 0, s, col, nx, ny, ntx, nty, has, nearPrev);
  return hipGetLastError();
}

hipError_t launch_compact(const uint8_t *has, uint8_t *nearPrev, uint8_t *tinfo, const uint8_t *col, int nx, int ntx,
                          int nty, uint32_t *actList, uint32_t *nearList, uint32_t *counts, int slot, hipStream_t s) {
  const int n = ntx * nty;
  hipLaunchKernelGGL(k_compact, dim3((n + 255) / 256), dim3(256), 0, s, has, nearPrev, tinfo, col, nx, ntx, nty,
                     actList, nearList, counts, slot);
  return hipGetLastError();
}

hipError_t launch_frac_curv(int mode, const FracParams &p, int grid, hipStream_t s) {
  if (mode == 1) hipLaunchKernelGGL(k_frac_curv<1>, dim3(grid), dim3(256), 0, s, p);
  else if (mode == 2) hipLaunchKernelGGL(k_frac_curv<2>, dim3(grid), dim3(256), 0, s, p);
  else hipLaunchKernelGGL(k_frac_curv<3>, dim3(grid), dim3(256), 0, s, p);
  return hipGetLastError();
}

}  // namespace ebit
