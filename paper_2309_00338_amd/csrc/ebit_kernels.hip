// EBIT interface step: gfx950 kernels.
//
// Layout in HBM (per grid): node colours as a bit plane in 16x16-node blocks
// (cb_word) and marker offsets as FP64 structure-of-arrays (hoff, voff), each
// twice (ping-pong: a sweep reads one copy and writes the other); centre
// colours as bytes, once (a sweep leaves
// them alone and its centre kernel rewrites the cells it settles in place). Every grid is cut into
// 16x16-cell tiles; the tiles of all grids an engine holds share one global
// index space, so one launch per phase serves any number of grids. Each tile
// keeps a small mask of where its own markers sit (anywhere, within 3 cells
// of each side, of each corner); a tile is "near" the interface when it holds
// markers or a neighbour holds markers close to their shared side or corner.
// Only tiles that are near in this sweep or were near in the previous one (so
// both copies stay coherent) are swept; only near tiles do polygon and
// height-function work; every other cell gets its tile's uniform colour as C
// and 0 as curvature in a pure write stream.
//
// A sweep is a gather: each output (node colour, edge offset, centre colour)
// is a function of the old state within two cells, so there are no atomics on
// state and no ordering between tiles. A workgroup stages its tile plus a
// 2-cell halo in LDS (node colours, advected aligned offsets), computes new
// colours and lander choices and queues the present new unaligned edges; the
// fit kernel then places them one per lane and the centre kernel sets the
// centre colours. Every FP64
// expression is written in one fixed order and the file is built with
// -ffp-contract=off.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ebit_internal.h"

namespace ebit {

__device__ __forceinline__ double lerp(double a, double b, double t) { return a + t * (b - a); }

// Pointers read from a grid descriptor are generic; accesses through them
// would be flat instructions, which also count against the LDS wait counter.
// Every per-grid array lives in device global memory, so kernels cast them.
#define GL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GL T *gp(T *p) {
  return (GL T *)p;
}

constexpr int HALO = 2;
constexpr int NH = TS + 2 * HALO + 1;  // staged nodes per side (21)
constexpr int NE = NH - 1;             // staged cells / edges per side (20)
constexpr int NN = TS + 1;             // new nodes per side (17)
constexpr int JOBCAP = 384;            // queued fit jobs per sweep workgroup (>= one tile's 256)
constexpr uint32_t NXCD = 8;          // XCDs of the GPU, each with its own L2

// marker-position mask bits of a tile: any marker; within STRIP cells of a
// side or corner; on the tile's own left / bottom border edge (shared with
// the cells of the neighbour on that side); on an edge of a cell of the
// tile's last column / top row
enum : uint16_t {
  M_ANY = 1, M_L = 2, M_R = 4, M_B = 8, M_T = 16, M_LB = 32, M_RB = 64, M_LT = 128, M_RT = 256, M_L0 = 512,
  M_B0 = 1024, M_R1 = 2048, M_T1 = 4096
};
constexpr int STRIP = 3;

// mask bits of a marker whose edge touches the local cells [lx0,lx1] x [ly0,ly1]
__device__ __forceinline__ uint16_t maskAt(int lx0, int lx1, int ly0, int ly1) {
  const bool l = lx0 < STRIP, r = lx1 >= TS - STRIP, b = ly0 < STRIP, t = ly1 >= TS - STRIP;
  uint16_t m = M_ANY;
  if (l) m |= M_L;
  if (r) m |= M_R;
  if (b) m |= M_B;
  if (t) m |= M_T;
  if (l && b) m |= M_LB;
  if (r && b) m |= M_RB;
  if (l && t) m |= M_LT;
  if (r && t) m |= M_RT;
  if (lx0 < 0) m |= M_L0;
  if (ly0 < 0) m |= M_B0;
  if (lx1 >= TS - 1) m |= M_R1;
  if (ly1 >= TS - 1) m |= M_T1;
  return m;
}
// mask of an H edge (i,j) / V edge (i,j) in the tile with origin (x0,y0)
__device__ __forceinline__ uint16_t maskH(int i, int j, int x0, int y0) {
  return maskAt(i - x0, i - x0, j - y0 - 1, j - y0);
}
__device__ __forceinline__ uint16_t maskV(int i, int j, int x0, int y0) {
  return maskAt(i - x0 - 1, i - x0, j - y0, j - y0);
}

// ---------------------------------------------------------------------------
// Global-memory index map of one sweep: "a" runs along the sweep direction,
// "b" across it. DIR 0 (x sweep): (a,b) = (i,j), aligned edges are H,
// unaligned edges are V, the velocity is u. DIR 1: (a,b) = (j,i), aligned V,
// unaligned H, velocity v.
// ---------------------------------------------------------------------------
template <int DIR>
struct GMap {
  int nx, ny, na, nb;
  __device__ GMap(int nx_, int ny_) : nx(nx_), ny(ny_), na(DIR == 0 ? nx_ : ny_), nb(DIR == 0 ? ny_ : nx_) {}
  __device__ size_t node(int a, int b) const {
    return DIR == 0 ? (size_t)b * (nx + 1) + a : (size_t)a * (nx + 1) + b;
  }
  __device__ size_t ale(int a, int b) const { return DIR == 0 ? (size_t)b * nx + a : (size_t)a * (nx + 1) + b; }
  __device__ size_t une(int a, int b) const { return DIR == 0 ? (size_t)b * (nx + 1) + a : (size_t)a * nx + b; }
  __device__ size_t cell(int a, int b) const { return DIR == 0 ? (size_t)b * nx + a : (size_t)a * nx + b; }
  // colour of frame node (a, b) from a bit plane
  __device__ int colour(const GL uint16_t *cb, int a, int b) const {
    const int x = DIR == 0 ? a : b, y = DIR == 0 ? b : a;
    return (int)((cb[cb_word(nx, x, y)] >> (x & 15)) & 1u);
  }
};

// colour of node (x, y), inside the grid, from a bit plane
__device__ __forceinline__ int colAt(const GL uint16_t *cb, int nx, int x, int y) {
  return (int)((cb[cb_word(nx, x, y)] >> (x & 15)) & 1u);
}

// ---------------------------------------------------------------------------
// Tile view over the LDS staging (frame coordinates).
// ---------------------------------------------------------------------------
// Old segments of a cell, packed: bits 0-1/2-3 the two edges of segment 0,
// bits 4-5/6-7 those of segment 1, bits 8-9 the number of segments (edges
// 0 bottom, 1 right, 2 top, 3 left). Two markers make one segment; four
// markers make two, each joining the pair around a corner whose colour differs
// from the centre CV, listed by ascending corner (0 BL, 1 BR, 2 TR, 3 TL).
__device__ __forceinline__ uint16_t segCodeOf(int k0, int k1, int k2, int k3, int cc) {
  const bool e0 = k0 != k1, e1 = k1 != k2, e2 = k3 != k2, e3 = k0 != k3;
  const int n = (int)e0 + (int)e1 + (int)e2 + (int)e3;
  if (n == 2) {
    int f = -1, g = -1;
    if (e0) f = 0;
    if (e1) { if (f < 0) f = 1; else g = 1; }
    if (e2) { if (f < 0) f = 2; else g = 2; }
    if (e3) g = 3;
    return (uint16_t)(f | (g << 2) | (1 << 8));
  }
  if (n == 4) {
    // isolated corners are either {BL, TR} or {BR, TL}
    if (k0 != cc) return (uint16_t)(3 | (0 << 2) | (1 << 4) | (2 << 6) | (2 << 8));  // (left,bottom), (right,top)
    return (uint16_t)(0 | (1 << 2) | (2 << 4) | (3 << 6) | (2 << 8));                // (bottom,right), (top,left)
  }
  return 0;
}

// The sweep's LDS view of its tile and halo: old colours and advected
// aligned offsets, enough to gather the landers of each new aligned edge.
struct Tile {
  int na, nb, a0, b0;
  const uint32_t *rows;       // old node colours: bit a-a0+2 of frame row b-b0+2, a in [a0-2, a0+18]
  const double (*sp)[NE];     // aligned (a,b): s' ; a in [a0-2,a0+17], b in [b0-2,b0+18]

  __device__ int C(int a, int b) const { return (int)((rows[b - b0 + HALO] >> (a - a0 + HALO)) & 1u); }
  __device__ bool presA(int a, int b) const { return C(a, b) != C(a + 1, b); }
  __device__ double spv(int a, int b) const { return sp[b - b0 + HALO][a - a0 + HALO]; }

  // aligned markers landing on edge (a,b): their number and the kept source
  // (-1 when none): one lander is kept, of three the middle source
  __device__ int landers(int a, int b, int *keepSrc) const {
    int n = 0, first = -1, second = -1;
    if (a >= 1 && presA(a - 1, b) && spv(a - 1, b) >= 1.0) { first = a - 1; n++; }
    if (presA(a, b)) {
      const double s = spv(a, b);
      if (s >= 0.0 && s < 1.0) {
        if (n == 0) first = a;
        else second = a;
        n++;
      }
    }
    if (a + 1 < na && presA(a + 1, b) && spv(a + 1, b) < 0.0) {
      if (n == 0) first = a + 1;
      else if (n == 1) second = a + 1;
      n++;
    }
    *keepSrc = n == 1 ? first : (n == 3 ? second : -1);
    return n;
  }
};

// Aligned markers landing on edge (a,b) of a fit view: their number and the
// kept source (-1 when none): one lander is kept, of three the middle source.
template <class View>
__device__ __forceinline__ int viewLanders(const View &T, int a, int b, int *keepSrc) {
  int n = 0, first = -1, second = -1;
  if (a >= 1 && T.presA(a - 1, b) && T.spv(a - 1, b) >= 1.0) { first = a - 1; n++; }
  if (T.presA(a, b)) {
    const double v = T.spv(a, b);
    if (v >= 0.0 && v < 1.0) {
      if (n == 0) first = a;
      else second = a;
      n++;
    }
  }
  if (a + 1 < T.na && T.presA(a + 1, b) && T.spv(a + 1, b) < 0.0) {
    if (n == 0) first = a + 1;
    else if (n == 1) second = a + 1;
    n++;
  }
  *keepSrc = n == 1 ? first : (n == 3 ? second : -1);
  return n;
}
// The aligned marker (p,q) landed on edge (target,q) and is the one kept there.
template <class View>
__device__ __forceinline__ bool viewKeptOn(const View &T, int p, int q, int target) {
  const double v = T.spv(p, q);
  int tg = v >= 1.0 ? p + 1 : (v < 0.0 ? p - 1 : p);
  if (tg < 0 || tg >= T.na) tg = -1;
  if (tg != target) return false;
  int keep;
  viewLanders(T, target, q, &keep);
  return keep == p;
}

// One of 8 or 3 named registers, chosen by a tree of selects on the bits of
// k (values kept in an array would be read with an index, from scratch)
__device__ __forceinline__ double pick8(int k, double v0, double v1, double v2, double v3, double v4, double v5,
                                        double v6, double v7) {
  const bool b0 = (k & 1) != 0, b1 = (k & 2) != 0, b2 = (k & 4) != 0;
  const double x01 = b0 ? v1 : v0, x23 = b0 ? v3 : v2, x45 = b0 ? v5 : v4, x67 = b0 ? v7 : v6;
  const double y03 = b1 ? x23 : x01, y47 = b1 ? x67 : x45;
  return b2 ? y47 : y03;
}
__device__ __forceinline__ double pick3(int k, double v0, double v1, double v2) {
  const double x01 = (k & 1) != 0 ? v1 : v0;
  return (k & 2) != 0 ? v2 : x01;
}

// One fit job's neighbourhood (used by the fit kernel, one lane per new
// unaligned marker on line a, row b), gathered in one round of independent
// loads: old node colours a-2..a+2 x b-1..b+2 as a bit mask (four 8-byte
// loads of the bit plane), the new colours of the line's two nodes,
// the advected offsets s' of the aligned edges a-2..a+1 on rows b and b+1 and
// the (t, d) pairs of the unaligned edges a-1..a+1 on row b. That covers every
// read of the crossing search, the circles' inner points and the centre rules;
// only the chain neighbours one row up or down or two lines away, and the old
// centre colour of a cell with four markers (rare), are read from memory. Window slots outside the grid are read at the nearest edge
// inside it (colours then masked to 0) and never used: every access of the
// logic is guarded by the grid bounds.
template <int DIR>
struct JobView {
  GMap<DIR> G;
  int na, nb, a, b;
  const GL uint16_t *__restrict__ col;   // old node colours (bit plane)
  const GL uint8_t *__restrict__ cen;    // old centre colours
  const GL uint16_t *__restrict__ ncol;  // new node colours (bit plane)
  const GL double *__restrict__ sp;     // aligned: s' (present edges)
  const GL double *__restrict__ td;     // unaligned: (old offset t, displacement d) pairs (present edges)
  uint32_t cm = 0;  // old node (a-2+i, b-1+j): bit j*5+i
  uint32_t nm = 0;  // new colours of nodes (a,b) and (a,b+1): bits 0, 1
  double s0, s1, s2, s3, s4, s5, s6, s7;  // s' of aligned (a-2+i, b+j): s<j*4+i>
  double t0, t1, t2, d0, d1, d2;          // (t, d) of unaligned (a-1+i, b): t<i>, d<i>
  __device__ JobView(const SweepView &W, int a_, int b_)
      : G(W.nx, W.ny), na(G.na), nb(G.nb), a(a_), b(b_), col(gp(W.col)), cen(gp(W.cen)), ncol(gp(W.ncol)),
        sp(gp(W.sp)), td(gp(W.dd)) {
    // Every load is unconditional (all issue before the first wait): indices
    // are clamped into the grid and slots outside it are masked afterwards.
    // The node window, in grid coordinates columns xs .. xs+NX-1 and rows
    // ys .. ys+NY-1 (x sweep 5 x 4 from (a-2, b-1), y sweep 4 x 5 from
    // (b-1, a-2)), lies in two groups of 4 rows (rows 4g .. 4g+3, one aligned
    // 8-byte piece of a block) in each of two block columns.
    auto cl = [](int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); };
    constexpr int NX = DIR == 0 ? 5 : 4, NY = DIR == 0 ? 4 : 5;
    const int xs = DIR == 0 ? a - 2 : b - 1, ys = DIR == 0 ? b - 1 : a - 2;
    const int nbx = cb_nbx(W.nx), nby = cb_nbx(W.ny);
    const int bxl = xs >> 4, g1 = ys >> 2;  // floor, also below 0
    auto piece = [&](int g, int bx) -> uint64_t {
      const int by = g >> 2;
      const size_t w = ((size_t)cl(by, 0, nby - 1) * (size_t)nbx + (size_t)cl(bx, 0, nbx - 1)) * 16u + 4u * (size_t)(g & 3);
      return *(const GL uint64_t *)(col + w);
    };
    const uint64_t q00 = piece(g1, bxl), q01 = piece(g1, bxl + 1), q10 = piece(g1 + 1, bxl),
                   q11 = piece(g1 + 1, bxl + 1);
    auto ncolAt = [&](int p, int q) -> uint32_t {
      const int x = DIR == 0 ? p : q, y = DIR == 0 ? q : p;
      return (uint32_t)(ncol[cb_word(W.nx, x, y)] >> (x & 15));
    };
    const uint32_t n0 = ncolAt(a, b), n1 = ncolAt(a, b + 1);
    auto al = [&](int i, int j) -> double { return sp[G.ale(cl(a - 2 + i, 0, na - 1), b + j)]; };
    s0 = al(0, 0), s1 = al(1, 0), s2 = al(2, 0), s3 = al(3, 0);
    s4 = al(0, 1), s5 = al(1, 1), s6 = al(2, 1), s7 = al(3, 1);
    // (t, d) pairs are 16-byte aligned: one load each
    struct alignas(16) TD {
      double t, d;
    };
    auto un = [&](int i) -> TD {
      const GL TD *q = (const GL TD *)td + G.une(cl(a - 1 + i, 0, na), b);
      return TD{q->t, q->d};
    };
    const TD p0 = un(0), p1 = un(1), p2 = un(2);
    t0 = p0.t, t1 = p1.t, t2 = p2.t;
    d0 = p0.d, d1 = p1.d, d2 = p2.d;
    // pieces of blocks outside the grid read as 0
    const bool okL = bxl >= 0, okR = bxl + 1 < nbx, ok1 = g1 >= 0, ok2 = ((g1 + 1) >> 2) < nby;
    const uint64_t p00 = okL && ok1 ? q00 : 0, p01 = okR && ok1 ? q01 : 0, p10 = okL && ok2 ? q10 : 0,
                   p11 = okR && ok2 ? q11 : 0;
#pragma unroll
    for (int r = 0; r < NY; r++) {
      // grid row ys + r: its group, its word in both block columns, the window's bits
      const int y = ys + r;
      const bool second = (y >> 2) != g1;
      const int sh = 16 * (y & 3);
      const uint32_t lo = (uint32_t)((second ? p10 : p00) >> sh) & 0xFFFFu;
      const uint32_t hi = (uint32_t)((second ? p11 : p01) >> sh) & 0xFFFFu;
      const uint32_t bits = ((lo | (hi << 16)) >> (xs & 15)) & ((1u << NX) - 1u);
      if (DIR == 0) {
        cm |= bits << (r * 5);  // frame row j = r, frame column i = bit
      } else {
#pragma unroll
        for (int c = 0; c < NX; c++) cm |= ((bits >> c) & 1u) << (c * 5 + r);  // frame (i, j) = (r, c)
      }
    }
    // nodes outside the grid are 0
#pragma unroll
    for (int j = 0; j < 4; j++)
#pragma unroll
      for (int i = 0; i < 5; i++) {
        const int x = a - 2 + i, y = b - 1 + j;
        if (!(x >= 0 && x <= na && y >= 0 && y <= nb)) cm &= ~(1u << (j * 5 + i));
      }
    nm = (n0 & 1u) | ((n1 & 1u) << 1);
  }
  __device__ int C(int p, int q) const {
    const int i = p - (a - 2), j = q - (b - 1);
    if (i >= 0 && i < 5 && j >= 0 && j < 4) return (int)((cm >> (j * 5 + i)) & 1u);
    return G.colour(col, p, q);
  }
  __device__ int cenv(int p, int q) const { return cen[G.cell(p, q)]; }
  __device__ bool presA(int p, int q) const { return C(p, q) != C(p + 1, q); }
  __device__ double spv(int p, int q) const {
    const int i = p - (a - 2), j = q - b;
    if (i >= 0 && i < 4 && j >= 0 && j < 2) return pick8(j * 4 + i, s0, s1, s2, s3, s4, s5, s6, s7);
    return sp[G.ale(p, q)];
  }
  __device__ double tU(int p, int q) const {
    const int i = p - (a - 1);
    if (q == b && i >= 0 && i < 3) return pick3(i, t0, t1, t2);
    return td[2 * G.une(p, q)];
  }
  __device__ double dU(int p, int q) const {
    const int i = p - (a - 1);
    if (q == b && i >= 0 && i < 3) return pick3(i, d0, d1, d2);
    return td[2 * G.une(p, q) + 1];
  }
  // the centre colour only decides the pairing of a cell with four markers
  __device__ uint16_t segc(int p, int q) const {
    const int k0 = C(p, q), k1 = C(p + 1, q), k2 = C(p + 1, q + 1), k3 = C(p, q + 1);
    const bool four = k0 != k1 && k1 != k2 && k3 != k2 && k0 != k3;
    return segCodeOf(k0, k1, k2, k3, four ? cenv(p, q) : 0);
  }
  __device__ int newC(int p, int q) const {
    if (p == a && q == b) return (int)(nm & 1u);
    if (p == a && q == b + 1) return (int)((nm >> 1) & 1u);
    return G.colour(ncol, p, q);
  }
};

struct MRef {
  int kind;  // 0 aligned, 1 unaligned
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

// advected marker in the frame of node (a0,b0): aligned markers move along
// their line (blue points), unaligned ones off it (gray points)
template <class View>
__device__ __forceinline__ void advPoint(const View &T, MRef m, int a0, int b0, double *X, double *Y) {
  if (m.kind == 0) {
    *X = (double)(m.a - a0) + T.spv(m.a, m.b);
    *Y = (double)(m.b - b0);
  } else {
    *X = (double)(m.a - a0) + T.dU(m.a, m.b);
    *Y = (double)(m.b - b0) + T.tU(m.a, m.b);
  }
}

// "left of line a = a0" iff x < a0, decided exactly on the offset
template <class View>
__device__ __forceinline__ bool leftOf(const View &T, MRef m, int a0) {
  if (m.kind == 0) return T.spv(m.a, m.b) < (double)(a0 - m.a);
  return T.dU(m.a, m.b) < (double)(a0 - m.a);
}

// chain neighbour of the marker on edge e of old cell (p,q), away from it:
// its partner in the cell across edge e
template <class View>
__device__ bool chainNb(const View &T, int p, int q, int e, MRef *out) {
  int pp = p, qq = q;
  if (e == 0) qq = q - 1;
  else if (e == 1) pp = p + 1;
  else if (e == 2) qq = q + 1;
  else pp = p - 1;
  if (pp < 0 || pp >= T.na || qq < 0 || qq >= T.nb) return false;
  const int eo = (e + 2) & 3;
  const uint32_t c = T.segc(pp, qq);
  const int nseg = (c >> 8) & 3;
  for (int k = 0; k < 2; k++) {
    if (k >= nseg) break;
    const int eA = (c >> (4 * k)) & 3, eB = (c >> (4 * k + 2)) & 3;
    if (eA == eo) { *out = edgeMarker(pp, qq, eB); return true; }
    if (eB == eo) { *out = edgeMarker(pp, qq, eA); return true; }
  }
  return false;
}

// Circle through three points as a(X^2+Y^2) + bX + cY + e = 0, intersected
// with X = 0; keeps the root across chord P2P3 from the outer point.
__device__ bool circleRoot(double Xa, double Ya, double Xb, double Yb, double Xc, double Yc, double Xo, double Yo,
                           double X2, double Y2, double X3, double Y3, double ysl, double *root, uint32_t *ties,
                           uint32_t *rejects) {
  const double Qa = Xa * Xa + Ya * Ya;
  const double Qb = Xb * Xb + Yb * Yb;
  const double Qc = Xc * Xc + Yc * Yc;
  const double ca = Xa * (Yb - Yc) + Xb * (Yc - Ya) + Xc * (Ya - Yb);
  const double cc = Qa * (Xb - Xc) + Qb * (Xc - Xa) + Qc * (Xa - Xb);
  const double ce = -(Qa * (Xb * Yc - Xc * Yb) + Qb * (Xc * Ya - Xa * Yc) + Qc * (Xa * Yb - Xb * Ya));
  double r;
  if (ca == 0.0) {
    if (cc == 0.0) return false;
    r = -ce / cc;
  } else {
    double disc = cc * cc - 4.0 * ca * ce;
    if (disc < 0.0) disc = 0.0;
    const double sq = sqrt(disc);
    const double q = -0.5 * (cc + (cc >= 0.0 ? sq : -sq));
    double r1, r2;
    if (q == 0.0) {
      r1 = 0.0;
      r2 = 0.0;
    } else {
      r1 = q / ca;
      r2 = ce / q;
    }
    const double DX = X3 - X2, DY = Y3 - Y2;
    const double L2 = DX * DX + DY * DY;
    const double so = DX * (Yo - Y2) - DY * (Xo - X2);
    const double s1 = DX * (r1 - Y2) - DY * (0.0 - X2);
    const double s2 = DX * (r2 - Y2) - DY * (0.0 - X2);
    if (fabs(s1) < TIE_EPS * L2 || fabs(s2) < TIE_EPS * L2) (*ties)++;
    const bool q1 = (s1 > 0.0 && so < 0.0) || (s1 < 0.0 && so > 0.0);
    const bool q2 = (s2 > 0.0 && so < 0.0) || (s2 < 0.0 && so > 0.0);
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

// Counters of one workgroup, in LDS (events are rare next to the work).
// this workgroup's counter partition
__device__ __forceinline__ unsigned long long *ctrPart(unsigned long long *ctr) {
  return ctr + (blockIdx.x % (uint32_t)CTR_PARTS) * CTR_STRIDE;
}

struct Counts {
  uint32_t *s;
  __device__ void add(int k, uint32_t v) const {
    if (v) atomicAdd(&s[k], v);
  }
};

// The fit jobs of one sweep direction, numbered 0 .. total()-1 across its
// queues: job w of queue q is entry q * region + (w - beg[q]), counted from
// the direction's end of the list. The queue counts are uniform, so the
// lookup is a few compares per lane.
static_assert(NJQ == NXCD, "one job queue per XCD share");
struct JobIndex {
  uint32_t beg[NJQ + 1];
  uint32_t region;
  // a count past its region (reservations whose entries were dropped, the
  // grid's error latched) is read as the region: no job outside it is read
  __device__ JobIndex(const uint32_t *counts, uint32_t nq, uint32_t reg) : region(reg) {
    beg[0] = 0;
#pragma unroll
    for (uint32_t q = 0; q < NJQ; q++) beg[q + 1] = beg[q] + (q < nq ? min(counts[CNT_LINE * q], reg) : 0u);
  }
  __device__ uint32_t total() const { return beg[NJQ]; }
  __device__ uint32_t entry(uint32_t w) const {
    // the last queue starting at or before w holds it (empty queues in
    // between start where the next one does)
    uint32_t base = 0, off = 0;
#pragma unroll
    for (uint32_t q = 1; q < NJQ; q++)
      if (w >= beg[q]) {
        base = q * region;
        off = beg[q];
      }
    return base + (w - off);
  }
};

// New unaligned marker on interior line a, row b (present by the new
// colours): its offset, and the centre-CV results for the cell right of the
// line (cell a) and left of it (cell a-1): -1 or the new centre colour.
template <class View>
__device__ double newUnaligned(const View &T, int a, int b, int *resRight, int *resLeft, const Counts &cnt, bool count,
                               bool line) {
  *resRight = -1;
  *resLeft = -1;
  uint32_t lties = 0, lrej = 0;
  // crossing segments of old cells (a-1,b) then (a,b); the first three kept
  int ncross = 0;
  int cp0 = 0, cp1 = 0, cp2 = 0, cl0 = 0, cl1 = 0, cl2 = 0, cr0 = 0, cr1 = 0, cr2 = 0;
  double ys0 = 0.0, ys1 = 0.0, ys2 = 0.0;
  for (int p = a - 1; p <= a; p++) {
    const uint32_t c = T.segc(p, b);
    const int nseg = (c >> 8) & 3;
    for (int k = 0; k < 2; k++) {
      if (k >= nseg) break;
      const int eA = (c >> (4 * k)) & 3, eB = (c >> (4 * k + 2)) & 3;
      const bool l1 = leftOf(T, edgeMarker(p, b, eA), a), l2 = leftOf(T, edgeMarker(p, b, eB), a);
      if (l1 == l2) continue;
      const int el = l1 ? eA : eB, er = l1 ? eB : eA;
      double X2, Y2, X3, Y3;
      advPoint(T, edgeMarker(p, b, el), a, b, &X2, &Y2);
      advPoint(T, edgeMarker(p, b, er), a, b, &X3, &Y3);
      const double ys = chordY(X2, Y2, X3, Y3);
      if (ncross == 0) { cp0 = p; cl0 = el; cr0 = er; ys0 = ys; }
      else if (ncross == 1) { cp1 = p; cl1 = el; cr1 = er; ys1 = ys; }
      else if (ncross == 2) { cp2 = p; cl2 = el; cr2 = er; ys2 = ys; }
      ncross++;
    }
  }
  int pick = -1;
  if (ncross == 1) {
    pick = 0;
  } else if (ncross == 3) {
    if (count) cnt.add(C_THREE_CROSSINGS, 1u);
    // the median by chord height, equal heights ordered by enumeration
    const int below0 = (ys1 < ys0) + (ys2 < ys0);
    const int below1 = (ys0 <= ys1) + (ys2 < ys1);
    const int below2 = (ys0 <= ys2) + (ys1 <= ys2);
    pick = below0 == 1 ? 0 : (below1 == 1 ? 1 : (below2 == 1 ? 2 : -1));
    lties += (fabs(ys0 - ys1) < TIE_EPS) + (fabs(ys0 - ys2) < TIE_EPS) + (fabs(ys1 - ys2) < TIE_EPS);
  }
  if (pick < 0) {
    if (count) {
      cnt.add(C_PARITY_FALLBACK, 1u);
      cnt.add(C_TIES, (uint32_t)(lties));
    }
    return 0.5;
  }
  const int p = pick == 0 ? cp0 : (pick == 1 ? cp1 : cp2);
  const int el = pick == 0 ? cl0 : (pick == 1 ? cl1 : cl2);
  const int er = pick == 0 ? cr0 : (pick == 1 ? cr1 : cr2);
  const double ysl = pick == 0 ? ys0 : (pick == 1 ? ys1 : ys2);
  const MRef m2 = edgeMarker(p, b, el), m3 = edgeMarker(p, b, er);
  double X2, Y2, X3, Y3;
  advPoint(T, m2, a, b, &X2, &Y2);
  advPoint(T, m3, a, b, &X3, &Y3);
  if (fabs(X2) < TIE_EPS || fabs(X3) < TIE_EPS) lties++;
  MRef m1, m4;
  const bool h1 = chainNb(T, p, b, el, &m1);
  const bool h4 = chainNb(T, p, b, er, &m4);
  double y;
  uint32_t fb = 0;
  if (X3 == 0.0) {
    y = Y3;
  } else if (line) {
    // straight-line placement: where segment P2P3 crosses the line
    y = ysl;
  } else {
    double rA = 0, rB = 0;
    bool okA = false, okB = false;
    if (h1) {
      double X1, Y1;
      advPoint(T, m1, a, b, &X1, &Y1);
      okA = circleRoot(X1, Y1, X2, Y2, X3, Y3, X1, Y1, X2, Y2, X3, Y3, ysl, &rA, &lties, &lrej);
    }
    if (h4) {
      double X4, Y4;
      advPoint(T, m4, a, b, &X4, &Y4);
      okB = circleRoot(X2, Y2, X3, Y3, X4, Y4, X4, Y4, X2, Y2, X3, Y3, ysl, &rB, &lties, &lrej);
    }
    if (okA && okB) y = (rA + rB) * 0.5;
    else if (okA) y = rA;
    else if (okB) y = rB;
    else {
      y = ysl;
      fb = 1;
    }
  }
  if (y < TIE_EPS || 1.0 - y < TIE_EPS) lties++;
  if (count) {
    cnt.add(C_TIES, (uint32_t)(lties));
    cnt.add(C_FIT_REJECT, (uint32_t)(lrej));
    cnt.add(C_FIT_FALLBACK, (uint32_t)(fb));
  }
  // Centre-CV candidates: for the cell right of the line, the crossing
  // endpoint on its side (P3) and, if that is an unaligned point, its chain
  // neighbour (P4); for the cell on the left, P2 then P1. A candidate counts
  // when it is an aligned marker kept on that cell's bottom or top edge; the
  // corner it shares with this line is then isolated.
  auto qualifies = [&](MRef m, int cellA) -> bool {
    return m.kind == 0 && (m.b == b || m.b == b + 1) && viewKeptOn(T, m.a, m.b, cellA);
  };
  if (a < T.na) {
    // cell a, right of the line
    if (qualifies(m3, a)) *resRight = 1 - T.newC(a, m3.b);
    else if (m3.kind == 1 && h4 && qualifies(m4, a)) *resRight = 1 - T.newC(a, m4.b);
  }
  if (a >= 1) {
    // cell a-1, left of the line
    if (qualifies(m2, a - 1)) *resLeft = 1 - T.newC(a, m2.b);
    else if (m2.kind == 1 && h1 && qualifies(m1, a - 1)) *resLeft = 1 - T.newC(a, m1.b);
  }
  return y;
}

// ---------------------------------------------------------------------------
// Sweep kernel: one workgroup per active tile (persistent over the list of
// active tiles of all grids). Frame coordinates: halo slot (la, lb) is node
// (a0-2+la, b0-2+lb). Colours are also kept as one bit mask per frame row, so
// present edges, new edges and 4-marker cells are found with a few word
// operations per row and only the edges that carry markers are visited one by
// one. The sweep direction is a property of the tile's grid (its step
// parity): the compaction lists the tiles of x-sweeping grids from the front
// of the active list and those of y-sweeping grids from its back, and each
// direction has its own launch.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// ONE: the engine holds a single grid, whose descriptor comes with the kernel
// arguments (loop-invariant, no descriptor loads per tile).
constexpr int SWEEP_BS = 128;
constexpr int NTILES_LDS = 32;  // tile entries read once at the start

// centre rules of one job (defined with the centre kernel below)
template <int DIR>
__device__ __forceinline__ void centreJob(const SweepView &W, uint32_t e, const Counts &cnt);

template <int DIR, bool ONE>
__global__ __launch_bounds__(SWEEP_BS, 8) void k_sweep(SweepArgs A, const Inst *__restrict__ inst) {
  __shared__ uint64_t sBlk[NH];     // colour words of halo row r: block columns tx-1, tx, tx+1
  __shared__ double sSp[NH][NE];
  __shared__ uint32_t sRow[NH];     // old colours, bit la of frame row lb
  __shared__ uint32_t sNRow[NN];    // new colours, bit a-a0 of row b-b0
  __shared__ uint32_t sRecv[NN];    // new aligned edges (a,b) that receive a lander, bit a-a0
  __shared__ uint2 sTiles[NTILES_LDS];  // this workgroup's first (tile, grid) entries
  __shared__ uint16_t sAdv[2 * NH * NE];
  __shared__ uint2 sJob[JOBCAP];    // new interior unaligned markers of this workgroup's tiles
  __shared__ uint32_t sNAdv, sNJob, sHas, sJobBase;
  __shared__ uint32_t sCnt[NCOUNTERS];

  const int tid = threadIdx.x;
  const uint32_t cur = A.cur;
  if (tid < NCOUNTERS) sCnt[tid] = 0;
  if (tid == 0) sNJob = 0;
  if (tid < NH) sRow[tid] = 0;
  const Counts cnt{sCnt};
  // the queued jobs go to this workgroup's queue of the fit kernel's list
  // with one reservation (entries past the queue's region, which the per-tile
  // bound rules out, are dropped and flagged)
  uint32_t jq = 0;
  auto flushJobs = [&]() {
    const uint32_t n = sNJob;
    if (tid == 0) sJobBase = atomicAdd(A.njobs + CNT_LINE * jq, n);
    __syncthreads();
    for (uint32_t w = tid; w < n; w += blockDim.x) {
      const uint32_t k = sJobBase + w;
      const uint32_t e = jq * A.jobRegion + k;
      if (k < A.jobRegion) A.jobs[DIR == 0 ? e : A.jobTop - 1u - e] = sJob[w];
      else atomicOr(ONE ? A.one.err : inst[sJob[w].x].err, ERRBIT_CAP);
    }
    __syncthreads();
    if (tid == 0) sNJob = 0;
  };

  // Staging of colours: the tile and its halo (nodes x0-2 .. x0+18, rows
  // y0-2 .. y0+18) sit in 3 x 3 blocks of the bit plane; lane k < 3 NH holds
  // the word of halo row k / 3 in block column tx-1 + k % 3. The next tile's
  // words are fetched into a register while the current tile computes. The
  // load is unconditional: its indices are clamped into the grid, and words of
  // rows or blocks outside it are zeroed when staged.
  static_assert(3 * NH <= SWEEP_BS && HALO <= TS && NH - HALO <= 2 * TS, "staging words");
  uint32_t pc = 0;
  bool pin = false;
  auto prefetch = [&](uint2 te) {
    const uint32_t gt = te.x;
    int nx, ny, ntx;
    uint32_t tile0;
    const GL uint16_t *col;
    if (ONE) {
      nx = A.one.nx, ny = A.one.ny, ntx = A.one.ntx, tile0 = A.one.tile0;
      col = gp(A.one.col);
    } else {
      const Inst &I = inst[te.y];
      nx = I.nx, ny = I.ny, ntx = I.ntx, tile0 = I.tile0;
      col = gp(I.col[cur]);
    }
    const uint32_t lt = gt - tile0;
    const int tx = (int)(lt % (uint32_t)ntx), py0 = (int)(lt / (uint32_t)ntx) * TS;
    const int k = min(tid, 3 * NH - 1), y = py0 - HALO + k / 3, bx = tx - 1 + k % 3, nbx = cb_nbx(nx);
    pin = y >= 0 && y <= ny && bx >= 0 && bx < nbx;
    pc = col[cb_word(nx, min(max(bx, 0), nbx - 1) * TS, min(max(y, 0), ny))];
  };

  const uint32_t ntile = *A.count;
  // this workgroup's tile indices, so no index load waits in the loop
  auto entry = [&](uint32_t it) -> uint2 { return A.list[DIR == 0 ? it : A.ntiles - 1u - it]; };
  // this workgroup's tiles: a stride of the list for one grid, a contiguous
  // chunk of it for many (consecutive entries mostly share a grid, and so do
  // the fit jobs the workgroup queues, which keeps fit wavefronts on one grid)
  uint32_t itBeg, itEnd, itStep;
  if (ONE && gridDim.x % NXCD == 0u) {
    // workgroups are dispatched round-robin over the XCDs, each with its own
    // L2: XCD x takes the x-th share of the list (neighbouring tiles, whose
    // halos overlap, sit close together in it), a stride of it per workgroup
    const uint32_t x = blockIdx.x % NXCD, per = gridDim.x / NXCD, share = (ntile + NXCD - 1u) / NXCD;
    itBeg = x * share + blockIdx.x / NXCD;
    itEnd = min(ntile, (x + 1u) * share);
    itStep = per;
    // the share's fit jobs go to queue x: returning atomics on one count
    // serialise, and thousands of workgroups flush near the sweep's end
    if (A.jobQ == NJQ) jq = x;
  } else if (ONE) {
    itBeg = blockIdx.x;
    itEnd = ntile;
    itStep = gridDim.x;
  } else {
    // at least A.minChunk tiles per workgroup: a workgroup queues its fit
    // jobs together, and the fit runs once per distinct grid of a wavefront,
    // so short chunks (few active tiles) would mix grids in every wavefront
    const uint32_t chunk = max((ntile + gridDim.x - 1) / gridDim.x, max(A.minChunk, 1u));
    itBeg = min(ntile, blockIdx.x * chunk);
    itEnd = min(ntile, itBeg + chunk);
    itStep = 1;
    // queue b % 8: its workgroups' chunks make at most a share plus a chunk
    if (A.jobQ == NJQ) jq = blockIdx.x % NJQ;
  }
  if (tid < NTILES_LDS && itBeg + tid * itStep < itEnd) sTiles[tid] = entry(itBeg + tid * itStep);
  __syncthreads();
  auto tileAt = [&](uint32_t it) -> uint2 {
    const uint32_t k = (it - itBeg) / itStep;
    const uint2 e = k < NTILES_LDS ? sTiles[k] : entry(it);
    return make_uint2(uni(e.x), uni(e.y));
  };
  if (itBeg < itEnd) prefetch(tileAt(itBeg));
  // one grid: lambda = dt / h from the view, or from the grid's device dt when
  // the call passes one per grid (a batch or pool holding a single grid)
  const double lamOne = ONE ? (A.dts ? A.dts[0] / inst[0].h : A.one.lam) : 0.0;
  if (ONE && A.pendJobs) {
    // the centre rules of the step's first sweep (the other direction, whose
    // jobs sit at the other end of the list), while the first tile's colours
    // are on their way
    const JobIndex J(A.pendJobs, A.jobQ, A.jobRegion);
    for (uint32_t w = blockIdx.x * blockDim.x + tid; w < J.total(); w += gridDim.x * blockDim.x) {
      const uint32_t e = J.entry(w);
      centreJob<1 - DIR>(A.pend, A.jobs[DIR == 1 ? e : A.jobTop - 1u - e].y, cnt);
    }
  }

  for (uint32_t it = itBeg; it < itEnd; it += itStep) {
    const uint2 te = tileAt(it);
    const uint32_t gt = te.x, kinst = ONE ? 0u : te.y;
    const SweepView W = ONE ? A.one
                            : sweep_view(inst[kinst], cur, DIR, A.u, A.v,
                                         (A.dts ? A.dts[kinst] : A.dt) / inst[kinst].h);
    const int nx = W.nx, ny = W.ny;
    const GMap<DIR> G(nx, ny);
    const int na = G.na, nb = G.nb;
    const double lam = ONE ? lamOne : W.lam;
    const GL double *__restrict__ alo = gp(DIR == 0 ? W.hoff : W.voff);
    const GL double *__restrict__ uno = gp(DIR == 0 ? W.voff : W.hoff);
    GL double *__restrict__ aln = gp(DIR == 0 ? W.nhoff : W.nvoff);
    GL double *__restrict__ unn = gp(DIR == 0 ? W.nvoff : W.nhoff);
    const GL double *__restrict__ vel = gp(W.vel);
    GL uint16_t *__restrict__ ncol = gp(W.ncol);
    GL double *__restrict__ spg = gp(W.sp);
    GL double *__restrict__ ddg = gp(W.dd);
    uint32_t *errg = W.err;  // written only on an error
    auto V = [&](int a, int r) -> double {
      r = r < 0 ? 0 : (r > nb - 1 ? nb - 1 : r);
      return vel[G.une(a, r)];
    };
    const uint32_t lt = gt - W.tile0;
    const int tx = (int)(lt % (uint32_t)W.ntx), ty = (int)(lt / (uint32_t)W.ntx);
    const int x0 = tx * TS, y0 = ty * TS;
    const int a0 = DIR == 0 ? x0 : y0, b0 = DIR == 0 ? y0 : x0;
    Tile T;
    T.na = na;
    T.nb = nb;
    T.rows = sRow;
    T.sp = sSp;
    T.a0 = a0;
    T.b0 = b0;
    __syncthreads();  // the previous tile is done with LDS
    if (tid == 0) {
      sNAdv = 0;
      sHas = 0;
    }
    if (tid < NN) sRecv[tid] = 0;
    // --- stage old colours -----------------------------------------------------
    if (tid < 3 * NH) ((uint16_t *)&sBlk[tid / 3])[tid % 3] = pin ? (uint16_t)pc : (uint16_t)0;
    __syncthreads();
    // frame-row masks: bit la of row lb is halo node (a0-2+la, b0-2+lb); the
    // halo nodes of physical row r are bits TS-HALO .. TS-HALO+NH-1 of its words
    if (tid < NH) {
      auto phys = [&](int r) -> uint32_t { return (uint32_t)(sBlk[r] >> (TS - HALO)) & ((1u << NH) - 1u); };
      if (DIR == 0) {
        sRow[tid] = phys(tid);
      } else {
        uint32_t m = 0;
        for (int r = 0; r < NH; r++) m |= ((phys(r) >> tid) & 1u) << r;
        sRow[tid] = m;
      }
    }
    __syncthreads();
    // --- list the present edges -----------------------------------------------
    // aligned (a,b) whose advected offsets feed this tile's landers and flips:
    // a in [a0-1, a0+16] (la in [1, 19)) inside [0, na), rows b in [b0, b0+16]
    // (lb in [2, 19)) inside [0, nb];
    // unaligned (a,b), only those of this tile (nothing reads the others):
    // lb in [2,18) with b < nb, la in [2,18) or the wall a = na
    const int laMinA = max(HALO - 1, HALO - a0), laMaxA = min(NE - 2, na - 1 - a0 + HALO);
    const int laMaxU = min(HALO + TS - 1 + (na - a0 == TS ? 1 : 0), na - a0 + HALO);
    const uint32_t maskA = laMaxA >= laMinA ? ((2u << laMaxA) - 1u) & ~((1u << laMinA) - 1u) : 0u;
    const uint32_t maskU = ((2u << laMaxU) - 1u) & ~((1u << HALO) - 1u);
    if (tid < NH) {
      const int lb = tid, b = b0 - HALO + lb;
      const uint32_t r = sRow[lb];
      if (lb >= HALO && lb <= HALO + TS && b <= nb) {
        uint32_t m = (r ^ (r >> 1)) & maskA;
        if (m) {
          uint32_t w = atomicAdd(&sNAdv, (uint32_t)__popc(m));
          while (m) {
            const int la = __ffs(m) - 1;
            m &= m - 1;
            sAdv[w++] = (uint16_t)(lb * NE + la);
          }
        }
      }
      if (lb >= HALO && lb < HALO + TS && b < nb) {
        uint32_t m = (r ^ sRow[lb + 1]) & maskU;
        if (m) {
          uint32_t w = atomicAdd(&sNAdv, (uint32_t)__popc(m));
          while (m) {
            const int la = __ffs(m) - 1;
            m &= m - 1;
            sAdv[w++] = (uint16_t)(0x8000u | (lb * NH + la));
          }
        }
      }
    }
    // new colours start from the old ones: node (a0+i, b0+j) = slot (i+2, j+2)
    if (tid < NN) sNRow[tid] = (sRow[tid + HALO] >> HALO) & ((1u << NN) - 1u);
    __syncthreads();
    // new colours out: the tile's own nodes and, where the tile ends at the
    // grid's last node row or column, those nodes too; one 16-bit word per
    // node row (the last column's node alone in its block's word)
    auto writeColours = [&]() {
      const int r = tid, y = y0 + r;
      if (r <= TS && y <= ny && (r < TS || y == ny)) {
        uint32_t w = 0;  // bit i: node (x0 + i, y), i in [0, TS]
        if (DIR == 0) {
          w = sNRow[r];
        } else {
          for (int i = 0; i < NN; i++) w |= ((sNRow[i] >> r) & 1u) << i;
        }
        w &= (2u << min(TS, nx - x0)) - 1u;
        ncol[cb_word(nx, x0, y)] = (uint16_t)w;
        if (x0 + TS == nx) ncol[cb_word(nx, nx, y)] = (uint16_t)(w >> TS);
      }
    };
    const uint32_t nadv = sNAdv;
    if (nadv == 0) {
      // no marker in reach: the tile keeps its state
      writeColours();
      if (tid == 0) {
        A.has[gt] = 0;
        cnt.add(C_TILES_EMPTY, 1u);
      }
      if (it + itStep < itEnd) prefetch(tileAt(it + itStep));
      continue;
    }
    if (tid == 0) cnt.add(C_TILES_SWEPT, 1u);
    // --- advect the listed markers (Eq. marker_dis), flip crossed nodes ------
    for (uint32_t w = tid; w < nadv; w += blockDim.x) {
      const uint32_t code = sAdv[w];
      if (!(code & 0x8000u)) {
        const int la = code % NE, lb = code / NE;
        const int a = a0 - HALO + la, b = b0 - HALO + lb;
        const double s = alo[G.ale(a, b)];
        const double ub = lerp(lerp(V(a, b - 1), V(a + 1, b - 1), s), lerp(V(a, b), V(a + 1, b), s), 0.5);
        const double d = ub * lam;
        const double spv = s + d;
        sSp[lb][la] = spv;
        const bool own = la >= HALO && la < HALO + TS && lb >= HALO && (lb < HALO + TS || b == nb);
        if (own) {
          spg[G.ale(a, b)] = spv;
          cnt.add(C_MARKERS, 1u);
          if (fabs(d) > 0.5) atomicOr(errg, ERRBIT_CFL);
          if ((spv >= 1.0 && a + 1 >= na) || (spv < 0.0 && a == 0)) atomicOr(errg, ERRBIT_DOMAIN);
        }
        // the crossed node flips; the edge it lands on receives a lander
        const int j = b - b0;
        if (j >= 0 && j < NN) {
          int flip = -1, t = a;
          if (spv >= 1.0) {
            if (a + 1 < na) flip = a + 1;
            t = a + 1 < na ? a + 1 : -1;
          } else if (spv < 0.0) {
            if (a > 0) flip = a;
            t = a > 0 ? a - 1 : -1;
          }
          if (flip >= a0 && flip <= a0 + TS) atomicXor(&sNRow[j], 1u << (flip - a0));
          if (t >= a0 && t < a0 + TS) atomicOr(&sRecv[j], 1u << (t - a0));
        }
      } else {
        const uint32_t c = code & 0x7fffu;
        const int la = c % NH, lb = c / NH;
        const int a = a0 - HALO + la, b = b0 - HALO + lb;
        const double t = uno[G.une(a, b)];
        const double v0 = V(a, b - 1), v1 = V(a, b), v2 = V(a, b + 1);
        const double ub = t < 0.5 ? lerp(v0, v1, t + 0.5) : lerp(v1, v2, t - 0.5);
        const double d = ub * lam;
        const bool wall = a == 0 || a == na;
        // every listed unaligned marker belongs to this tile
        // old offset and displacement side by side: the fit reads both
        const size_t e2 = 2 * G.une(a, b);
        ddg[e2] = t;
        ddg[e2 + 1] = wall ? 0.0 : d;
        // walls hold their markers (wall nodes never change colour)
        if (wall) unn[G.une(a, b)] = t;
        cnt.add(C_MARKERS, 1u);
        if (fabs(d) > 0.5) atomicOr(errg, ERRBIT_CFL);
        if (wall && d != 0.0) cnt.add(C_WALL_VIOLATION, 1u);
      }
    }
    // the next tile's colours are fetched while this one computes
    if (it + itStep < itEnd) prefetch(tileAt(it + itStep));
    __syncthreads();
    uint32_t hasm = 0;
    // --- new node colours out; new aligned edges; unaligned work list --------
    writeColours();
    if (tid < NN) {
      // new aligned edges (a,b), a in [a0, a0+15], on row b = b0+tid
      const int j = tid, b = b0 + j;
      const uint32_t valid = (1u << min(TS, max(0, na - a0))) - 1u;
      if (b <= nb && (j < TS || b == nb)) {
        const uint32_t nr = sNRow[j];
        const uint32_t pres = (nr ^ (nr >> 1)) & valid;
        uint32_t m = pres | (sRecv[j] & valid);
        while (m) {
          const int i = __ffs(m) - 1;
          m &= m - 1;
          const int a = a0 + i;
          int keep;
          const int n = T.landers(a, b, &keep);
          if (n == 3) cnt.add(C_THREE_LANDERS, 1u);
          cnt.add(C_ANNIHILATED, (uint32_t)(n - (n & 1)));
          const bool newpres = (pres >> i) & 1u;
          if ((int)newpres != (n & 1)) cnt.add(C_INVARIANT_FAIL, 1u);
          double o = 0.0;
          if (keep >= 0) {
            const double spv = T.spv(keep, b);
            o = keep < a ? spv - 1.0 : (keep > a ? spv + 1.0 : spv);
            if (o < TIE_EPS || 1.0 - o < TIE_EPS) cnt.add(C_TIES, 1u);
          }
          if (newpres) {
            aln[G.ale(a, b)] = o;
            hasm |= DIR == 0 ? maskH(a, b, x0, y0) : maskV(b, a, x0, y0);
          }
        }
      }
    } else if (tid >= 64 && tid < 64 + TS) {
      // new unaligned edges on lines a in [a0, a0+16], row b = b0+j
      const int j = tid - 64, b = b0 + j;
      if (b < nb) {
        const uint32_t lines = (1u << min(NN, max(0, na + 1 - a0))) - 1u;
        uint32_t m = (sNRow[j] ^ sNRow[j + 1]) & lines;
        while (m) {
          const int i = __ffs(m) - 1;
          m &= m - 1;
          const int a = a0 + i;
          const bool own = i < TS || a == na;
          if (a == 0 || a == na) {
            // a wall marker (its offset was copied while advecting)
            if (own) hasm |= DIR == 0 ? maskV(a, b, x0, y0) : maskH(b, a, x0, y0);
          } else if (own) {
            // interior line owned by this tile: one fit job
            sJob[atomicAdd(&sNJob, 1u)] = make_uint2(kinst, (uint32_t)G.une(a, b));
            hasm |= DIR == 0 ? maskV(a, b, x0, y0) : maskH(b, a, x0, y0);
          }
        }
      }
    }
    // centre colours stay where they are (one array); the centre kernel
    // applies rules (1)-(5) to the cells next to this sweep's new markers
    if (hasm) atomicOr(&sHas, hasm);
    __syncthreads();
    if (tid == 0) A.has[gt] = (uint16_t)sHas;
    // keep room for a full tile of jobs
    if (sNJob > JOBCAP - TS * TS) flushJobs();
  }
  __syncthreads();
  if (sNJob) flushJobs();
  if (tid < NCOUNTERS && sCnt[tid]) atomicAdd(&ctrPart(A.ctr)[tid], (unsigned long long)sCnt[tid]);
}

// ---------------------------------------------------------------------------
// Fit kernel: one lane per new unaligned marker of the sweep (the job list),
// so the circle fits of all tiles share full wavefronts. Reads the old state,
// the advected offsets and displacements the sweep wrote and the new colours;
// writes the marker's offset and, per edge, the centre-CV results for the cell
// right of the line (bits 0-1, value + 1) and the cell left of it (bits 2-3).
// ---------------------------------------------------------------------------
// Runs f(k) on the lanes whose grid is k, one grid of the wavefront at a time
// (taken from the first lane still pending), so k is wave-uniform and the
// grid's descriptor stays in scalar registers. Lanes with k == NO_INST idle.
template <class F>
__device__ __forceinline__ void eachGrid(uint32_t k, F f) {
  bool pending = k != NO_INST;
  for (;;) {
    const uint64_t m = __ballot(pending);
    if (m == 0) break;
    const uint32_t k0 = (uint32_t)__builtin_amdgcn_readlane((int)k, (int)(__ffsll((unsigned long long)m) - 1));
    if (pending && k == k0) {
      f(k0);
      pending = false;
    }
  }
}

// The fit on the register window, with every call inlined (the window then
// stays in registers; a call taking it by reference would put it in scratch
// memory).
template <int DIR>
__device__ __attribute__((always_inline, flatten)) double fitWindow(const SweepView &W, int a, int b, int *rR,
                                                                     int *rL, const Counts &cnt) {
  const JobView<DIR> V(W, a, b);
  return newUnaligned(V, a, b, rR, rL, cnt, true, W.line != 0);
}

template <int DIR>
__device__ __forceinline__ void fitJob(const SweepView &W, uint32_t e, const Counts &cnt) {
  GL double *__restrict__ unn = gp(DIR == 0 ? W.nvoff : W.nhoff);
  int a, b;
  if (DIR == 0) { b = (int)(e / (uint32_t)(W.nx + 1)); a = (int)(e % (uint32_t)(W.nx + 1)); }
  else { a = (int)(e / (uint32_t)W.nx); b = (int)(e % (uint32_t)W.nx); }
  int rR, rL;
  const double y = fitWindow<DIR>(W, a, b, &rR, &rL, cnt);
  unn[e] = y;
  gp(W.zr)[e] = (uint8_t)((rR + 1) | ((rL + 1) << 2));
}

// The near tests of tile (tx, ty) from its own and its 8 neighbours' marker
// masks, loaded together (indices clamped into the grid, masks outside it 0):
// nr (the sweeps' set): a marker in the tile or one close enough to a shared
// side or corner; fr (the fraction pass): a marker on an edge of one of the
// tile's cells, its own or one on the left border of the right neighbour or
// the bottom border of the one above (edges on the right and top borders
// belong to those neighbours, except at the walls, where the tile owns them);
// ns (the interface consumers): fr, or a cut cell in the left neighbour's
// last column or the lower neighbour's top row (a face the tile writes lies
// between them and the tile's cells; every other tile has equal C on both
// sides of all its faces).
struct NearTests {
  bool nr, fr, ns;
};
__device__ __forceinline__ NearTests nearTests(const uint16_t *__restrict__ has, int tx, int ty, int ntx, int nty) {
  auto H = [&](int dx, int dy) -> uint32_t {
    const int x = tx + dx, y = ty + dy;
    const bool in = x >= 0 && y >= 0 && x < ntx && y < nty;
    const uint32_t v = has[min(max(y, 0), nty - 1) * ntx + min(max(x, 0), ntx - 1)];
    return in ? v : 0u;
  };
  const uint32_t c = H(0, 0), l = H(-1, 0), r = H(1, 0), d = H(0, -1), u = H(0, 1);
  const uint32_t ld = H(-1, -1), rd = H(1, -1), lu = H(-1, 1), ru = H(1, 1);
  NearTests t;
  t.nr = ((c & M_ANY) | (l & M_R) | (r & M_L) | (d & M_T) | (u & M_B) | (ld & M_RT) | (rd & M_LT) | (lu & M_RB) |
          (ru & M_LB)) != 0u;
  t.fr = ((c & M_ANY) | (r & M_L0) | (u & M_B0)) != 0u;
  t.ns = t.fr || ((l & M_R1) | (d & M_T1)) != 0u;
  return t;
}

constexpr int CPT = 8;  // tiles per thread in the compaction

// nearPrev bits: 0 near at the latest compaction, 1 near at the one before.
// After a sweep the latest becomes the one before; a compaction without a
// sweep in between (grids added or removed) keeps it. Active tiles of grids
// whose next sweep runs along x go to the front of the active list, the others
// to its back.
template <bool ONE>
__device__ void compactBlock(const CompactArgs &C, uint32_t blk) {
  __shared__ uint32_t sA[256], sB[256], sN[256], sF[256];
  __shared__ uint32_t sBaseA, sBaseB, sBaseN, sBaseF;
  const int tid = threadIdx.x;
  if (blk == 0 && tid == 0) {
    // the other slot's list counts start the next compaction from zero, and
    // this slot's job counts the next sweep (the fits and centre colours of the
    // sweep before still read the other slot's job counts)
    uint32_t *other = C.counts + NSLOT * (C.slot ^ 1), *mine = C.counts + NSLOT * C.slot;
    other[CNT_ACT_X] = 0;
    other[CNT_ACT_Y] = 0;
    other[CNT_NEAR] = 0;
    other[CNT_FRAC] = 0;
    for (uint32_t q = 0; q < NJQ; q++) {
      mine[CNT_JOBS_X + CNT_LINE * q] = 0;
      mine[CNT_JOBS_Y + CNT_LINE * q] = 0;
    }
  }
  const uint32_t base = (blk * blockDim.x + tid) * CPT;
  uint32_t actBits = 0, dirBits = 0, nearBits = 0, fracBits = 0;
  uint32_t kq[CPT];
  // one tile's lists and bookkeeping from its tests, history and colour
  auto finish = [&](int q, uint32_t t, const Inst &I, NearTests nt, uint32_t pv, int colour) {
    const uint32_t prev = C.afterSweep ? (pv & 1u) : ((pv >> 1) & 1u);
    const bool act = nt.nr || prev;
    C.nearPrev[t] = (uint8_t)((nt.nr ? 1u : 0u) | (prev << 1));
    C.tinfo[t] = (uint8_t)((nt.ns ? TI_NEAR : 0) | (nt.fr ? TI_FRAC : 0) | (colour ? TI_COLOUR : 0));
    actBits |= (uint32_t)act << q;
    dirBits |= (uint32_t)(act && sweep_dir(I, C.stepNo, C.phase) == 1) << q;
    nearBits |= (uint32_t)nt.ns << q;
    fracBits |= (uint32_t)nt.fr << q;
  };
  if (ONE) {
    // one grid: every load of a group of the thread's tiles first (indices
    // clamped into the tile range), then the tests and stores
    const Inst &I = C.one;
    constexpr int CG = 4;
    static_assert(CPT % CG == 0, "whole groups");
#pragma unroll
    for (int q0 = 0; q0 < CPT; q0 += CG) {
      NearTests nt[CG];
      uint32_t pv[CG];
      int colour[CG];
#pragma unroll
      for (int k = 0; k < CG; k++) {
        const uint32_t t = min(base + q0 + k, C.ntiles - 1u);
        const uint32_t lt = t - I.tile0;
        const int tx = (int)(lt % (uint32_t)I.ntx), ty = (int)(lt / (uint32_t)I.ntx);
        nt[k] = nearTests(C.has + I.tile0, tx, ty, I.ntx, I.nty);
        pv[k] = C.nearPrev[t];
        colour[k] = colAt(gp(I.col[C.cur]), I.nx, tx * TS, ty * TS);
      }
#pragma unroll
      for (int k = 0; k < CG; k++) {
        const uint32_t t = base + q0 + k;
        kq[q0 + k] = 0;
        if (t < C.ntiles) finish(q0 + k, t, I, nt[k], pv[k], colour[k]);
      }
    }
  } else {
    for (int q = 0; q < CPT; q++) {
      const uint32_t t = base + q;
      kq[q] = 0;
      if (t >= C.ntiles) break;
      const uint32_t k = C.tileInst[t];
      kq[q] = k;
      if (k == NO_INST) continue;
      const Inst &I = C.inst[k];
      const uint32_t lt = t - I.tile0;
      const int tx = (int)(lt % (uint32_t)I.ntx), ty = (int)(lt / (uint32_t)I.ntx);
      finish(q, t, I, nearTests(C.has + I.tile0, tx, ty, I.ntx, I.nty), C.nearPrev[t],
             colAt(gp(I.col[C.cur]), I.nx, tx * TS, ty * TS));
    }
  }
  // exclusive block scan of the per-thread counts
  const uint32_t cb = __popc(dirBits), ca = __popc(actBits) - cb, cn = __popc(nearBits), cf = __popc(fracBits);
  sA[tid] = ca;
  sB[tid] = cb;
  sN[tid] = cn;
  sF[tid] = cf;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t xa = tid >= off ? sA[tid - off] : 0, xb = tid >= off ? sB[tid - off] : 0,
                   xn = tid >= off ? sN[tid - off] : 0, xf = tid >= off ? sF[tid - off] : 0;
    __syncthreads();
    sA[tid] += xa;
    sB[tid] += xb;
    sN[tid] += xn;
    sF[tid] += xf;
    __syncthreads();
  }
  uint32_t *cs = C.counts + NSLOT * C.slot;
  if (tid == 255) {
    sBaseA = sA[255] ? atomicAdd(&cs[CNT_ACT_X], sA[255]) : 0;
    sBaseB = sB[255] ? atomicAdd(&cs[CNT_ACT_Y], sB[255]) : 0;
    sBaseN = sN[255] ? atomicAdd(&cs[CNT_NEAR], sN[255]) : 0;
    sBaseF = sF[255] ? atomicAdd(&cs[CNT_FRAC], sF[255]) : 0;
  }
  __syncthreads();
  uint32_t pa = sBaseA + sA[tid] - ca, pb = sBaseB + sB[tid] - cb, pn = sBaseN + sN[tid] - cn,
           pf = sBaseF + sF[tid] - cf;
  for (int q = 0; q < CPT; q++) {
    if (actBits >> q & 1) {
      if (dirBits >> q & 1) C.actList[C.ntiles - 1u - pb++] = make_uint2(base + q, kq[q]);
      else C.actList[pa++] = make_uint2(base + q, kq[q]);
    }
    if (nearBits >> q & 1) C.nearList[pn++] = make_uint2(base + q, kq[q]);
    if (fracBits >> q & 1) C.fracList[pf++] = make_uint2(base + q, kq[q]);
  }
}

template <bool ONE>
__global__ __launch_bounds__(256) void k_compact(CompactArgs C) {
  compactBlock<ONE>(C, blockIdx.x);
}

// The same launch also runs the compaction of the state this sweep produced
// (it reads only what the sweep wrote): workgroups [0, compactBlocks) compact,
// the others fit, so the compaction's latency hides under the fits.
template <int DIR, bool ONE>
__global__ __launch_bounds__(256) void k_fit(SweepArgs A, const Inst *__restrict__ inst, CompactArgs C,
                                             uint32_t compactBlocks) {
  if (blockIdx.x < compactBlocks) {
    compactBlock<ONE>(C, blockIdx.x);
    return;
  }
  __shared__ uint32_t sCnt[NCOUNTERS];
  const int tid = threadIdx.x;
  if (tid < NCOUNTERS) sCnt[tid] = 0;
  __syncthreads();
  const Counts cnt{sCnt};
  const JobIndex J(A.njobs, A.jobQ, A.jobRegion);
  const uint32_t nj = J.total();
  const uint32_t fb = blockIdx.x - compactBlocks;
  const uint32_t stride = (gridDim.x - compactBlocks) * blockDim.x;
  for (uint32_t w0 = fb * blockDim.x; w0 < nj; w0 += stride) {
    const uint32_t w = w0 + tid, e = J.entry(w);
    const uint2 jb = w < nj ? A.jobs[DIR == 0 ? e : A.jobTop - 1u - e] : make_uint2(NO_INST, 0u);
    if (ONE) {
      if (w < nj) fitJob<DIR>(A.one, jb.y, cnt);
    } else {
      eachGrid(jb.x, [&](uint32_t k) { fitJob<DIR>(sweep_view(inst[k], A.cur, DIR, A.u, A.v, 0.0), jb.y, cnt); });
    }
  }
  __syncthreads();
  if (tid < NCOUNTERS && sCnt[tid]) atomicAdd(&ctrPart(A.ctr)[tid], (unsigned long long)sCnt[tid]);
}

// Centre kernel: rules (1)-(5) of Sec. 2.3 for the cells next to new
// unaligned markers. A cell takes the result of the marker on its left edge,
// else of the one on its right edge, else keeps its centre colour (already
// carried over by the sweep). The job on line a settles cell a and, when line
// a-1 holds no job, cell a-1.
template <int DIR>
__device__ __forceinline__ void centreJob(const SweepView &W, uint32_t e, const Counts &cnt) {
  const GMap<DIR> G(W.nx, W.ny);
  const int na = G.na;
  const GL uint16_t *__restrict__ ncol = gp(W.ncol);
  GL uint8_t *__restrict__ ncen = gp(W.ncen);
  const GL uint8_t *__restrict__ zr = gp(W.zr);
  auto newC = [&](int a, int b) -> int { return G.colour(ncol, a, b); };
  int a, b;
  if (DIR == 0) { b = (int)(e / (uint32_t)(W.nx + 1)); a = (int)(e % (uint32_t)(W.nx + 1)); }
  else { a = (int)(e / (uint32_t)W.nx); b = (int)(e % (uint32_t)W.nx); }
  auto isJob = [&](int l) -> bool { return l > 0 && l < na && newC(l, b) != newC(l, b + 1); };
  auto settle = [&](int c, int left, int right) {
    int cc = -1;
    if (left >= 0) {
      cc = left;
      cnt.add(C_CV_SET, 1u);
      if (right >= 0 && right != left) cnt.add(C_CV_CONFLICT, 1u);
    } else if (right >= 0) {
      cc = right;
      cnt.add(C_CV_SET, 1u);
    } else {
      const int k0 = newC(c, b), k1 = newC(c + 1, b), k2 = newC(c + 1, b + 1), k3 = newC(c, b + 1);
      if (k0 != k1 && k1 != k2 && k3 != k2 && k0 != k3) cnt.add(C_CV_UNRESOLVED, 1u);
    }
    if (cc >= 0) ncen[G.cell(c, b)] = (uint8_t)cc;
  };
  const uint32_t z = zr[e];
  // cell a, right of line a
  {
    const int right = isJob(a + 1) ? (int)((zr[G.une(a + 1, b)] >> 2) & 3u) - 1 : -1;
    settle(a, (int)(z & 3u) - 1, right);
  }
  // cell a-1, left of line a, when its own left line holds no job
  if (!isJob(a - 1)) settle(a - 1, -1, (int)((z >> 2) & 3u) - 1);
}

template <int DIR, bool ONE>
__global__ __launch_bounds__(256) void k_centre(SweepArgs A, const Inst *__restrict__ inst) {
  __shared__ uint32_t sCnt[NCOUNTERS];
  const int tid = threadIdx.x;
  if (tid < NCOUNTERS) sCnt[tid] = 0;
  __syncthreads();
  const Counts cnt{sCnt};
  const JobIndex J(A.njobs, A.jobQ, A.jobRegion);
  const uint32_t nj = J.total();
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t w0 = blockIdx.x * blockDim.x; w0 < nj; w0 += stride) {
    const uint32_t w = w0 + tid, e = J.entry(w);
    const uint2 jb = w < nj ? A.jobs[DIR == 0 ? e : A.jobTop - 1u - e] : make_uint2(NO_INST, 0u);
    if (ONE) {
      if (w < nj) centreJob<DIR>(A.one, jb.y, cnt);
    } else {
      eachGrid(jb.x, [&](uint32_t k) { centreJob<DIR>(sweep_view(inst[k], A.cur, DIR, A.u, A.v, 0.0), jb.y, cnt); });
    }
  }
  __syncthreads();
  if (tid < NCOUNTERS && sCnt[tid]) atomicAdd(&ctrPart(A.ctr)[tid], (unsigned long long)sCnt[tid]);
}

// ---------------------------------------------------------------------------
// Tile bookkeeping: tiles of a newly placed grid (owner, marker masks), tiles
// of a removed grid, and the per-sweep compaction into the active list (near
// now or near before the previous compaction) and the near list. Each
// compaction workgroup scans 1024 tiles and reserves its list slots with one
// atomic per list.
// ---------------------------------------------------------------------------
__global__ void k_init_tiles(const Inst *__restrict__ inst, uint32_t kinst, uint32_t cur, uint32_t *tileInst,
                             uint16_t *has, uint8_t *nearPrev) {
  const Inst &I = inst[kinst];
  const uint32_t lt = blockIdx.x;
  if (lt >= (uint32_t)(I.ntx * I.nty)) return;
  const int nx = I.nx, ny = I.ny;
  const int tx = (int)(lt % (uint32_t)I.ntx), ty = (int)(lt / (uint32_t)I.ntx);
  const int x0 = tx * TS, y0 = ty * TS;
  const GL uint16_t *__restrict__ col = gp(I.col[cur]);
  __shared__ uint32_t sh;
  if (threadIdx.x == 0) sh = 0;
  __syncthreads();
  uint32_t m = 0;
  for (int k = threadIdx.x; k < NN * NN; k += blockDim.x) {
    const int li = k % NN, lj = k / NN;
    const int i = x0 + li, j = y0 + lj;
    if (i > nx || j > ny) continue;
    const bool ownI = li < TS || i == nx;
    const bool ownJ = lj < TS || j == ny;
    const int c = colAt(col, nx, i, j);
    if (i < nx && li < TS && ownJ && c != colAt(col, nx, i + 1, j)) m |= maskH(i, j, x0, y0);
    if (j < ny && lj < TS && ownI && c != colAt(col, nx, i, j + 1)) m |= maskV(i, j, x0, y0);
  }
  if (m) atomicOr(&sh, m);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t gt = I.tile0 + lt;
    has[gt] = (uint16_t)sh;
    nearPrev[gt] = 0;
    tileInst[gt] = kinst;
  }
}

__global__ void k_clear_tiles(uint32_t *tileInst, uint16_t *has, uint8_t *nearPrev, uint8_t *tinfo, uint32_t tile0,
                              uint32_t n) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  tileInst[tile0 + t] = NO_INST;
  has[tile0 + t] = 0;
  nearPrev[tile0 + t] = 0;
  tinfo[tile0 + t] = TI_DEAD;
}

// ---------------------------------------------------------------------------
// Volume fraction and height-function curvature.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int mirrorCell(int k, int n) { return k < 0 ? -1 - k : (k >= n ? 2 * n - 1 - k : k); }
__device__ __forceinline__ int mirrorNode(int k, int n) { return k < 0 ? -k : (k > n ? 2 * n - k : k); }
// halo slots farther than one reflection (grids narrower than the halo) are
// clamped into the grid; the stencils never read them
__device__ __forceinline__ int haloCell(int k, int n) {
  k = mirrorCell(k, n);
  return k < 0 ? 0 : (k >= n ? n - 1 : k);
}

struct FracCtx {
  int nx, ny;
  const GL uint16_t *__restrict__ col;
  const GL uint8_t *__restrict__ cen;
  const GL double *__restrict__ hoff;
  const GL double *__restrict__ voff;
};

// area of colour 1 in cell (i,j) from its corner colours (BL, BR, TR, TL)
__device__ double cellFraction(const FracCtx &P, int i, int j, int kBL, int kBR, int kTR, int kTL) {
  const size_t W1 = (size_t)P.nx + 1;
  const bool pb = kBL != kBR, pr = kBR != kTR, pt = kTL != kTR, pl = kBL != kTL;
  const int n = (int)pb + (int)pr + (int)pt + (int)pl;
  if (n == 0) return (double)kBL;
  const double hb = pb ? P.hoff[(size_t)j * P.nx + i] : 0.0;
  const double ht = pt ? P.hoff[(size_t)(j + 1) * P.nx + i] : 0.0;
  const double vl = pl ? P.voff[(size_t)j * W1 + i] : 0.0;
  const double vr = pr ? P.voff[(size_t)j * W1 + i + 1] : 0.0;
  if (n == 2) {
    // the chord cuts off a corner triangle (markers on two adjacent edges) or
    // splits the cell into two trapezoids (opposite edges): the area of the
    // part holding corner k, which has k's colour (the same area as the
    // polygon of the colour-1 corners and the markers, up to rounding)
    double area;
    int k;
    if (pb && pt) {
      area = 0.5 * (hb + ht);
      k = kBL;
    } else if (pl && pr) {
      area = 0.5 * (vl + vr);
      k = kBL;
    } else if (pb) {
      if (pl) {
        area = 0.5 * (hb * vl);
        k = kBL;
      } else {
        area = 0.5 * ((1.0 - hb) * vr);
        k = kBR;
      }
    } else if (pl) {
      area = 0.5 * (ht * (1.0 - vl));
      k = kTL;
    } else {
      area = 0.5 * ((1.0 - ht) * (1.0 - vr));
      k = kTR;
    }
    return k ? area : 1.0 - area;
  }
  // four markers: isolated corner triangles keep their corner colour, the
  // central region carries the centre colour
  const int cen = P.cen[(size_t)j * P.nx + i];
  const double tBL = 0.5 * (hb * vl), tBR = 0.5 * ((1.0 - hb) * vr);
  const double tTR = 0.5 * ((1.0 - vr) * (1.0 - ht)), tTL = 0.5 * (ht * (1.0 - vl));
  const double s = (kBL != cen) ? tBL + tTR : tBR + tTL;
  return cen ? 1.0 - s : s;
}

// Heights along columns (rows == 0) or rows (rows == 1) around cell (i,j);
// returns 1 and kappa on success.
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

// Integer node-colour gradient around cell (i,j) over the 4x4 nodes
// i-1..i+2, j-1..j+2 (mirrored across walls); points into colour 1.
template <class NodeAt>
__device__ __forceinline__ void nodeGradient(int i, int j, int nx, int ny, NodeAt nodeAt, int *gx, int *gy) {
  auto nodeC = [&](int a, int b) -> int { return nodeAt(mirrorNode(a, nx), mirrorNode(b, ny)); };
  int ncx = 0, ncy = 0;
  for (int m = j - 1; m <= j + 2; m++) ncx += nodeC(i + 2, m) + nodeC(i + 1, m) - nodeC(i, m) - nodeC(i - 1, m);
  for (int l = i - 1; l <= i + 2; l++) ncy += nodeC(l, j + 2) + nodeC(l, j + 1) - nodeC(l, j) - nodeC(l, j - 1);
  *gx = ncx;
  *gy = ncy;
}

// Where no height is valid: the least-squares parabola through the markers on
// the edges of the 5x5 cells around (i,j), in the frame of the node-colour
// gradient (gx, gy) (pointing into colour 1); kappa = 2c / (1 + b^2)^(3/2) / h.
// Points are summed H edges first (rows y, then x), then V edges. node(x,y),
// hoffAt(x,y) and voffAt(x,y) read the state in the window x in [i-2, i+3],
// y in [j-2, j+3]. The present edges are found first as a bit mask (bit
// q*5+p the H edge (i-2+p, j-2+q), bit 30+q*6+p the V edge (i-2+p, j-2+q)),
// then summed in ascending bit order, which is the order above: a wavefront
// runs as many rounds as its busiest lane has markers, not one per edge.
template <class GetN, class GetH, class GetV>
__device__ bool ghfFit(int nx, int ny, double h, int i, int j, int gx, int gy, GetN node, GetH hoffAt, GetV voffAt,
                       double *kap) {
  if (gx == 0 && gy == 0) return false;
  // node colours of the 6x6 window, bit q*6+p = node(i-2+p, j-2+q)
  unsigned long long nb = 0;
#pragma unroll
  for (int q = 0; q < 6; q++)
#pragma unroll
    for (int p = 0; p < 6; p++) nb |= (unsigned long long)(node(i - 2 + p, j - 2 + q) & 1) << (q * 6 + p);
  unsigned long long em = 0;
#pragma unroll
  for (int q = 0; q < 6; q++)
#pragma unroll
    for (int p = 0; p < 5; p++) {
      const int x = i - 2 + p, y = j - 2 + q;
      const bool on = x >= 0 && x < nx && y >= 0 && y <= ny && ((nb >> (q * 6 + p)) & 1) != ((nb >> (q * 6 + p + 1)) & 1);
      em |= (unsigned long long)on << (q * 5 + p);
    }
#pragma unroll
  for (int q = 0; q < 5; q++)
#pragma unroll
    for (int p = 0; p < 6; p++) {
      const int x = i - 2 + p, y = j - 2 + q;
      const bool on = x >= 0 && x <= nx && y >= 0 && y < ny && ((nb >> (q * 6 + p)) & 1) != ((nb >> (q * 6 + p + 6)) & 1);
      em |= (unsigned long long)on << (30 + q * 6 + p);
    }
  const double gl = sqrt((double)gx * (double)gx + (double)gy * (double)gy);
  const double nX = (double)gx / gl, nY = (double)gy / gl;
  const double xc = i + 0.5, yc = j + 0.5;
  double S0 = 0.0, S1 = 0.0, S2 = 0.0, S3 = 0.0, S4 = 0.0, T0 = 0.0, T1 = 0.0, T2 = 0.0;
  while (em) {
    const int b = __ffsll((long long)em) - 1;
    em &= em - 1;
    double px, py;
    if (b < 30) {
      const int x = i - 2 + b % 5, y = j - 2 + b / 5;
      px = x + hoffAt(x, y);
      py = (double)y;
    } else {
      const int x = i - 2 + (b - 30) % 6, y = j - 2 + (b - 30) / 6;
      px = (double)x;
      py = y + voffAt(x, y);
    }
    const double dx = px - xc, dy = py - yc;
    const double X = dx * (-nY) + dy * nX;
    const double Y = dx * nX + dy * nY;
    const double X2 = X * X;
    S0 += 1.0;
    S1 += X;
    S2 += X2;
    S3 += X2 * X;
    S4 += X2 * X2;
    T0 += Y;
    T1 += X * Y;
    T2 += X2 * Y;
  }
  if (S0 < 3.0) return false;
  const double det = S0 * (S2 * S4 - S3 * S3) - S1 * (S1 * S4 - S3 * S2) + S2 * (S1 * S3 - S2 * S2);
  if (!(det > 1e-10 * (S0 * S2 * S4))) return false;
  const double db = S0 * (T1 * S4 - S3 * T2) - T0 * (S1 * S4 - S3 * S2) + S2 * (S1 * T2 - T1 * S2);
  const double dc = S0 * (S2 * T2 - T1 * S3) - S1 * (S1 * T2 - T1 * S2) + T0 * (S1 * S3 - S2 * S2);
  const double b = db / det, cc = dc / det;
  const double g = 1.0 + b * b;
  *kap = (2.0 * cc) / (h * g * sqrt(g));
  return true;
}

// Fraction and/or curvature of every grid in one launch. Workgroups
// [0, nearBlocks) take the near tiles of the list (static stride): node
// colours of the tile plus halo in LDS; C, marker count and BL colour of every
// halo cell (mirrored across walls), polygons only where markers are; then C
// and/or kappa of the tile's cells (one per thread). Cells whose heights fail
// in both directions are handed to k_ghf (one entry per 64 cells that have
// any), which keeps the rare parabola fit out of this kernel's register
// budget. Workgroups are 256 threads, 8 resident per CU; the first ones (5.5
// per CU, so that the fill runs beside them) take the near tiles. Every later
// workgroup fills 16 consecutive global
// tiles: cells of tiles that are neither near nor unowned get their tile's
// colour as C and zero curvature, one 8-byte store per lane and row, lanes
// along a grid row. MODE 1: C only; 2: kappa from the caller's C; 3: both.
constexpr int FRAC_BS = 256;
constexpr int NEAR_ENT = 16;  // tile entries a near workgroup keeps in LDS
constexpr int NS_FILL_TILES = 16;

// A grid whose rows are not whole lines (nx not a multiple of 16, or an
// output not line-aligned), and every grid of several (each grid's arrays
// start on a 256-byte boundary of the packed fields): the array seen with a virtual row pitch P = nx
// rounded up to 16, which makes every virtual row start on a line boundary
// (given a line-aligned base), and filled like the per-tile fill below: fill
// workgroup f takes 256-element run f % nseg of virtual rows 16 (f / nseg) ..
// + 15, a lane one virtual column. A lane's element e then steps by P per
// virtual row, and its real (x, y) = divmod(e, nx) by Q = P / nx rows and
// R = P % nx columns, wrapping at most once into the next row (R < nx; Q is 1
// for rows of 16 cells or more, and up to 4 for rows narrower than 8), so it
// needs no division past the first; each wavefront store covers whole lines. The fill shares the CUs
// with the near tiles, so its work per store is what counts: the linear
// fill's per-element division cost the 8190^2 fraction call ~20 us.
template <int MODE>
__device__ __forceinline__ void fracPitchFill(const FracArgs &A, const Inst &I, uint32_t f) {
  const int nx = I.nx, ny = I.ny;
  const size_t n = (size_t)nx * (size_t)ny;
  const size_t P = ((size_t)nx + 15) & ~(size_t)15;
  const uint32_t nseg = (uint32_t)((P + 255) / 256);
  const size_t g = f / nseg;
  const uint32_t vc = (f % nseg) * 256u + threadIdx.x;
  if (vc >= P) return;  // lanes past the last run's virtual row (no barrier follows)
  size_t e = g * 16 * P + vc;
  if (e >= n) return;
  const int Q = (int)((uint32_t)P / (uint32_t)nx), R = (int)P - Q * nx;
  int y = (int)(e / (size_t)nx), x = (int)(e - (size_t)y * (size_t)nx);
  // every element's tile info first, then the stores
  uint8_t ti[16];
  size_t ee[16];
#pragma unroll
  for (int i = 0; i < 16; i++) {
    ee[i] = e;
    ti[i] = e < n ? A.tinfo[I.tile0 + (uint32_t)(y >> 4) * (uint32_t)I.ntx + (uint32_t)(x >> 4)] : (uint8_t)TI_FRAC;
    e += P;
    y += Q;
    x += R;
    if (x >= nx) {
      x -= nx;
      y += 1;
    }
  }
  double *Cp = (MODE & 1) ? A.Cout + I.coff : nullptr;
  double *Kp = (MODE & 2) ? A.Kout + I.koff : nullptr;
#pragma unroll
  for (int i = 0; i < 16; i++) {
    if (ti[i] & TI_FRAC) continue;
    if (MODE & 1) __builtin_nontemporal_store((ti[i] & TI_COLOUR) ? 1.0 : 0.0, &Cp[ee[i]]);
    if (MODE & 2) __builtin_nontemporal_store(0.0, &Kp[ee[i]]);
  }
}

// One grid whose 16-cell tile rows are whole 128-byte lines (nx a multiple of
// 16, both outputs line-aligned): a fill workgroup takes 16 consecutive tiles
// of a tile row, a lane a column, and stores 16 rows. Tiles of a row start at
// FILL_CHUNK / (16 * 16) = 16 tiles per chunk, so chunk f covers tiles
// 16 f .. 16 f + 15 of the grid.
template <int MODE>
__device__ __forceinline__ bool wholeLineRows(const FracArgs &A, const Inst &I) {
  if ((I.nx & 15) != 0) return false;
  uintptr_t al = 0;
  if (MODE & 1) al |= (uintptr_t)(A.Cout + I.coff);
  if (MODE & 2) al |= (uintptr_t)(A.Kout + I.koff);
  return (al & 127u) == 0;
}
template <int MODE>
__device__ __forceinline__ void fracTileFill(const FracArgs &A, const Inst &I, uint32_t f) {
  constexpr uint32_t TPB = FILL_CHUNK / (TS * TS);
  static_assert(TPB * TS == FRAC_BS, "a lane per column of the chunk's tiles");
  const uint32_t lt = f * TPB + threadIdx.x / TS;
  if (lt >= (uint32_t)(I.ntx * I.nty)) return;
  const uint8_t ti = A.tinfo[I.tile0 + lt];
  if (ti & TI_FRAC) return;
  const int tx = (int)(lt % (uint32_t)I.ntx), ty = (int)(lt / (uint32_t)I.ntx);
  const int nx = I.nx, x = tx * TS + (int)(threadIdx.x % TS), rows = min(TS, I.ny - ty * TS);
  const double c = (ti & TI_COLOUR) ? 1.0 : 0.0;
  double *Cp = (MODE & 1) ? A.Cout + I.coff + (size_t)(ty * TS) * nx + x : nullptr;
  double *Kp = (MODE & 2) ? A.Kout + I.koff + (size_t)(ty * TS) * nx + x : nullptr;
#pragma unroll 4
  for (int r = 0; r < rows; r++) {
    if (MODE & 1) __builtin_nontemporal_store(c, &Cp[(size_t)r * nx]);
    if (MODE & 2) __builtin_nontemporal_store(0.0, &Kp[(size_t)r * nx]);
  }
}

template <int MODE, bool ONE>
__global__ __launch_bounds__(FRAC_BS, 8) void k_frac_curv(FracArgs A, const Inst *__restrict__ inst,
                                                       const uint32_t *__restrict__ tileInst) {
  constexpr int W = TS + 6;  // halo cells per side
  constexpr int WN = W + 1;  // halo nodes per side
  const int tid = threadIdx.x;
  if ((int)blockIdx.x >= A.nearBlocks) {
    // --- uniform cells: linear fill -------------------------------------------
    uint32_t f = blockIdx.x - (uint32_t)A.nearBlocks;
    if (ONE && wholeLineRows<MODE>(A, A.one)) {
      fracTileFill<MODE>(A, A.one, f);
    } else if (ONE) {
      fracPitchFill<MODE>(A, A.one, f);
    } else {
      // the grid of chunk f: the last table entry starting at or before it
      uint32_t lo = 0, hi = A.fillGrids;
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (A.fillTab[mid].x <= f) lo = mid;
        else hi = mid;
      }
      const uint2 t = A.fillTab[lo];
      fracPitchFill<MODE>(A, inst[t.y], f - t.x);
    }
    return;
  }
  static_assert(TS * TS % FRAC_BS == 0 && FRAC_BS % 64 == 0, "whole cells per thread, whole wavefronts");
  __shared__ uint8_t sNode[WN][WN];
  __shared__ double sC[W][W];
  __shared__ uint8_t sN[W][W];
  __shared__ uint8_t sB[W][W];
  __shared__ uint32_t sCnt[2];
  __shared__ uint2 sEnt[NEAR_ENT];
  if (tid < 2) sCnt[tid] = 0;
  if ((MODE & 2) && blockIdx.x == 0 && tid == 0) *A.ghfClear = 0u;  // the next curvature launch's count
  uint32_t interf = 0, hffail = 0;
  const uint32_t ntile = *A.count;
  uint32_t ntiles_done = 0;
  // node colours of the tile plus halo (nodes x0-3 .. x0+19, rows y0-3 ..
  // y0+19: 3 x 3 blocks of the bit plane): lane k < 3 WN holds the word of
  // halo row k / 3 in block column tx-1 + k % 3, fetched for the next tile
  // while this one computes (clamped indices; words of rows or blocks outside
  // the grid are zeroed when staged)
  static_assert(3 * WN <= FRAC_BS && 3 <= TS && WN - 3 <= 2 * TS, "staging words");
  __shared__ uint64_t sBlk[WN];
  uint32_t pn = 0;
  bool pin = false;
  // this workgroup's first tile entries, read once: the colour prefetch of
  // the next tile then needs no load of its entry first
  if (tid < NEAR_ENT) {
    const uint32_t it = blockIdx.x + (uint32_t)tid * (uint32_t)A.nearBlocks;
    if (it < ntile) sEnt[tid] = A.list[it];
  }
  __syncthreads();
  auto entry = [&](uint32_t it, uint32_t n) -> uint2 {
    const uint2 e = n < (uint32_t)NEAR_ENT ? sEnt[n] : A.list[it];
    return make_uint2(uni(e.x), uni(e.y));
  };
  auto prefetch = [&](uint2 te) {
    const Inst &I = ONE ? A.one : inst[te.y];
    const int nx = I.nx, ny = I.ny;
    const uint32_t lt = te.x - I.tile0;
    const int tx = (int)(lt % (uint32_t)I.ntx), y0 = (int)(lt / (uint32_t)I.ntx) * TS;
    const GL uint16_t *col = gp(I.col[A.cur]);
    const int k = min(tid, 3 * WN - 1), y = y0 - 3 + k / 3, bx = tx - 1 + k % 3, nbx = cb_nbx(nx);
    pin = y >= 0 && y <= ny && bx >= 0 && bx < nbx;
    pn = col[cb_word(nx, min(max(bx, 0), nbx - 1) * TS, min(max(y, 0), ny))];
  };
  if (blockIdx.x < ntile) prefetch(entry(blockIdx.x, 0));
  uint32_t n = 0;  // this workgroup's tile count
  for (uint32_t it = blockIdx.x; it < ntile; it += (uint32_t)A.nearBlocks, n++) {
    __syncthreads();
    const uint2 te = entry(it, n);
    const Inst &I = ONE ? A.one : inst[te.y];
    const int nx = I.nx, ny = I.ny;
    const FracCtx P{nx, ny, gp(I.col[A.cur]), gp(I.cen[A.cur]), gp(I.hoff[A.cur]), gp(I.voff[A.cur])};
    const uint32_t lt = te.x - I.tile0;
    const int tx = (int)(lt % (uint32_t)I.ntx), ty = (int)(lt / (uint32_t)I.ntx);
    const int x0 = tx * TS, y0 = ty * TS;
    // every cell's 4x4 gradient nodes lie inside the grid
    const bool inner = x0 >= 1 && y0 >= 1 && x0 + TS + 1 <= nx && y0 + TS + 1 <= ny;
    ntiles_done++;
    if (tid < 3 * WN) ((uint16_t *)&sBlk[tid / 3])[tid % 3] = pin ? (uint16_t)pn : (uint16_t)0;
    __syncthreads();
    // halo node (x0-3+hx, y0-3+hy) is bit TS-3+hx of row hy's words
    for (int k = tid; k < WN * WN; k += FRAC_BS) {
      const int hx = k % WN, hy = k / WN;
      sNode[hy][hx] = (uint8_t)((sBlk[hy] >> (TS - 3 + hx)) & 1u);
    }
    __syncthreads();
    for (int k = tid; k < W * W; k += blockDim.x) {
      const int li = k % W, lj = k / W;
      const int gx = x0 - 3 + li, gy = y0 - 3 + lj;
      int kBL, kBR, kTR, kTL, gi, gj;
      if (gx >= 0 && gy >= 0 && gx < nx && gy < ny) {
        gi = gx;
        gj = gy;
        kBL = sNode[lj][li];
        kBR = sNode[lj][li + 1];
        kTR = sNode[lj + 1][li + 1];
        kTL = sNode[lj + 1][li];
      } else {
        // ghost cell: the data of its mirror cell
        gi = haloCell(gx, nx);
        gj = haloCell(gy, ny);
        kBL = colAt(P.col, nx, gi, gj);
        kBR = colAt(P.col, nx, gi + 1, gj);
        kTR = colAt(P.col, nx, gi + 1, gj + 1);
        kTL = colAt(P.col, nx, gi, gj + 1);
      }
      const int nm = (kBL != kBR) + (kBR != kTR) + (kTL != kTR) + (kBL != kTL);
      double c;
      if (MODE == 2) c = A.Cin[I.coff + (size_t)gj * nx + gi];
      else c = cellFraction(P, gi, gj, kBL, kBR, kTR, kTL);
      sC[lj][li] = c;
      sN[lj][li] = (uint8_t)nm;
      sB[lj][li] = (uint8_t)kBL;
    }
    // the next tile's colours are fetched while this one's heights run
    if (it + (uint32_t)A.nearBlocks < ntile) prefetch(entry(it + (uint32_t)A.nearBlocks, n + 1));
    __syncthreads();
#pragma unroll 1
    for (int r = 0; r < TS * TS / FRAC_BS; r++) {
      const int k = tid + FRAC_BS * r;
      const int li = k % TS, lj = k / TS;
      const int i = x0 + li, j = y0 + lj;
      const bool in = i < nx && j < ny;
      const size_t id = (size_t)j * nx + i;
      if ((MODE & 1) && in) A.Cout[I.coff + id] = sC[lj + 3][li + 3];
      if (MODE & 2) {
        bool fallback = false;
        if (in) {
          double kap = 0.0;
          if (sN[lj + 3][li + 3] >= 2) {
            interf++;
            int ncx = 0, ncy = 0;
            if (inner) {
              // nodes i-1..i+2, j-1..j+2 are all inside the grid: the same sums
              // without mirroring (node (i-1, j-1) is slot (li+2, lj+2))
#pragma unroll
              for (int m = 0; m < 4; m++)
                ncx += sNode[lj + 2 + m][li + 5] + sNode[lj + 2 + m][li + 4] - sNode[lj + 2 + m][li + 3] -
                       sNode[lj + 2 + m][li + 2];
#pragma unroll
              for (int l = 0; l < 4; l++)
                ncy += sNode[lj + 5][li + 2 + l] + sNode[lj + 4][li + 2 + l] - sNode[lj + 3][li + 2 + l] -
                       sNode[lj + 2][li + 2 + l];
            } else {
              nodeGradient(i, j, nx, ny, [&](int a, int b) -> int { return sNode[b - y0 + 3][a - x0 + 3]; }, &ncx,
                           &ncy);
            }
            const int firstRows = abs(ncy) >= abs(ncx) ? 0 : 1;
            auto getC = [&](int a, int b) -> double { return sC[b - y0 + 3][a - x0 + 3]; };
            auto getN = [&](int a, int b) -> int { return sN[b - y0 + 3][a - x0 + 3]; };
            auto getB = [&](int a, int b) -> int { return sB[b - y0 + 3][a - x0 + 3]; };
            if (!hfTry(i, j, firstRows, I.h, getC, getN, getB, &kap) &&
                !hfTry(i, j, 1 - firstRows, I.h, getC, getN, getB, &kap)) {
              hffail++;
              fallback = true;
              kap = __builtin_nan("");  // k_ghf overwrites it where the parabola fit succeeds
            }
          }
          A.Kout[I.koff + id] = kap;
        }
        // one entry per 64 cells k .. k+63 (a wavefront) with any fallback cell
        const unsigned long long need = __ballot(fallback);
        if (need && (tid & 63) == 0) {
          const uint32_t slot = atomicAdd(A.ghfCount, 1u);
          A.ghf[slot] = GhfEntry{te.x, te.y * 4u + (uint32_t)(k >> 6), need};
        }
      }
    }
  }
  if (MODE & 2) {
    if (interf) atomicAdd(&sCnt[0], interf);
    if (hffail) atomicAdd(&sCnt[1], hffail);
    __syncthreads();
    if (tid == 0) {
      if (sCnt[0]) atomicAdd(&ctrPart(A.ctr)[C_INTERFACIAL], (unsigned long long)sCnt[0]);
      if (sCnt[1]) atomicAdd(&ctrPart(A.ctr)[C_HF_FAIL], (unsigned long long)sCnt[1]);
      if (ntiles_done) atomicAdd(&ctrPart(A.ctr)[C_TILES_NEAR], (unsigned long long)ntiles_done);
    }
  }
}

// The parabola fit of the cells a curvature launch left (heights failed in
// both directions): one single-wavefront workgroup per entry, one lane per
// cell. The entry's 4 rows x 16 cells need nodes x0-2..x0+18 and y0-2..y0+6
// around them (y0 the first row), H offsets x0-2..x0+17, y0-2..y0+6 and V
// offsets x0-2..x0+18, y0-2..y0+5: staged in LDS in one round of independent
// loads (indexes clamped into the grid; clamped slots are never read). kappa
// stays NaN where the fit has too few points or a singular system.
constexpr int GW_X = 21, GW_Y = 9;  // node window
template <bool ONE>
__global__ __launch_bounds__(64, 4) void k_ghf(FracArgs A, const Inst *__restrict__ inst) {
  __shared__ uint8_t sNw[GW_Y][GW_X];
  __shared__ double sHw[GW_Y][GW_X - 1];
  __shared__ double sVw[GW_Y - 1][GW_X];
  const int lane = threadIdx.x;
  const uint32_t n = *A.ghfCount;
  for (uint32_t it = blockIdx.x; it < n; it += gridDim.x) {
    const GhfEntry en = A.ghf[it];
    const uint32_t tile = uni(en.tile), gw = uni(en.gridWave);
    const unsigned long long mask = en.mask;
    const Inst &I = ONE ? A.one : inst[gw >> 2];
    const int nx = I.nx, ny = I.ny;
    const uint32_t lt = tile - I.tile0;
    const int wx0 = (int)(lt % (uint32_t)I.ntx) * TS - 2, wy0 = (int)(lt / (uint32_t)I.ntx) * TS + 4 * (int)(gw & 3u) - 2;
    const GL uint16_t *col = gp(I.col[A.cur]);
    const GL double *hoff = gp(I.hoff[A.cur]);
    const GL double *voff = gp(I.voff[A.cur]);
    const size_t W1 = (size_t)nx + 1;
    __syncthreads();  // the previous entry's reads are done
    constexpr int NW = (GW_Y * GW_X + 63) / 64;
    uint8_t rn[NW];
    double rh[NW], rv[NW];
#pragma unroll
    for (int r = 0; r < NW; r++) {
      const int k = lane + 64 * r;
      const int p = k % GW_X, q = k / GW_X;
      const int x = min(max(wx0 + p, 0), nx), y = min(max(wy0 + q, 0), ny);
      if (k < GW_Y * GW_X) {
        rn[r] = (uint8_t)colAt(col, nx, x, y);
        rh[r] = hoff[(size_t)y * nx + min(x, nx - 1)];
        rv[r] = voff[(size_t)min(y, ny - 1) * W1 + x];
      }
    }
#pragma unroll
    for (int r = 0; r < NW; r++) {
      const int k = lane + 64 * r;
      const int p = k % GW_X, q = k / GW_X;
      if (k < GW_Y * GW_X) {
        sNw[q][p] = rn[r];
        if (p < GW_X - 1) sHw[q][p] = rh[r];
        if (q < GW_Y - 1) sVw[q][p] = rv[r];
      }
    }
    __syncthreads();
    bool ok = false;
    if ((mask >> lane) & 1ull) {
      const int k = (int)(gw & 3u) * 64 + lane;
      const int i = wx0 + 2 + k % TS, j = wy0 + 2 + lane / TS;
      auto node = [&](int a, int b) -> int { return sNw[b - wy0][a - wx0]; };
      auto hoffAt = [&](int a, int b) -> double { return sHw[b - wy0][a - wx0]; };
      auto voffAt = [&](int a, int b) -> double { return sVw[b - wy0][a - wx0]; };
      // the gradient's 4x4 nodes, mirrored across walls, lie in the window
      int gx, gy;
      nodeGradient(i, j, nx, ny, node, &gx, &gy);
      double kap;
      ok = ghfFit(nx, ny, I.h, i, j, gx, gy, node, hoffAt, voffAt, &kap);
      if (ok) A.Kout[I.koff + (size_t)j * nx + i] = kap;
    }
    const unsigned long long got = __ballot(ok);
    if (got && lane == 0) atomicAdd(&ctrPart(A.ctr)[C_GHF_FIT], (unsigned long long)__popcll(got));
  }
}

// ---------------------------------------------------------------------------
// Consumers of the interface (Sec. 2.5, Eq. physical and the surface-tension
// term of Eq. NS): rho and mu from C per cell, and the face force
// sigma * kappa_f * (C_right - C_left) / h, kappa_f the curvature of the
// face's cells that carry one (two or more markers, finite), their mean when
// both do, else 0. Near tiles stage the tile plus one cell on the left and
// bottom (colours, C, kappa) in LDS; every other tile is uniform up to and
// including its border faces, so it gets constant rho, mu and zero forces.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double mixOf(double c, double a, double b) { return c * a + (1.0 - c) * b; }

// With one grid the uniform part is written as plain linear passes over each
// output array: workgroup b takes elements [b * NS_CHUNK, (b + 1) * NS_CHUNK)
// of one array, so that every wavefront store covers whole 128-byte lines
// (fx rows are nx + 1 long and start anywhere in a line; per-tile rows left a
// partial line at both ends of every wavefront's segment). Element (x, y) of a
// W-wide array belongs to tile (min(x, nx-1) / 16, min(y, ny-1) / 16), the
// tile whose near pass writes it; elements of near tiles are skipped. The
// stores are streaming (non-temporal): whole lines that nothing reads back
// soon, kept out of the caches.
constexpr int NS_CHUNK = 4096;
template <class Val>
__device__ __forceinline__ void nsLinearFill(double *arr, size_t size, size_t k0, int W, const NsArgs &A,
                                             const Inst &I, Val val) {
  constexpr int NE_T = 16;  // elements per thread and group, 256 apart
  size_t k = k0 + threadIdx.x;
  int y = (int)(k / (size_t)W), x = (int)(k - (size_t)y * (size_t)W);
  for (int g = 0; g < NS_CHUNK / (256 * NE_T); g++, k += 256 * NE_T) {
    // owner tiles first, then all tile-info loads at once, then the stores
    uint32_t tix[NE_T];
#pragma unroll
    for (int i = 0; i < NE_T; i++) {
      tix[i] = I.tile0 + (uint32_t)(min(y, I.ny - 1) / TS) * (uint32_t)I.ntx + (uint32_t)(min(x, I.nx - 1) / TS);
      x += 256;
      while (x >= W) {
        x -= W;
        y++;
      }
    }
    uint8_t ti[NE_T];
#pragma unroll
    for (int i = 0; i < NE_T; i++) ti[i] = k + 256u * i < size ? A.tinfo[tix[i]] : (uint8_t)TI_NEAR;
#pragma unroll
    for (int i = 0; i < NE_T; i++)
      if (!(ti[i] & (TI_NEAR | TI_DEAD))) __builtin_nontemporal_store(val(ti[i]), &arr[k + 256u * i]);
  }
}

template <bool ONE>
__global__ __launch_bounds__(256) void k_ns(NsArgs A, const Inst *__restrict__ inst,
                                            const uint32_t *__restrict__ tileInst) {
  constexpr int WC = TS + 1;  // cells per side with the left / bottom halo
  const int tid = threadIdx.x;
  if (ONE && (int)blockIdx.x >= A.nearBlocks) {
    // --- uniform part, one grid: linear passes over rho, mu, fx, fy ---------
    const Inst &I = A.one;
    const int nx = I.nx, ny = I.ny;
    const size_t sc = (size_t)nx * ny, sx = (size_t)(nx + 1) * ny, sy = (size_t)nx * (ny + 1);
    const uint32_t cc = (uint32_t)((sc + NS_CHUNK - 1) / NS_CHUNK), cx = (uint32_t)((sx + NS_CHUNK - 1) / NS_CHUNK);
    uint32_t b = blockIdx.x - (uint32_t)A.nearBlocks;
    auto colourOf = [](uint8_t ti) -> double { return (ti & TI_COLOUR) ? 1.0 : 0.0; };
    if (b < cc) {
      if (A.rho)
        nsLinearFill(A.rho + I.coff, sc, (size_t)b * NS_CHUNK, nx, A, I,
                     [&](uint8_t ti) { return mixOf(colourOf(ti), A.rho1, A.rho2); });
      return;
    }
    b -= cc;
    if (b < cc) {
      if (A.mu)
        nsLinearFill(A.mu + I.coff, sc, (size_t)b * NS_CHUNK, nx, A, I,
                     [&](uint8_t ti) { return mixOf(colourOf(ti), A.mu1, A.mu2); });
      return;
    }
    b -= cc;
    if (b < cx) {
      if (A.fx) nsLinearFill(A.fx + I.uoff, sx, (size_t)b * NS_CHUNK, nx + 1, A, I, [](uint8_t) { return 0.0; });
      return;
    }
    b -= cx;
    if (A.fy) nsLinearFill(A.fy + I.voffv, sy, (size_t)b * NS_CHUNK, nx, A, I, [](uint8_t) { return 0.0; });
    return;
  }
  if (!ONE && (int)blockIdx.x >= A.nearBlocks) {
    // --- uniform tiles: 16 consecutive global tiles, lanes along grid rows ---
    const uint32_t t = (blockIdx.x - (uint32_t)A.nearBlocks) * NS_FILL_TILES + (uint32_t)tid / TS;
    if (t >= A.ntiles) return;
    const uint8_t ti = A.tinfo[t];
    if (ti & (TI_NEAR | TI_DEAD)) return;
    const Inst &I = inst[tileInst[t]];
    const uint32_t lt = t - I.tile0;
    const int tx = (int)(lt % (uint32_t)I.ntx), ty = (int)(lt / (uint32_t)I.ntx);
    const int x = tx * TS + tid % TS;
    if (x >= I.nx) return;
    const int nx = I.nx, ny = I.ny, y0 = ty * TS, rows = min(TS, ny - y0);
    const double c = (ti & TI_COLOUR) ? 1.0 : 0.0;
    const double r = mixOf(c, A.rho1, A.rho2), m = mixOf(c, A.mu1, A.mu2);
    for (int q = 0; q < rows; q++) {
      const int y = y0 + q;
      if (A.rho) A.rho[I.coff + (size_t)y * nx + x] = r;
      if (A.mu) A.mu[I.coff + (size_t)y * nx + x] = m;
      if (A.fx) {
        A.fx[I.uoff + (size_t)y * (nx + 1) + x] = 0.0;
        if (x == nx - 1) A.fx[I.uoff + (size_t)y * (nx + 1) + nx] = 0.0;
      }
      if (A.fy) A.fy[I.voffv + (size_t)y * nx + x] = 0.0;
    }
    if (A.fy && y0 + rows == ny) A.fy[I.voffv + (size_t)ny * nx + x] = 0.0;
    return;
  }
  __shared__ uint8_t sNode[WC + 1][WC + 1];
  __shared__ double sC[WC][WC], sK[WC][WC];
  __shared__ uint8_t sDef[WC][WC];
  __shared__ uint2 sEnt[NEAR_ENT];
  const uint32_t ntile = *A.count;
  // this workgroup's first tile entries, read once
  if (tid < NEAR_ENT) {
    const uint32_t it = blockIdx.x + (uint32_t)tid * (uint32_t)A.nearBlocks;
    if (it < ntile) sEnt[tid] = A.list[it];
  }
  uint32_t n = 0;
  for (uint32_t it = blockIdx.x; it < ntile; it += (uint32_t)A.nearBlocks, n++) {
    __syncthreads();
    const uint2 e = n < (uint32_t)NEAR_ENT ? sEnt[n] : A.list[it];
    const uint2 te = make_uint2(uni(e.x), uni(e.y));
    const Inst &I = ONE ? A.one : inst[te.y];
    const int nx = I.nx, ny = I.ny;
    const uint32_t lt = te.x - I.tile0;
    const int x0 = (int)(lt % (uint32_t)I.ntx) * TS, y0 = (int)(lt / (uint32_t)I.ntx) * TS;
    const GL uint16_t *col = gp(I.col[A.cur]);
    const GL double *Cg = gp(A.C + I.coff);
    const GL double *Kg = gp(A.K + I.koff);
    // nodes x0-1 .. x0+16, cells x0-1 .. x0+15 (and the same in y)
    for (int k = tid; k < (WC + 1) * (WC + 1); k += blockDim.x) {
      const int li = k % (WC + 1), lj = k / (WC + 1);
      const int gx = x0 - 1 + li, gy = y0 - 1 + lj;
      sNode[lj][li] = (gx >= 0 && gy >= 0 && gx <= nx && gy <= ny) ? (uint8_t)colAt(col, nx, gx, gy) : (uint8_t)0;
    }
    for (int k = tid; k < WC * WC; k += blockDim.x) {
      const int li = k % WC, lj = k / WC;
      const int gx = x0 - 1 + li, gy = y0 - 1 + lj;
      const bool in = gx >= 0 && gy >= 0 && gx < nx && gy < ny;
      sC[lj][li] = in ? Cg[(size_t)gy * nx + gx] : 0.0;
      sK[lj][li] = in ? Kg[(size_t)gy * nx + gx] : 0.0;
    }
    __syncthreads();
    for (int k = tid; k < WC * WC; k += blockDim.x) {
      const int li = k % WC, lj = k / WC;
      const int bl = sNode[lj][li], br = sNode[lj][li + 1], tr = sNode[lj + 1][li + 1], tl = sNode[lj + 1][li];
      const int nm = (bl != br) + (br != tr) + (tl != tr) + (bl != tl);
      sDef[lj][li] = (uint8_t)(nm >= 2 && isfinite(sK[lj][li]));
    }
    __syncthreads();
    auto faceK = [&](int la, int ja, int lb, int jb) -> double {
      const bool da = sDef[ja][la], db = sDef[jb][lb];
      if (da && db) return (sK[ja][la] + sK[jb][lb]) * 0.5;
      if (da) return sK[ja][la];
      if (db) return sK[jb][lb];
      return 0.0;
    };
    for (int k = tid; k < TS * TS; k += blockDim.x) {
      const int li = k % TS, lj = k / TS;
      const int x = x0 + li, y = y0 + lj;
      if (x >= nx || y >= ny) continue;
      const int ci = li + 1, cj = lj + 1;  // LDS slot of cell (x, y)
      const double c = sC[cj][ci];
      if (A.rho) A.rho[I.coff + (size_t)y * nx + x] = mixOf(c, A.rho1, A.rho2);
      if (A.mu) A.mu[I.coff + (size_t)y * nx + x] = mixOf(c, A.mu1, A.mu2);
      if (A.fx) {
        // x-face x (left side of the cell); the wall face x = nx by the last column
        double f = 0.0;
        if (x > 0) {
          const double cl = sC[cj][ci - 1];
          if (cl != c) f = A.sigma * faceK(ci - 1, cj, ci, cj) * (c - cl) / I.h;
        }
        A.fx[I.uoff + (size_t)y * (nx + 1) + x] = f;
        if (x == nx - 1) A.fx[I.uoff + (size_t)y * (nx + 1) + nx] = 0.0;
      }
      if (A.fy) {
        double f = 0.0;
        if (y > 0) {
          const double cb = sC[cj - 1][ci];
          if (cb != c) f = A.sigma * faceK(ci, cj - 1, ci, cj) * (c - cb) / I.h;
        }
        A.fy[I.voffv + (size_t)y * nx + x] = f;
        if (y == ny - 1) A.fy[I.voffv + (size_t)ny * nx + x] = 0.0;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// State import and export in the caller's device buffers (the layout of the
// public header: node colours one byte per node, centre colours one byte per
// cell, offsets row-major), for the entry point that keeps no state of its own
// between calls. Import writes both state copies; a colour byte above 1, or an
// offset outside [0, 1] (or NaN) on an edge whose end colours differ, latches
// ERRBIT_ARG.
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) p[k] = v;
}

__global__ void k_put_inst(Inst I, Inst *dst) {
  if (threadIdx.x == 0) *dst = I;
}

// one thread per colour word (16 nodes of one row) of the bit plane
__global__ void k_import_colours(Inst I, const uint8_t *__restrict__ node) {
  const int nx = I.nx, ny = I.ny, nbx = cb_nbx(nx);
  const size_t words = (size_t)nbx * (size_t)(ny + 1);
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < words; k += (size_t)gridDim.x * blockDim.x) {
    const int y = (int)(k / (size_t)nbx), x0 = (int)(k % (size_t)nbx) * TS;
    uint32_t w = 0, bad = 0;
    for (int i = 0; i < TS && x0 + i <= nx; i++) {
      const uint32_t c = node[(size_t)y * (nx + 1) + x0 + i];
      bad |= c > 1u;
      w |= (c & 1u) << i;
    }
    const size_t at = cb_word(nx, x0, y);
    gp(I.col[0])[at] = (uint16_t)w;
    gp(I.col[1])[at] = (uint16_t)w;
    if (bad) atomicOr(I.err, ERRBIT_ARG);
  }
  // block rows past the last node row are part of the plane: zero them
  const size_t tail = cb_words(nx, ny) - (size_t)(ny + 1) * (size_t)nbx;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < tail; k += (size_t)gridDim.x * blockDim.x) {
    const size_t r = (size_t)(ny + 1) + k / (size_t)nbx, bx = k % (size_t)nbx;
    const size_t at = ((r >> 4) * (size_t)nbx + bx) * 16u + (r & 15u);
    gp(I.col[0])[at] = 0;
    gp(I.col[1])[at] = 0;
  }
}

__device__ __forceinline__ int nodeByte(const uint8_t *__restrict__ node, int nx, int x, int y) {
  return node[(size_t)y * (nx + 1) + x] & 1;
}

// offsets and centre colours into both copies (one thread per element)
__global__ void k_import_rest(Inst I, const uint8_t *__restrict__ node, const uint8_t *__restrict__ cell,
                              const double *__restrict__ hoff, const double *__restrict__ voff) {
  const int nx = I.nx, ny = I.ny;
  const size_t nh = (size_t)nx * (ny + 1), nv = (size_t)(nx + 1) * ny, nc = (size_t)nx * ny;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  uint32_t bad = 0;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < nh; k += stride) {
    const double o = hoff[k];
    const int y = (int)(k / (size_t)nx), x = (int)(k % (size_t)nx);
    if (nodeByte(node, nx, x, y) != nodeByte(node, nx, x + 1, y) && !(o >= 0.0 && o <= 1.0)) bad = 1;
    gp(I.hoff[0])[k] = o;
    gp(I.hoff[1])[k] = o;
  }
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < nv; k += stride) {
    const double o = voff[k];
    const int y = (int)(k / (size_t)(nx + 1)), x = (int)(k % (size_t)(nx + 1));
    if (nodeByte(node, nx, x, y) != nodeByte(node, nx, x, y + 1) && !(o >= 0.0 && o <= 1.0)) bad = 1;
    gp(I.voff[0])[k] = o;
    gp(I.voff[1])[k] = o;
  }
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < nc; k += stride) {
    const uint8_t c = cell[k];
    bad |= c > 1u;
    gp(I.cen[0])[k] = c;
  }
  if (bad) atomicOr(I.err, ERRBIT_ARG);
}

// copy `cur` of the state back to the caller's buffers
__global__ void k_export_state(Inst I, uint32_t cur, uint8_t *__restrict__ node, uint8_t *__restrict__ cell,
                               double *__restrict__ hoff, double *__restrict__ voff) {
  const int nx = I.nx, ny = I.ny;
  const size_t nn = (size_t)(nx + 1) * (ny + 1), nh = (size_t)nx * (ny + 1), nv = (size_t)(nx + 1) * ny,
               nc = (size_t)nx * ny;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const GL uint16_t *col = gp(I.col[cur]);
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < nn; k += stride) {
    const int y = (int)(k / (size_t)(nx + 1)), x = (int)(k % (size_t)(nx + 1));
    node[k] = (uint8_t)colAt(col, nx, x, y);
  }
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < nh; k += stride) hoff[k] = gp(I.hoff[cur])[k];
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < nv; k += stride) voff[k] = gp(I.voff[cur])[k];
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < nc; k += stride) cell[k] = gp(I.cen[cur])[k];
}

// latched error bits as status codes of the public header, one per grid
__global__ void k_status(const uint32_t *err, int32_t *status, uint32_t n) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const uint32_t b = err[k];
    status[k] = (b & ERRBIT_ARG) ? 1 : ((b & ERRBIT_CFL) ? 3 : ((b & ERRBIT_DOMAIN) ? 4 : 0));
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Workgroups of a kernel that are resident on one CU at once (persistent
// grids are sized to exactly fill the GPU, so the static tile shares of all
// workgroups run concurrently).
int resident_blocks(int which) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (which) {
    case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_sweep<0, true>, SWEEP_BS, 0); break;
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_fit<0, false>, 256, 0); break;  // fits only
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_centre<0, false>, 256, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_frac_curv<1, false>, FRAC_BS, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_frac_curv<2, false>, FRAC_BS, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_frac_curv<3, false>, FRAC_BS, 0); break;
  }
  if (e != hipSuccess) (void)hipGetLastError();  // a failed query must not surface at the next launch
  return (e == hipSuccess && n > 0) ? n : 1;
}

#define EBIT_LAUNCH(K, grid, s, ...) \
  do {                               \
    hipLaunchKernelGGL(K, dim3(grid), dim3(256), 0, s, __VA_ARGS__); \
  } while (0)

hipError_t launch_sweep(int dir, bool one, const SweepArgs &a, int grid, hipStream_t s) {
  if (dir == 0) {
    if (one) hipLaunchKernelGGL((k_sweep<0, true>), dim3(grid), dim3(SWEEP_BS), 0, s, a, a.inst);
    else hipLaunchKernelGGL((k_sweep<0, false>), dim3(grid), dim3(SWEEP_BS), 0, s, a, a.inst);
  } else {
    if (one) hipLaunchKernelGGL((k_sweep<1, true>), dim3(grid), dim3(SWEEP_BS), 0, s, a, a.inst);
    else hipLaunchKernelGGL((k_sweep<1, false>), dim3(grid), dim3(SWEEP_BS), 0, s, a, a.inst);
  }
  return hipGetLastError();
}

uint32_t compact_blocks(uint32_t ntiles) {
  const uint32_t per = 256 * CPT;
  return ntiles ? (ntiles + per - 1) / per : 1;
}

hipError_t launch_fit(int dir, bool one, const SweepArgs &a, int grid, const CompactArgs *c, hipStream_t s) {
  CompactArgs none{};
  const uint32_t cb = c ? compact_blocks(c->ntiles) : 0u;
  const CompactArgs &ca = c ? *c : none;
  const int g = grid + (int)cb;
  if (dir == 0) {
    if (one) EBIT_LAUNCH((k_fit<0, true>), g, s, a, a.inst, ca, cb);
    else EBIT_LAUNCH((k_fit<0, false>), g, s, a, a.inst, ca, cb);
  } else {
    if (one) EBIT_LAUNCH((k_fit<1, true>), g, s, a, a.inst, ca, cb);
    else EBIT_LAUNCH((k_fit<1, false>), g, s, a, a.inst, ca, cb);
  }
  return hipGetLastError();
}

hipError_t launch_centre(int dir, bool one, const SweepArgs &a, int grid, hipStream_t s) {
  if (dir == 0) {
    if (one) EBIT_LAUNCH((k_centre<0, true>), grid, s, a, a.inst);
    else EBIT_LAUNCH((k_centre<0, false>), grid, s, a, a.inst);
  } else {
    if (one) EBIT_LAUNCH((k_centre<1, true>), grid, s, a, a.inst);
    else EBIT_LAUNCH((k_centre<1, false>), grid, s, a, a.inst);
  }
  return hipGetLastError();
}

hipError_t launch_init_tiles(const Inst *inst, uint32_t kinst, uint32_t ntiles, uint32_t cur, uint32_t *tileInst,
                             uint16_t *has, uint8_t *nearPrev, hipStream_t s) {
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_tiles, dim3(ntiles), dim3(256), 0, s, inst, kinst, cur, tileInst, has, nearPrev);
  return hipGetLastError();
}

hipError_t launch_clear_tiles(uint32_t *tileInst, uint16_t *has, uint8_t *nearPrev, uint8_t *tinfo, uint32_t tile0,
                              uint32_t ntiles, hipStream_t s) {
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_clear_tiles, dim3((ntiles + 255) / 256), dim3(256), 0, s, tileInst, has, nearPrev, tinfo,
                     tile0, ntiles);
  return hipGetLastError();
}

hipError_t launch_compact(bool one, const CompactArgs &a, hipStream_t s) {
  const uint32_t blocks = compact_blocks(a.ntiles);
  if (one) EBIT_LAUNCH(k_compact<true>, blocks, s, a);
  else EBIT_LAUNCH(k_compact<false>, blocks, s, a);
  return hipGetLastError();
}

int ns_fill_blocks(uint32_t ntiles) { return (int)((ntiles + NS_FILL_TILES - 1) / NS_FILL_TILES); }
int ns_linear_blocks(int nx, int ny) {
  auto chunks = [](size_t n) { return (int)((n + NS_CHUNK - 1) / NS_CHUNK); };
  return 2 * chunks((size_t)nx * ny) + chunks((size_t)(nx + 1) * ny) + chunks((size_t)nx * (ny + 1));
}

hipError_t launch_ns(bool one, const NsArgs &a, int grid, hipStream_t s) {
  if (one) hipLaunchKernelGGL(k_ns<true>, dim3(grid), dim3(256), 0, s, a, a.inst, a.tileInst);
  else hipLaunchKernelGGL(k_ns<false>, dim3(grid), dim3(256), 0, s, a, a.inst, a.tileInst);
  return hipGetLastError();
}

hipError_t launch_ghf(bool one, const FracArgs &a, int grid, hipStream_t s) {
  if (one) hipLaunchKernelGGL(k_ghf<true>, dim3(grid), dim3(64), 0, s, a, a.inst);
  else hipLaunchKernelGGL(k_ghf<false>, dim3(grid), dim3(64), 0, s, a, a.inst);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t b = (n + 255) / 256;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)(b < 4096 ? b : 4096)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_put_inst(const Inst &I, Inst *dst, hipStream_t s) {
  hipLaunchKernelGGL(k_put_inst, dim3(1), dim3(64), 0, s, I, dst);
  return hipGetLastError();
}

hipError_t launch_import_state(const Inst &I, const uint8_t *node, const uint8_t *cell, const double *hoff,
                               const double *voff, hipStream_t s) {
  hipLaunchKernelGGL(k_import_colours, dim3(256), dim3(256), 0, s, I, node);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_import_rest, dim3(1024), dim3(256), 0, s, I, node, cell, hoff, voff);
  return hipGetLastError();
}

hipError_t launch_export_state(const Inst &I, uint32_t cur, uint8_t *node, uint8_t *cell, double *hoff, double *voff,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_export_state, dim3(1024), dim3(256), 0, s, I, cur, node, cell, hoff, voff);
  return hipGetLastError();
}

hipError_t launch_status(const uint32_t *err, int32_t *status, hipStream_t s) {
  return launch_status_many(err, status, 1u, s);
}

hipError_t launch_status_many(const uint32_t *err, int32_t *status, uint32_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_status, dim3((n + 255) / 256), dim3(256), 0, s, err, status, n);
  return hipGetLastError();
}

hipError_t launch_frac_curv(int mode, bool one, const FracArgs &a, int grid, hipStream_t s) {
  const dim3 g(grid), b(FRAC_BS);
  if (one) {
    if (mode == 1) hipLaunchKernelGGL((k_frac_curv<1, true>), g, b, 0, s, a, a.inst, a.tileInst);
    else if (mode == 2) hipLaunchKernelGGL((k_frac_curv<2, true>), g, b, 0, s, a, a.inst, a.tileInst);
    else hipLaunchKernelGGL((k_frac_curv<3, true>), g, b, 0, s, a, a.inst, a.tileInst);
  } else {
    if (mode == 1) hipLaunchKernelGGL((k_frac_curv<1, false>), g, b, 0, s, a, a.inst, a.tileInst);
    else if (mode == 2) hipLaunchKernelGGL((k_frac_curv<2, false>), g, b, 0, s, a, a.inst, a.tileInst);
    else hipLaunchKernelGGL((k_frac_curv<3, false>), g, b, 0, s, a, a.inst, a.tileInst);
  }
  return hipGetLastError();
}

}  // namespace ebit
