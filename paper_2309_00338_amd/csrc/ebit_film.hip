// Two markers per edge: the thin-film extension named at the end of Sec. 2.4
// and in Sec. 4, in the reading stated in include/ebit_film.h.
//
// Each sweep is five passes over global memory, one lane per edge, node or
// cell, in the physical (row-major) order of what the lane writes, so every
// pass stores coalesced. A launch is two-dimensional: x runs along an array
// row and each lane takes a run of consecutive rows of its column, so no lane
// divides a 64-bit index and the run's reads issue together. Most of the grid
// is away from the interface, and there a lane only copies counts and
// colours: the per-edge scratch (advected offsets) and the new offset pairs
// are written only for edges that hold markers. The two passes with heavy
// per-element work (the crossing search with its circle fits, and the
// fraction's polygons) are split: a quiet pass settles the elements with no
// marker near and lists the others in its workgroup's own slots with a count,
// and a heavy pass gives each wavefront the items of a few quiet workgroups,
// one per lane, so the heavy work runs in full wavefronts (no atomics on
// global memory anywhere).
//   advect  aligned markers to s' = s + u dt/h (Eq. Eq_marker_dis), unaligned
//           ones to their gray points (displacement only; walls hold);
//   flip    a node changes colour once per marker that passes it (Sec. 2.3);
//   land    each aligned edge gathers the markers landing on it from itself
//           and its two neighbours and keeps them by the landing rule;
//   cross   each new unaligned edge gathers the advected segments of its two
//           cells that cross its line, keeps them by the same rule and places
//           each kept one by the circle fit (Sec. 2.2), with the centre-colour
//           candidates of rules (1)-(5) (Sec. 2.3);
//   centre  each cell takes its left line's first result, else its right
//           line's, else keeps its centre colour.
// A sweep is written in its own frame: a runs along the sweep, b across; the
// y sweep is the x sweep of the transposed grid (H and V swap roles), which is
// also the order the CPU reading follows, so both visit a cell's markers in
// the same order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <new>

#include "ebit_film.h"

namespace ebit_film_impl {

constexpr uint32_t ERR_CFL = 1u, ERR_DOMAIN = 2u;
enum { F_MARKERS = 0, F_ANNIH, F_ANNIH_UN, F_THREE, F_PARITY, F_NCTR };
// counter partitions, a 256-byte line each (summed on the host)
constexpr int F_PARTS = 64, F_STRIDE = 32;
static_assert(F_NCTR <= F_STRIDE, "counters fit one partition");
constexpr int BS = 256;

__device__ __forceinline__ double lerp(double a, double b, double t) { return a + t * (b - a); }

// One copy of the state on the device (physical layout of ebit_film.h).
struct Buf {
  uint8_t *col, *cen, *hn, *vn;
  double2 *ho, *vo;
};

// Compaction of the elements of a row launch that need the heavy path,
// without atomics on global memory: the quiet pass puts the (row, column) of
// each such element in its workgroup's own slot range (as many slots as the
// workgroup has elements) and their number in cnt; the heavy pass gives each
// wavefront GW consecutive quiet workgroups and lets its lanes take their
// items one each, so the heavy path runs with full wavefronts.
struct Compact {
  uint2 *slot;
  uint32_t *cnt;
};
constexpr int GW = 8;  // quiet workgroups per heavy wavefront

// The items of quiet workgroups b0 .. b0+GW-1 (those below nq), one per lane:
// work(row, col) for each. `cap` is the slot range of one quiet workgroup.
template <class Fn>
__device__ __forceinline__ void walkItems(const Compact &W, uint32_t nq, uint32_t cap, Fn work) {
  const int lane = (int)threadIdx.x;
  const uint32_t b0 = blockIdx.x * GW;
  const uint32_t mine = lane < GW && b0 + (uint32_t)lane < nq ? W.cnt[b0 + lane] : 0u;
  uint32_t inc = mine;
#pragma unroll
  for (int d = 1; d < GW; d <<= 1) {
    const uint32_t v = (uint32_t)__shfl_up((int)inc, d);
    if (lane >= d) inc += v;
  }
  // exclusive offsets of the GW workgroups, wave-uniform
  uint32_t e[GW];
#pragma unroll
  for (int q = 0; q < GW; q++) e[q] = (uint32_t)__builtin_amdgcn_readlane((int)(inc - mine), q);
  const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)inc, GW - 1);
  for (uint32_t i = (uint32_t)lane; i < total; i += 64u) {
    // the last workgroup whose first item is at or before i (workgroups with
    // no items share their successor's offset and are passed over)
    int k = 0;
    uint32_t base = 0;
#pragma unroll
    for (int q = 0; q < GW; q++)
      if (e[q] <= i) {
        k = q;
        base = e[q];
      }
    const uint2 it = W.slot[(size_t)(b0 + (uint32_t)k) * cap + (i - base)];
    work((int)it.x, (int)it.y);
  }
}

struct SweepArgs {
  int nx, ny;
  double lam, delta;
  Buf cur, nxt;
  const double *vel;  // u for the x sweep, v for the y sweep
  double2 *sp;        // per aligned edge of the frame: advected offsets s' of its markers
  double2 *dv;        // per unaligned edge of the frame: displacements of its markers
  uint8_t *kept;      // 2 per aligned edge: 1 if that marker was kept where it landed
  int8_t *res;        // 4 per unaligned edge: (right, left) results of kept crossings 0 and 1
  uint32_t *err;
  unsigned long long *ctr;
  Compact wk;         // the edges of the crossing pass that need the search
};

// The sweep frame over a state copy. DIR 0: aligned edges are H, unaligned V;
// DIR 1: the transposed grid, aligned edges V, unaligned H.
template <int DIR>
struct Frame {
  int nx, ny, na, nb;
  const uint8_t *col, *cen, *an, *un;
  const double2 *ao, *uo;
  __device__ Frame(int nx_, int ny_, const Buf &B)
      : nx(nx_), ny(ny_), na(DIR == 0 ? nx_ : ny_), nb(DIR == 0 ? ny_ : nx_), col(B.col), cen(B.cen),
        an(DIR == 0 ? B.hn : B.vn), un(DIR == 0 ? B.vn : B.hn), ao(DIR == 0 ? B.ho : B.vo),
        uo(DIR == 0 ? B.vo : B.ho) {}
  __device__ size_t node(int a, int b) const { return DIR == 0 ? (size_t)b * (nx + 1) + a : (size_t)a * (nx + 1) + b; }
  __device__ size_t ale(int a, int b) const { return DIR == 0 ? (size_t)b * nx + a : (size_t)a * (nx + 1) + b; }
  __device__ size_t une(int a, int b) const { return DIR == 0 ? (size_t)b * (nx + 1) + a : (size_t)a * nx + b; }
  __device__ size_t cell(int a, int b) const { return DIR == 0 ? (size_t)b * nx + a : (size_t)a * nx + b; }
};

__device__ __forceinline__ double pick(const double2 &v, int k) { return k == 0 ? v.x : v.y; }

// Every array of the state is row-major; in the sweep frame its element
// (row, col) is (a, b) = (col, row) for the x sweep and (row, col) for the y
// sweep (the frame is the transposed grid).
template <int DIR>
__device__ __forceinline__ void frameOf(int row, int col, int &a, int &b) {
  a = DIR == 0 ? col : row;
  b = DIR == 0 ? row : col;
}

// A lane's run of K rows r0 .. r0+K-1 of its column (rows past `rows` are
// skipped): first need(row) for every row, which reads only a few counts and
// whose loads issue together (indices clamped to the last row, so every read
// is inside the array), then quiet(row) for the rows that need nothing (the
// plain copy away from the interface) and work(row) for the others.
template <int K, class Need, class Quiet, class Work>
__device__ __forceinline__ void rowRun(int r0, int rows, Need need, Quiet quiet, Work work) {
  uint32_t busy = 0, in = 0;
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int row = r0 + k < rows ? r0 + k : rows - 1;
    const uint32_t ok = r0 + k < rows ? 1u : 0u;
    in |= ok << k;
    busy |= (ok & (need(row) ? 1u : 0u)) << k;
  }
#pragma unroll
  for (int k = 0; k < K; k++)
    if (((in & ~busy) >> k) & 1u) quiet(r0 + k);
  while (busy) {
    const int k = __ffs(busy) - 1;
    busy &= busy - 1u;
    work(r0 + k);
  }
}
constexpr int KR = 8;  // rows per lane in the plain passes
constexpr int KX = 4;  // rows per lane in the crossing pass (seven counts per row)

// Workgroup sums of the counters, one atomic per counter and workgroup, into
// partition (linear workgroup index) % F_PARTS: atomics on one line are
// served one after another, and the thousands of workgroups of a pass end at
// about the same time.
__device__ void addCounters(unsigned long long *ctr, const uint32_t *v) {
  __shared__ uint32_t s[F_NCTR];
  if (threadIdx.x < F_NCTR) s[threadIdx.x] = 0;
  __syncthreads();
  for (int k = 0; k < F_NCTR; k++)
    if (v[k]) atomicAdd(&s[k], v[k]);
  __syncthreads();
  const uint32_t part = (blockIdx.x + blockIdx.y * gridDim.x) % (uint32_t)F_PARTS;
  if (threadIdx.x < F_NCTR && s[threadIdx.x])
    atomicAdd(&ctr[part * F_STRIDE + threadIdx.x], (unsigned long long)s[threadIdx.x]);
}

// ---------------------------------------------------------------------------
// advect
// ---------------------------------------------------------------------------
template <int DIR>
__global__ __launch_bounds__(BS) void k_film_advect(SweepArgs A) {
  const Frame<DIR> F(A.nx, A.ny, A.cur);
  uint32_t err = 0, c[F_NCTR] = {0, 0, 0, 0, 0};
  auto V = [&](int a, int r) -> double {
    r = r < 0 ? 0 : (r > F.nb - 1 ? F.nb - 1 : r);
    return A.vel[F.une(a, r)];
  };
  // rows of the aligned array, then rows of the unaligned one
  const int rA = DIR == 0 ? A.ny + 1 : A.ny, wA = DIR == 0 ? A.nx : A.nx + 1;
  const int rU = DIR == 0 ? A.ny : A.ny + 1, wU = DIR == 0 ? A.nx + 1 : A.nx;
  const int col = (int)(blockIdx.x * BS + threadIdx.x);
  auto need = [&](int row) -> bool {
    if (row < rA) return col < wA && F.an[(size_t)row * (size_t)wA + (size_t)col] != 0;
    return col < wU && F.un[(size_t)(row - rA) * (size_t)wU + (size_t)col] != 0;
  };
  auto work = [&](int row) {
    if (row < rA) {
      const size_t t = (size_t)row * (size_t)wA + (size_t)col;
      const int n = F.an[t];
      int a, b;
      frameOf<DIR>(row, col, a, b);
      const double2 o = F.ao[t];
      double r[2] = {0.0, 0.0};
      for (int k = 0; k < n; k++) {
        const double sv = pick(o, k);
        const double ub = lerp(lerp(V(a, b - 1), V(a + 1, b - 1), sv), lerp(V(a, b), V(a + 1, b), sv), 0.5);
        const double d = ub * A.lam;
        if (fabs(d) > 0.5) err |= ERR_CFL;
        r[k] = sv + d;
        if ((r[k] >= 1.0 && a + 1 >= F.na) || (r[k] < 0.0 && a == 0)) err |= ERR_DOMAIN;
      }
      A.sp[t] = make_double2(r[0], r[1]);
      c[F_MARKERS] += (uint32_t)n;
    } else {
      const int ur = row - rA;
      const size_t e = (size_t)ur * (size_t)wU + (size_t)col;
      const int n = F.un[e];
      int a, b;
      frameOf<DIR>(ur, col, a, b);
      const double2 o = F.uo[e];
      double r[2] = {0.0, 0.0};
      for (int k = 0; k < n; k++) {
        const double sv = pick(o, k);
        const double ub = sv < 0.5 ? lerp(V(a, b - 1), V(a, b), sv + 0.5) : lerp(V(a, b), V(a, b + 1), sv - 0.5);
        const double d = ub * A.lam;
        if (fabs(d) > 0.5) err |= ERR_CFL;
        r[k] = (a == 0 || a == F.na) ? 0.0 : d;
      }
      A.dv[e] = make_double2(r[0], r[1]);
      c[F_MARKERS] += (uint32_t)n;
    }
  };
  // edges without markers leave no scratch (nothing reads it for them)
  for (int r0 = (int)blockIdx.y * KR; r0 < rA + rU; r0 += (int)gridDim.y * KR)
    rowRun<KR>(r0, rA + rU, need, [](int) {}, work);
  if (err) atomicOr(A.err, err);
  addCounters(A.ctr, c);
}

// ---------------------------------------------------------------------------
// flip
// ---------------------------------------------------------------------------
template <int DIR>
__global__ __launch_bounds__(BS) void k_film_flip(SweepArgs A) {
  const Frame<DIR> F(A.nx, A.ny, A.cur);
  const int col = (int)(blockIdx.x * BS + threadIdx.x);
  if (col > A.nx) return;
  auto at = [&](int row) { return (size_t)row * (size_t)(A.nx + 1) + (size_t)col; };
  // a node flips once per marker that passes it: only the aligned edges on its
  // two sides can carry one
  auto need = [&](int row) -> bool {
    int a, b;
    frameOf<DIR>(row, col, a, b);
    return (a >= 1 && F.an[F.ale(a - 1, b)] != 0) || (a < F.na && F.an[F.ale(a, b)] != 0);
  };
  auto quiet = [&](int row) { A.nxt.col[at(row)] = F.col[at(row)]; };
  auto work = [&](int row) {
    int a, b;
    frameOf<DIR>(row, col, a, b);
    int flips = 0;
    if (a >= 1) {
      const size_t e = F.ale(a - 1, b);
      const int n = F.an[e];
      if (n) {
        const double2 sv = A.sp[e];
        for (int k = 0; k < n; k++) flips += pick(sv, k) >= 1.0 ? 1 : 0;
      }
    }
    if (a < F.na) {
      const size_t e = F.ale(a, b);
      const int n = F.an[e];
      if (n) {
        const double2 sv = A.sp[e];
        for (int k = 0; k < n; k++) flips += pick(sv, k) < 0.0 ? 1 : 0;
      }
    }
    A.nxt.col[at(row)] = (uint8_t)(F.col[at(row)] ^ (uint8_t)(flips & 1));
  };
  for (int r0 = (int)blockIdx.y * KR; r0 <= A.ny; r0 += (int)gridDim.y * KR) rowRun<KR>(r0, A.ny + 1, need, quiet, work);
}

// ---------------------------------------------------------------------------
// land: the landing rule on each aligned edge
// ---------------------------------------------------------------------------
template <int DIR>
__global__ __launch_bounds__(BS) void k_film_land(SweepArgs A) {
  const Frame<DIR> F(A.nx, A.ny, A.cur);
  uint32_t c[F_NCTR] = {0, 0, 0, 0, 0};
  const int rA = DIR == 0 ? A.ny + 1 : A.ny, wA = DIR == 0 ? A.nx : A.nx + 1;
  const int col = (int)(blockIdx.x * BS + threadIdx.x);
  uint8_t *dn = DIR == 0 ? A.nxt.hn : A.nxt.vn;
  double2 *dof = DIR == 0 ? A.nxt.ho : A.nxt.vo;
  // landers can come only from the edge and its two neighbours on the row
  auto need = [&](int row) -> bool {
    int a, b;
    frameOf<DIR>(row, col, a, b);
    return (a >= 1 && F.an[F.ale(a - 1, b)] != 0) || F.an[F.ale(a, b)] != 0 ||
           (a + 1 < F.na && F.an[F.ale(a + 1, b)] != 0);
  };
  auto quiet = [&](int row) { dn[(size_t)row * (size_t)wA + (size_t)col] = 0; };
  auto work = [&](int row) {
    const size_t t = (size_t)row * (size_t)wA + (size_t)col;
    int a, b;
    frameOf<DIR>(row, col, a, b);
    // landers in source order (a-1, a, a+1; first marker first), then a stable
    // insertion sort by position
    double o[6];
    size_t src[6];
    int kk[6];
    int n = 0;
    for (int q = a - 1; q <= a + 1; q++) {
      if (q < 0 || q >= F.na) continue;
      const size_t e = F.ale(q, b);
      const int ne = F.an[e];
      if (ne == 0) continue;
      const double2 s2 = A.sp[e];
      for (int k = 0; k < ne; k++) {
        const double s = pick(s2, k);
        const int tgt = s >= 1.0 ? q + 1 : (s < 0.0 ? q - 1 : q);
        if (tgt != a) continue;
        double v = q < a ? s - 1.0 : (q > a ? s + 1.0 : s);
        size_t se = e;
        int sk = k;
        int m = n++;
        while (m > 0 && o[m - 1] > v) {
          o[m] = o[m - 1];
          src[m] = src[m - 1];
          kk[m] = kk[m - 1];
          m--;
        }
        o[m] = v;
        src[m] = se;
        kk[m] = sk;
      }
    }
    int lo = 0, nk = 0;  // kept: o[lo .. lo+nk)
    if (n & 1) {
      lo = n / 2;
      nk = 1;
    } else if (n > 0 && o[n / 2] - o[n / 2 - 1] >= A.delta) {
      lo = n / 2 - 1;
      nk = 2;
    }
    for (int m = 0; m < n; m++) A.kept[2 * src[m] + kk[m]] = (uint8_t)(m >= lo && m < lo + nk);
    dn[t] = (uint8_t)nk;
    if (nk > 0) dof[t] = make_double2(o[lo], nk > 1 ? o[lo + 1] : 0.0);
    c[F_ANNIH] += (uint32_t)(n - nk);
  };
  if (col < wA)
    for (int r0 = (int)blockIdx.y * KR; r0 < rA; r0 += (int)gridDim.y * KR) rowRun<KR>(r0, rA, need, quiet, work);
  addCounters(A.ctr, c);
}

// ---------------------------------------------------------------------------
// cross: new unaligned edges
// ---------------------------------------------------------------------------
// Markers of a cell in counter-clockwise order from corner BL (edge ids 0
// bottom left to right, 1 right bottom to top, 2 top right to left, 3 left top
// to bottom) and its segments: the marker after which each boundary arc whose
// colour differs from the centre colour starts, the arc round BL first.
struct Bnd {
  int n, nseg;
  uint8_t e[8], k[8];
  double o[8];
  uint8_t seg[8];  // segment s joins markers seg[s] and (seg[s] + 1) % n
};

template <int DIR>
__device__ void boundary(const Frame<DIR> &F, int p, int q, Bnd &B) {
  B.n = 0;
  {
    const size_t e = F.ale(p, q);
    const double2 o = F.ao[e];
    for (int k = 0; k < F.an[e]; k++) { B.e[B.n] = 0; B.k[B.n] = (uint8_t)k; B.o[B.n++] = pick(o, k); }
  }
  {
    const size_t e = F.une(p + 1, q);
    const double2 o = F.uo[e];
    for (int k = 0; k < F.un[e]; k++) { B.e[B.n] = 1; B.k[B.n] = (uint8_t)k; B.o[B.n++] = pick(o, k); }
  }
  {
    const size_t e = F.ale(p, q + 1);
    const double2 o = F.ao[e];
    for (int k = F.an[e] - 1; k >= 0; k--) { B.e[B.n] = 2; B.k[B.n] = (uint8_t)k; B.o[B.n++] = pick(o, k); }
  }
  {
    const size_t e = F.une(p, q);
    const double2 o = F.uo[e];
    for (int k = F.un[e] - 1; k >= 0; k--) { B.e[B.n] = 3; B.k[B.n] = (uint8_t)k; B.o[B.n++] = pick(o, k); }
  }
  B.nseg = 0;
  if (B.n == 0) return;
  const int col0 = F.col[F.node(p, q)], cc = F.cen[F.cell(p, q)];
  for (int s = 0; s < B.n; s++) {
    const int idx = s == 0 ? B.n - 1 : s - 1;
    if ((col0 ^ ((idx + 1) & 1)) != cc) B.seg[B.nseg++] = (uint8_t)idx;
  }
}

// A marker reference: kind 0 aligned edge (i, j) of the frame, 1 unaligned
// edge (i, j); k its index in the edge's list; kind -1 none.
struct Ref {
  int kind, i, j, k;
};
__device__ __forceinline__ Ref refOf(int p, int q, int e, int k) {
  switch (e) {
    case 0: return Ref{0, p, q, k};
    case 1: return Ref{1, p + 1, q, k};
    case 2: return Ref{0, p, q + 1, k};
    default: return Ref{1, p, q, k};
  }
}

// Circle through three points met with the line X = 0, as the one-marker
// method's fit (Sec. 2.2): the root on the far side of chord P2P3 from the
// outer point O, else the one nearer the chord's height ysl; false when there
// is none or it leaves the edge.
__device__ bool circleRoot(double Xa, double Ya, double Xb, double Yb, double Xc, double Yc, double Xo, double Yo,
                           double X2, double Y2, double X3, double Y3, double ysl, double *out) {
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
    const double qq = -0.5 * (cc + (cc >= 0.0 ? sq : -sq));
    double r1, r2;
    if (qq == 0.0) {
      r1 = 0.0;
      r2 = 0.0;
    } else {
      r1 = qq / ca;
      r2 = ce / qq;
    }
    const double DX = X3 - X2, DY = Y3 - Y2;
    const double so = DX * (Yo - Y2) - DY * (Xo - X2);
    const double s1 = DX * (r1 - Y2) - DY * (0.0 - X2);
    const double s2 = DX * (r2 - Y2) - DY * (0.0 - X2);
    const bool q1 = (s1 > 0.0 && so < 0.0) || (s1 < 0.0 && so > 0.0);
    const bool q2 = (s2 > 0.0 && so < 0.0) || (s2 < 0.0 && so > 0.0);
    if (q1 && !q2) r = r1;
    else if (q2 && !q1) r = r2;
    else r = fabs(r1 - ysl) <= fabs(r2 - ysl) ? r1 : r2;
  }
  if (!(0.0 <= r && r <= 1.0)) return false;
  *out = r;
  return true;
}

template <int DIR>
__global__ __launch_bounds__(BS) void k_film_cross_quiet(SweepArgs A) {
  const Frame<DIR> F(A.nx, A.ny, A.cur);
  const int rU = DIR == 0 ? A.ny : A.ny + 1, wU = DIR == 0 ? A.nx + 1 : A.nx;
  const int col = (int)(blockIdx.x * BS + threadIdx.x);
  uint8_t *dn = DIR == 0 ? A.nxt.vn : A.nxt.hn;
  // an interior edge whose two cells hold no marker: nothing crosses it, and
  // no node of theirs flips (their aligned edges hold none), so it stays empty
  auto need = [&](int row) -> bool {
    int a, b;
    frameOf<DIR>(row, col, a, b);
    if (a == 0 || a == F.na) return true;
    return (F.an[F.ale(a - 1, b)] | F.an[F.ale(a - 1, b + 1)] | F.an[F.ale(a, b)] | F.an[F.ale(a, b + 1)] |
            F.un[F.une(a - 1, b)] | F.un[F.une(a, b)] | F.un[F.une(a + 1, b)]) != 0;
  };
  // the edges that need nothing are written here; the others go to the
  // workgroup's slots for the search pass
  const uint32_t blk = blockIdx.y * gridDim.x + blockIdx.x;
  uint2 *slot = A.wk.slot + (size_t)blk * (BS * KX);
  __shared__ uint32_t sN;
  if (threadIdx.x == 0) sN = 0;
  __syncthreads();
  if (col < wU)
    for (int r0 = (int)blockIdx.y * KX; r0 < rU; r0 += (int)gridDim.y * KX)
      rowRun<KX>(r0, rU, need, [&](int row) { dn[(size_t)row * (size_t)wU + (size_t)col] = 0; },
                 [&](int row) { slot[atomicAdd(&sN, 1u)] = make_uint2((uint32_t)row, (uint32_t)col); });
  __syncthreads();
  if (threadIdx.x == 0) A.wk.cnt[blk] = sN;
}

template <int DIR>
__global__ __launch_bounds__(64) void k_film_cross(SweepArgs A, uint32_t nq) {
  const Frame<DIR> F(A.nx, A.ny, A.cur);
  uint32_t c[F_NCTR] = {0, 0, 0, 0, 0};
  const int wU = DIR == 0 ? A.nx + 1 : A.nx;
  uint8_t *dn = DIR == 0 ? A.nxt.vn : A.nxt.hn;
  double2 *dof = DIR == 0 ? A.nxt.vo : A.nxt.ho;
  // the edges the quiet pass listed: walls, and interior edges with markers
  // in one of their two cells
  auto work = [&](int row, int col) {
    const size_t t = (size_t)row * (size_t)wU + (size_t)col;
    int a, b;
    frameOf<DIR>(row, col, a, b);
    if (a == 0 || a == F.na) {
      // walls keep their markers
      const int n = F.un[t];
      dn[t] = (uint8_t)n;
      if (n) dof[t] = F.uo[t];
    } else {
      // advected position of a marker in the frame of node (a, b), integer part first
      auto pos = [&](const Ref &r, double &X, double &Y) {
        if (r.kind == 0) {
          X = (double)(r.i - a) + pick(A.sp[F.ale(r.i, r.j)], r.k);
          Y = (double)(r.j - b);
        } else {
          const size_t e = F.une(r.i, r.j);
          X = (double)(r.i - a) + pick(A.dv[e], r.k);
          Y = (double)(r.j - b) + pick(F.uo[e], r.k);
        }
      };
      // left of line a, decided on the offsets
      auto leftOf = [&](const Ref &r) -> bool {
        const double v = r.kind == 0 ? pick(A.sp[F.ale(r.i, r.j)], r.k) : pick(A.dv[F.une(r.i, r.j)], r.k);
        return v < (double)(a - r.i);
      };
      struct Cross {
        double y, X2, Y2, X3, Y3;
        int p;
        uint8_t e2, k2, e3, k3;
      };
      Cross cr[8];
      int n = 0;
      Bnd B;
      for (int p = a - 1; p <= a; p++) {
        boundary<DIR>(F, p, b, B);
        for (int s = 0; s < B.nseg; s++) {
          int ia = B.seg[s], ib = (B.seg[s] + 1) % B.n;
          Ref ra = refOf(p, b, B.e[ia], B.k[ia]), rb = refOf(p, b, B.e[ib], B.k[ib]);
          const bool la = leftOf(ra), lb = leftOf(rb);
          if (la == lb) continue;
          if (!la) {
            const Ref tr = ra;
            ra = rb;
            rb = tr;
            const int ti = ia;
            ia = ib;
            ib = ti;
          }
          double X2, Y2, X3, Y3;
          pos(ra, X2, Y2);
          pos(rb, X3, Y3);
          double y = Y2 + (Y3 - Y2) * (0.0 - X2) / (X3 - X2);
          y = 0.0 > y ? 0.0 : y;
          y = 1.0 < y ? 1.0 : y;
          // stable insertion by height (ties keep the order found)
          int m = n++;
          while (m > 0 && cr[m - 1].y > y) {
            cr[m] = cr[m - 1];
            m--;
          }
          cr[m] = Cross{y, X2, Y2, X3, Y3, p, B.e[ia], B.k[ia], B.e[ib], B.k[ib]};
        }
      }
      const int nc0 = A.nxt.col[F.node(a, b)], nc1 = A.nxt.col[F.node(a, b + 1)];
      if ((n & 1) != (nc0 != nc1 ? 1 : 0)) c[F_PARITY] += 1;
      int lo = 0, nk = 0;
      if (n & 1) {
        lo = n / 2;
        nk = 1;
      } else if (n > 0 && cr[n / 2].y - cr[n / 2 - 1].y >= A.delta) {
        lo = n / 2 - 1;
        nk = 2;
      }
      if (n == 3) c[F_THREE] += 1;
      c[F_ANNIH_UN] += (uint32_t)(n - nk);
      // chain neighbour: the partner, in the cell across edge e of cell (p, q),
      // of marker k of that edge
      auto partner = [&](int p, int q, int e, int k) -> Ref {
        const int pp = e == 1 ? p + 1 : (e == 3 ? p - 1 : p), qq = e == 0 ? q - 1 : (e == 2 ? q + 1 : q);
        if (pp < 0 || pp >= F.na || qq < 0 || qq >= F.nb) return Ref{-1, 0, 0, 0};
        Bnd N;
        boundary<DIR>(F, pp, qq, N);
        const int eo = (e + 2) & 3;
        for (int s = 0; s < N.nseg; s++) {
          const int x0 = N.seg[s], y0 = (N.seg[s] + 1) % N.n;
          if (N.e[x0] == eo && N.k[x0] == k) return refOf(pp, qq, N.e[y0], N.k[y0]);
          if (N.e[y0] == eo && N.k[y0] == k) return refOf(pp, qq, N.e[x0], N.k[x0]);
        }
        return Ref{-1, 0, 0, 0};
      };
      // centre-colour candidate (rules (1)-(5)): the first aligned marker of
      // (first, then second when first is unaligned) kept on an edge of the
      // cell's bottom or top that lies in cell `cell`
      auto rule = [&](const Ref &first, const Ref &second, int cell) -> int {
        for (int w = 0; w < 2; w++) {
          const Ref &m = w == 0 ? first : second;
          if (w == 1 && first.kind != 1) break;
          if (m.kind != 0) continue;
          if (m.j != b && m.j != b + 1) continue;
          const size_t e = F.ale(m.i, m.j);
          if (!A.kept[2 * e + m.k]) continue;
          const double s = pick(A.sp[e], m.k);
          const int tgt = s >= 1.0 ? m.i + 1 : (s < 0.0 ? m.i - 1 : m.i);
          if (tgt == cell) return 1 - (int)A.nxt.col[F.node(a, m.j)];
        }
        return -1;
      };
      double ys[2] = {0.0, 0.0};
      for (int q = 0; q < nk; q++) {
        const Cross &K = cr[lo + q];
        const Ref r2 = refOf(K.p, b, K.e2, K.k2), r3 = refOf(K.p, b, K.e3, K.k3);
        const Ref m1 = partner(K.p, b, K.e2, K.k2), m4 = partner(K.p, b, K.e3, K.k3);
        double y;
        if (K.X3 == 0.0) {
          y = K.Y3;
        } else {
          double got[2];
          int ng = 0;
          if (m1.kind >= 0) {
            double X1, Y1, r;
            pos(m1, X1, Y1);
            if (circleRoot(X1, Y1, K.X2, K.Y2, K.X3, K.Y3, X1, Y1, K.X2, K.Y2, K.X3, K.Y3, K.y, &r)) got[ng++] = r;
          }
          if (m4.kind >= 0) {
            double X4, Y4, r;
            pos(m4, X4, Y4);
            if (circleRoot(K.X2, K.Y2, K.X3, K.Y3, X4, Y4, X4, Y4, K.X2, K.Y2, K.X3, K.Y3, K.y, &r)) got[ng++] = r;
          }
          y = ng == 2 ? (got[0] + got[1]) * 0.5 : (ng == 1 ? got[0] : K.y);
        }
        ys[q] = y;
        A.res[4 * t + 2 * q] = (int8_t)rule(r3, m4, a);
        A.res[4 * t + 2 * q + 1] = (int8_t)rule(r2, m1, a - 1);
      }
      if (nk == 2 && ys[1] < ys[0]) {
        const double tmp = ys[0];
        ys[0] = ys[1];
        ys[1] = tmp;
      }
      dn[t] = (uint8_t)nk;
      if (nk > 0) dof[t] = make_double2(ys[0], ys[1]);
    }
  };
  walkItems(A.wk, nq, BS * KX, work);
  addCounters(A.ctr, c);
}

// ---------------------------------------------------------------------------
// centre
// ---------------------------------------------------------------------------
template <int DIR>
__global__ __launch_bounds__(BS) void k_film_centre(SweepArgs A) {
  const Frame<DIR> F(A.nx, A.ny, A.cur);
  const int col = (int)(blockIdx.x * BS + threadIdx.x);
  if (col >= A.nx) return;
  const uint8_t *nn = DIR == 0 ? A.nxt.vn : A.nxt.hn;  // new unaligned counts (kept crossings)
  auto at = [&](int row) { return (size_t)row * (size_t)A.nx + (size_t)col; };
  // a cell takes a new colour only from a kept crossing on its left or right line
  auto need = [&](int row) -> bool {
    int a, b;
    frameOf<DIR>(row, col, a, b);
    return (a >= 1 && nn[F.une(a, b)] != 0) || (a + 1 <= F.na - 1 && nn[F.une(a + 1, b)] != 0);
  };
  auto quiet = [&](int row) { A.nxt.cen[at(row)] = F.cen[at(row)]; };
  auto work = [&](int row) {
    const size_t t = at(row);
    int a, b;
    frameOf<DIR>(row, col, a, b);
    int r = -1;
    if (a >= 1) {
      const size_t e = F.une(a, b);
      for (int q = 0; q < nn[e] && r < 0; q++) r = A.res[4 * e + 2 * q] >= 0 ? A.res[4 * e + 2 * q] : -1;
    }
    if (r < 0 && a + 1 <= F.na - 1) {
      const size_t e = F.une(a + 1, b);
      for (int q = 0; q < nn[e] && r < 0; q++) r = A.res[4 * e + 2 * q + 1] >= 0 ? A.res[4 * e + 2 * q + 1] : -1;
    }
    A.nxt.cen[t] = r >= 0 ? (uint8_t)r : F.cen[t];
  };
  for (int r0 = (int)blockIdx.y * KR; r0 < A.ny; r0 += (int)gridDim.y * KR) rowRun<KR>(r0, A.ny, need, quiet, work);
}

// ---------------------------------------------------------------------------
// volume fraction
// ---------------------------------------------------------------------------
__device__ __forceinline__ double tauOf(int e, double o) {
  return e == 0 ? o : (e == 1 ? 1.0 + o : (e == 2 ? 3.0 - o : 4.0 - o));
}
__device__ __forceinline__ void pointOf(double tau, double &x, double &y) {
  while (tau >= 4.0) tau -= 4.0;  // tau in [0, 8]: each subtraction is exact
  if (tau <= 1.0) { x = tau; y = 0.0; }
  else if (tau <= 2.0) { x = 1.0; y = tau - 1.0; }
  else if (tau <= 3.0) { x = 3.0 - tau; y = 1.0; }
  else { x = 0.0; y = 4.0 - tau; }
}

// Volume fraction of cell (p, q) with markers on its boundary: the regions the
// segments cut off, or the cell minus them.
__device__ void cellFraction(const Frame<0> &F, int p, int q, double *out) {
  Bnd B;
  boundary<0>(F, p, q, B);
  if (B.n == 0) {
    *out = (double)F.col[F.node(p, q)];
    return;
  }
  double cut = 0.0;
  for (int s = 0; s < B.nseg; s++) {
    const int ia = B.seg[s], ib = (B.seg[s] + 1) % B.n;
    const double ta = tauOf(B.e[ia], B.o[ia]);
    double tb = tauOf(B.e[ib], B.o[ib]);
    if (tb < ta) tb += 4.0;
    double px[6], py[6];
    int np = 0;
    pointOf(ta, px[np], py[np]);
    np++;
    for (int k = 1; k <= 7; k++)
      if (ta < (double)k && (double)k < tb) {
        pointOf((double)k, px[np], py[np]);
        np++;
      }
    pointOf(tb, px[np], py[np]);
    np++;
    double ar = 0.0;
    for (int k = 0; k < np; k++) {
      const int k1 = k + 1 == np ? 0 : k + 1;
      ar += px[k] * py[k1] - px[k1] * py[k];
    }
    cut += fabs(0.5 * ar);
  }
  *out = F.cen[F.cell(p, q)] == 1 ? 1.0 - cut : cut;
}

// a cell with no marker on its boundary has one colour
__device__ __forceinline__ bool cellNeeds(const Frame<0> &F, int p, int q) {
  return (F.an[F.ale(p, q)] | F.an[F.ale(p, q + 1)] | F.un[F.une(p, q)] | F.un[F.une(p + 1, q)]) != 0;
}

// the one-colour cells; the others go to the workgroup's slots
__global__ __launch_bounds__(BS) void k_film_fraction_quiet(int nx, int ny, Buf S, double *C, Compact W) {
  const int p = (int)(blockIdx.x * BS + threadIdx.x);
  const Frame<0> F(nx, ny, S);
  const uint32_t blk = blockIdx.y * gridDim.x + blockIdx.x;
  uint2 *slot = W.slot + (size_t)blk * (BS * KR);
  __shared__ uint32_t sN;
  if (threadIdx.x == 0) sN = 0;
  __syncthreads();
  if (p < nx)
    for (int r0 = (int)blockIdx.y * KR; r0 < ny; r0 += (int)gridDim.y * KR)
      rowRun<KR>(r0, ny, [&](int q) { return cellNeeds(F, p, q); },
                 [&](int q) { C[(size_t)q * (size_t)nx + p] = (double)F.col[F.node(p, q)]; },
                 [&](int q) { slot[atomicAdd(&sN, 1u)] = make_uint2((uint32_t)q, (uint32_t)p); });
  __syncthreads();
  if (threadIdx.x == 0) W.cnt[blk] = sN;
}

// the cells with markers on their boundary that the quiet pass listed
__global__ __launch_bounds__(64) void k_film_fraction(int nx, int ny, Buf S, double *C, Compact W, uint32_t nq) {
  const Frame<0> F(nx, ny, S);
  walkItems(W, nq, BS * KR, [&](int q, int p) { cellFraction(F, p, q, C + (size_t)q * (size_t)nx + p); });
}
// ---------------------------------------------------------------------------
// host
// ---------------------------------------------------------------------------
struct Carve {
  char *base;
  size_t off = 0;
  template <class T>
  T *take(size_t n) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? (T *)(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

bool grid_ok(const ebit_grid *g) {
  return g && g->nx >= 4 && g->ny >= 4 && g->nx <= 65535 && g->ny <= 65535 && isfinite(g->h) && g->h > 0.0 &&
         g->flags == 0u;
}

int validate(const ebit_grid *g, const ebit_film_state *s) {
  if (!s || !s->node_color || !s->cell_color || !s->hcount || !s->hoff || !s->vcount || !s->voff) return EBIT_ERR_ARG;
  const size_t nx = g->nx, ny = g->ny;
  const uint8_t *c = s->node_color;
  for (size_t k = 0; k < (nx + 1) * (ny + 1); k++)
    if (c[k] > 1) return EBIT_ERR_ARG;
  for (size_t k = 0; k < nx * ny; k++)
    if (s->cell_color[k] > 1) return EBIT_ERR_ARG;
  auto edge_ok = [](int n, int differ, const double *o) -> bool {
    if (n > 2 || (n & 1) != differ) return false;
    for (int k = 0; k < n; k++)
      if (!(o[k] >= 0.0 && o[k] <= 1.0)) return false;
    return n < 2 || o[0] <= o[1];
  };
  for (size_t j = 0; j <= ny; j++)
    for (size_t i = 0; i < nx; i++) {
      const size_t e = j * nx + i;
      if (!edge_ok(s->hcount[e], c[j * (nx + 1) + i] != c[j * (nx + 1) + i + 1], s->hoff + 2 * e)) return EBIT_ERR_ARG;
    }
  for (size_t j = 0; j < ny; j++)
    for (size_t i = 0; i <= nx; i++) {
      const size_t e = j * (nx + 1) + i;
      if (!edge_ok(s->vcount[e], c[j * (nx + 1) + i] != c[(j + 1) * (nx + 1) + i], s->voff + 2 * e))
        return EBIT_ERR_ARG;
    }
  return EBIT_OK;
}

struct Layout {
  Buf buf[2];
  double2 *sp, *dv;
  uint8_t *kept;
  int8_t *res;
  uint32_t *err;
  unsigned long long *ctr;
  Compact wk;
  size_t bytes;
};

Layout carve(const ebit_grid &g, char *base) {
  const size_t nx = g.nx, ny = g.ny, N = (nx + 1) * (ny + 1), Cn = nx * ny, H = (ny + 1) * nx, V = ny * (nx + 1);
  const size_t M = H > V ? H : V;
  Carve c{base};
  Layout L;
  for (int k = 0; k < 2; k++) {
    L.buf[k].col = c.take<uint8_t>(N);
    L.buf[k].cen = c.take<uint8_t>(Cn);
    L.buf[k].hn = c.take<uint8_t>(H);
    L.buf[k].vn = c.take<uint8_t>(V);
    L.buf[k].ho = c.take<double2>(H);
    L.buf[k].vo = c.take<double2>(V);
  }
  L.sp = c.take<double2>(M);
  L.dv = c.take<double2>(M);
  L.kept = c.take<uint8_t>(2 * M);
  L.res = c.take<int8_t>(4 * M);
  L.err = c.take<uint32_t>(1);
  L.ctr = c.take<unsigned long long>((size_t)F_PARTS * F_STRIDE);
  // a count per workgroup of the widest, tallest quiet launch, and a slot per
  // element of it
  const size_t side = (nx > ny ? nx : ny) + 1;
  const size_t bx = (side + BS - 1) / BS, runs = (side + KX - 1) / KX;
  const size_t nq = bx * (runs < 32768 ? runs : 32768);
  L.wk.cnt = c.take<uint32_t>(nq);
  L.wk.slot = c.take<uint2>(nq * (BS * KX > BS * KR ? BS * KX : BS * KR));
  L.bytes = (c.off + 255) & ~(size_t)255;
  return L;
}

}  // namespace ebit_film_impl

using namespace ebit_film_impl;

struct ebit_film {
  ebit_grid g;
  double delta;
  hipStream_t stream;
  int64_t step;
  int cur;
  Layout L;
};

namespace {

int upload(ebit_film *f, const ebit_film_state *s) {
  const size_t nx = f->g.nx, ny = f->g.ny, N = (nx + 1) * (ny + 1), Cn = nx * ny, H = (ny + 1) * nx,
               V = ny * (nx + 1);
  const Buf &B = f->L.buf[f->cur];
  bool ok = hipMemcpyAsync(B.col, s->node_color, N, hipMemcpyHostToDevice, f->stream) == hipSuccess &&
            hipMemcpyAsync(B.cen, s->cell_color, Cn, hipMemcpyHostToDevice, f->stream) == hipSuccess &&
            hipMemcpyAsync(B.hn, s->hcount, H, hipMemcpyHostToDevice, f->stream) == hipSuccess &&
            hipMemcpyAsync(B.vn, s->vcount, V, hipMemcpyHostToDevice, f->stream) == hipSuccess &&
            hipMemcpyAsync(B.ho, s->hoff, H * sizeof(double2), hipMemcpyHostToDevice, f->stream) == hipSuccess &&
            hipMemcpyAsync(B.vo, s->voff, V * sizeof(double2), hipMemcpyHostToDevice, f->stream) == hipSuccess &&
            hipMemsetAsync(f->L.err, 0, sizeof(uint32_t), f->stream) == hipSuccess &&
            hipMemsetAsync(f->L.ctr, 0, (size_t)F_PARTS * F_STRIDE * sizeof(unsigned long long), f->stream) == hipSuccess &&
            hipStreamSynchronize(f->stream) == hipSuccess;
  return ok ? EBIT_OK : EBIT_ERR_DEVICE;
}

// a launch over `rows` rows of `width` elements: x along a row, y over the rows
// (grid rows stride the array's rows beyond the y limit)
dim3 rowsGrid(size_t width, size_t rows, int k) {
  const size_t runs = (rows + (size_t)k - 1) / (size_t)k;
  return dim3((unsigned)((width + BS - 1) / BS), (unsigned)(runs < 32768 ? runs : 32768));
}

template <int DIR>
int sweep(ebit_film *f, const double *vel, double lam) {
  SweepArgs A;
  A.nx = f->g.nx;
  A.ny = f->g.ny;
  A.lam = lam;
  A.delta = f->delta;
  A.cur = f->L.buf[f->cur];
  A.nxt = f->L.buf[f->cur ^ 1];
  A.vel = vel;
  A.sp = f->L.sp;
  A.dv = f->L.dv;
  A.kept = f->L.kept;
  A.res = f->L.res;
  A.err = f->L.err;
  A.ctr = f->L.ctr;
  A.wk = f->L.wk;
  const size_t nx = A.nx, ny = A.ny;
  // physical shapes (rows x width) of the frame's aligned and unaligned arrays
  const size_t rA = DIR == 0 ? ny + 1 : ny, wA = DIR == 0 ? nx : nx + 1;
  const size_t rU = DIR == 0 ? ny : ny + 1, wU = DIR == 0 ? nx + 1 : nx;
  hipLaunchKernelGGL(k_film_advect<DIR>, rowsGrid(nx + 1, rA + rU, KR), dim3(BS), 0, f->stream, A);
  hipLaunchKernelGGL(k_film_flip<DIR>, rowsGrid(nx + 1, ny + 1, KR), dim3(BS), 0, f->stream, A);
  hipLaunchKernelGGL(k_film_land<DIR>, rowsGrid(wA, rA, KR), dim3(BS), 0, f->stream, A);
  const dim3 gq = rowsGrid(wU, rU, KX);
  const uint32_t nq = gq.x * gq.y;
  hipLaunchKernelGGL(k_film_cross_quiet<DIR>, gq, dim3(BS), 0, f->stream, A);
  hipLaunchKernelGGL(k_film_cross<DIR>, dim3((nq + GW - 1) / GW), dim3(64), 0, f->stream, A, nq);
  hipLaunchKernelGGL(k_film_centre<DIR>, rowsGrid(nx, ny, KR), dim3(BS), 0, f->stream, A);
  if (hipGetLastError() != hipSuccess) return EBIT_ERR_DEVICE;
  f->cur ^= 1;
  return EBIT_OK;
}

int latched(ebit_film *f) {
  if (hipStreamSynchronize(f->stream) != hipSuccess) return EBIT_ERR_DEVICE;
  uint32_t e = 0;
  if (hipMemcpy(&e, f->L.err, sizeof e, hipMemcpyDeviceToHost) != hipSuccess) return EBIT_ERR_DEVICE;
  if (e & ERR_CFL) return EBIT_ERR_CFL;
  if (e & ERR_DOMAIN) return EBIT_ERR_DOMAIN;
  return EBIT_OK;
}

}  // namespace

extern "C" {

int ebit_film_workspace_bytes(const ebit_grid *grid, size_t *bytes) {
  if (!grid_ok(grid) || !bytes) return EBIT_ERR_ARG;
  *bytes = carve(*grid, nullptr).bytes;
  return EBIT_OK;
}

int ebit_film_create(const ebit_grid *grid, double delta, const ebit_film_state *init, int64_t step, void *ws_dev,
                     size_t ws_bytes, void *stream, ebit_film **out) {
  if (!out) return EBIT_ERR_ARG;
  *out = nullptr;
  if (!grid_ok(grid) || !ws_dev || !(delta >= 0.0) || step < 0) return EBIT_ERR_ARG;
  const int rc = validate(grid, init);
  if (rc) return rc;
  const Layout L = carve(*grid, (char *)ws_dev);
  if (ws_bytes < L.bytes) return EBIT_ERR_NOMEM;
  ebit_film *f = new (std::nothrow) ebit_film;
  if (!f) return EBIT_ERR_NOMEM;
  f->g = *grid;
  f->delta = delta;
  f->stream = (hipStream_t)stream;
  f->step = step;
  f->cur = 0;
  f->L = L;
  const int up = upload(f, init);
  if (up) {
    delete f;
    return up;
  }
  *out = f;
  return EBIT_OK;
}

int ebit_film_advect(ebit_film *f, const double *u_dev, const double *v_dev, double dt) {
  if (!f || !u_dev || !v_dev || !isfinite(dt)) return EBIT_ERR_ARG;
  const double lam = dt / f->g.h;
  const bool xFirst = (f->step & 1) == 0;
  int rc = xFirst ? sweep<0>(f, u_dev, lam) : sweep<1>(f, v_dev, lam);
  if (!rc) rc = xFirst ? sweep<1>(f, v_dev, lam) : sweep<0>(f, u_dev, lam);
  f->step++;
  return rc;
}

int ebit_film_fraction(ebit_film *f, double *C_dev) {
  if (!f || !C_dev) return EBIT_ERR_ARG;
  const dim3 gq = rowsGrid(f->g.nx, f->g.ny, KR);
  const uint32_t nq = gq.x * gq.y;
  hipLaunchKernelGGL(k_film_fraction_quiet, gq, dim3(BS), 0, f->stream, f->g.nx, f->g.ny, f->L.buf[f->cur], C_dev,
                     f->L.wk);
  hipLaunchKernelGGL(k_film_fraction, dim3((nq + GW - 1) / GW), dim3(64), 0, f->stream, f->g.nx, f->g.ny,
                     f->L.buf[f->cur], C_dev, f->L.wk, nq);
  return hipGetLastError() == hipSuccess ? EBIT_OK : EBIT_ERR_DEVICE;
}

int ebit_film_get_state(ebit_film *f, const ebit_film_out *out) {
  if (!f || !out || !out->node_color || !out->cell_color || !out->hcount || !out->hoff || !out->vcount || !out->voff)
    return EBIT_ERR_ARG;
  const int rc = latched(f);
  if (rc) return rc;
  const size_t nx = f->g.nx, ny = f->g.ny, N = (nx + 1) * (ny + 1), Cn = nx * ny, H = (ny + 1) * nx,
               V = ny * (nx + 1);
  const Buf &B = f->L.buf[f->cur];
  const bool ok = hipMemcpy(out->node_color, B.col, N, hipMemcpyDeviceToHost) == hipSuccess &&
                  hipMemcpy(out->cell_color, B.cen, Cn, hipMemcpyDeviceToHost) == hipSuccess &&
                  hipMemcpy(out->hcount, B.hn, H, hipMemcpyDeviceToHost) == hipSuccess &&
                  hipMemcpy(out->vcount, B.vn, V, hipMemcpyDeviceToHost) == hipSuccess &&
                  hipMemcpy(out->hoff, B.ho, H * sizeof(double2), hipMemcpyDeviceToHost) == hipSuccess &&
                  hipMemcpy(out->voff, B.vo, V * sizeof(double2), hipMemcpyDeviceToHost) == hipSuccess;
  if (!ok) return EBIT_ERR_DEVICE;
  // the device writes offset pairs only for edges that hold markers: the
  // slots past each edge's count read as 0
  for (size_t e = 0; e < H; e++)
    for (int k = out->hcount[e]; k < 2; k++) out->hoff[2 * e + k] = 0.0;
  for (size_t e = 0; e < V; e++)
    for (int k = out->vcount[e]; k < 2; k++) out->voff[2 * e + k] = 0.0;
  return EBIT_OK;
}

int ebit_film_set_state(ebit_film *f, const ebit_film_state *s, int64_t step) {
  if (!f || step < 0) return EBIT_ERR_ARG;
  const int rc = validate(&f->g, s);
  if (rc) return rc;
  if (hipStreamSynchronize(f->stream) != hipSuccess) return EBIT_ERR_DEVICE;
  f->step = step;
  return upload(f, s);
}

int ebit_film_stats(ebit_film *f, ebit_film_counters *out) {
  if (!f || !out) return EBIT_ERR_ARG;
  const int rc = latched(f);
  if (rc) return rc;
  unsigned long long p[F_PARTS * F_STRIDE], c[F_NCTR] = {0, 0, 0, 0, 0};
  if (hipMemcpy(p, f->L.ctr, sizeof p, hipMemcpyDeviceToHost) != hipSuccess) return EBIT_ERR_DEVICE;
  for (int q = 0; q < F_PARTS; q++)
    for (int k = 0; k < F_NCTR; k++) c[k] += p[q * F_STRIDE + k];
  out->markers = (int64_t)c[F_MARKERS];
  out->annihilated = (int64_t)c[F_ANNIH];
  out->annihilated_unaligned = (int64_t)c[F_ANNIH_UN];
  out->three_crossings = (int64_t)c[F_THREE];
  out->parity_fail = (int64_t)c[F_PARITY];
  return EBIT_OK;
}

int ebit_film_sync(ebit_film *f) {
  if (!f) return EBIT_ERR_ARG;
  return latched(f);
}

int ebit_film_destroy(ebit_film *f) {
  if (!f) return EBIT_ERR_ARG;
  delete f;
  return EBIT_OK;
}

}  // extern "C"
