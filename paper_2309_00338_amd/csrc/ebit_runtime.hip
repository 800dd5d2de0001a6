// EBIT interface step: host runtime behind the C-ABI in include/ebit.h.
//
// An engine holds any number of grids in one device workspace: the shared
// tile tables, lists and counters, a descriptor per grid, and per grid both
// copies of the state and the sweep scratch. One launch per phase serves all
// grids. The single-grid handle is an engine with one grid; the batch holds a
// fixed set of grids whose velocities and output fields the caller packs into
// shared buffers; the pool admits and retires grids between steps and keeps
// each grid's velocities and fields in its own arena. Nothing here allocates
// device memory: every byte comes from the caller's workspace.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <vector>

#include "ebit.h"
#include "ebit_internal.h"

using namespace ebit;

namespace {

// the last failed HIP call of this thread, for ebit_device_error()
thread_local char g_devErr[256] = "";

int device_failed(hipError_t err, const char *what, int line) {
  snprintf(g_devErr, sizeof g_devErr, "%s (%d) from %.160s at runtime line %d", hipGetErrorName(err), (int)err, what,
           line);
  return EBIT_ERR_DEVICE;
}

#define HIPCHK(x)                                                    \
  do {                                                               \
    const hipError_t err_ = (x);                                     \
    if (err_ != hipSuccess) return device_failed(err_, #x, __LINE__); \
  } while (0)

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

struct Carve {
  size_t off = 0;
  template <class T>
  T *take(char *base, size_t n) {
    off = align256(off);
    T *p = base ? (T *)(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

bool grid_ok(const ebit_grid *g) {
  return g && g->nx >= 4 && g->ny >= 4 && g->nx <= 65535 && g->ny <= 65535 && isfinite(g->h) && g->h > 0.0 &&
         (g->flags & ~3u) == 0;
}

uint32_t tiles_of(const ebit_grid &g) { return (uint32_t)(((g.nx + TS - 1) / TS) * ((g.ny + TS - 1) / TS)); }

constexpr uint32_t MAX_POOL_TILES = (1u << 24) - 1u;  // keeps the job list within 32-bit indices
constexpr uint32_t JOBS_PER_TILE = TS * TS;            // interior unaligned edges a tile owns, at most

// Job-queue region of an engine of one grid: a share of its active list (at
// most ceil(tiles / NJQ) tiles) queues at most JOBS_PER_TILE jobs per tile.
size_t one_job_region(const ebit_grid &g) { return (size_t)JOBS_PER_TILE * ((tiles_of(g) + NJQ - 1) / NJQ); }

// Fit-job list entries a grid needs. A sweep queues one job per new interior
// unaligned marker: at most (nx-1)*ny for an x sweep, nx*(ny-1) for a y sweep.
// With several grids each grid sweeps one direction per phase and its centre
// rules run before the next phase, so one direction's bound suffices. An
// engine of one grid leaves the first sweep's jobs in the list (read from the
// other end) until the second sweep's launch has run their centre rules, so
// both directions' jobs are alive at once, and each direction queues them in
// NJQ regions: the list holds 2 NJQ regions (at least both directions'
// bounds, since a region covers TS * TS cells of every tile of a share).
size_t jobs_of(const ebit_grid &g, bool both) {
  const size_t x = (size_t)(g.nx - 1) * g.ny, y = (size_t)g.nx * (g.ny - 1);
  return both ? 2 * NJQ * one_job_region(g) : std::max(x, y);
}

// Job-queue span of an engine of several grids. A sweep launch hands
// workgroup b a contiguous chunk of c = max(ceil(n / G), m) of its n active
// tiles (G workgroups, m the minimum chunk) and b queues on queue b % NJQ, so
// queue q takes at most c ceil(ceil(n / c) / NJQ) < n / NJQ + c tiles, and at
// most n. The x- and y-sweep launches of a phase share the list from both
// ends (n_x + n_y <= N tiles), queue q of the one and NJQ-1-q of the other in
// span q, which therefore holds JOBS_PER_TILE min(N, ceil(N / NJQ) + 1 + 2 c)
// entries, c taken at N.
size_t multi_job_span(uint32_t N, uint32_t G, uint32_t m) {
  const size_t c = std::max<size_t>((N + (size_t)G - 1) / std::max<uint32_t>(G, 1u), std::max<uint32_t>(m, 1u));
  return (size_t)JOBS_PER_TILE * std::min<size_t>(N, (N + NJQ - 1) / NJQ + 1 + 2 * c);
}
// the list of several grids (or a pool's N tiles) is sized for NJQ spans at
// the default schedule on a GPU of at least this many sweep workgroups; a
// smaller launch, or a larger minimum chunk, falls back to one queue
constexpr uint32_t REF_SWEEP_BLOCKS = 2048;
constexpr uint32_t REF_MIN_CHUNK = 8;
// entries for N tiles whose one-queue bound is `single`: the larger of the
// two, unless the spans would pass 32-bit indices
size_t multi_job_cap(uint32_t N, size_t single) {
  const size_t q = NJQ * multi_job_span(N, REF_SWEEP_BLOCKS, REF_MIN_CHUNK);
  return q < 0xffffffffull ? std::max(single, q) : single;
}

// Host records of an engine's grids. One grid is held inline, so that an
// engine of one grid needs no heap memory (the entry point that allocates
// nothing relies on it); more grids live on the heap.
template <class T>
struct GridRecords {
  T inl{};
  std::vector<T> heap;
  T *p = &inl;
  GridRecords() = default;
  GridRecords(const GridRecords &) = delete;
  GridRecords &operator=(const GridRecords &) = delete;
  void assign(size_t n, const T &v) {
    if (n <= 1) {
      inl = v;
      p = &inl;
    } else {
      heap.assign(n, v);
      p = heap.data();
    }
  }
  void assign(const T *b, const T *e) {
    if (e - b <= 1) {
      if (e > b) inl = *b;
      p = &inl;
    } else {
      heap.assign(b, e);
      p = heap.data();
    }
  }
  T &operator[](size_t i) { return p[i]; }
  const T &operator[](size_t i) const { return p[i]; }
};

}  // namespace

// One grid's host-side descriptor copy lives here; the device copy is what
// the kernels read.
struct Engine {
  hipStream_t stream = nullptr;
  uint32_t ntiles = 0;  // global tile space
  uint32_t maxGrids = 0;
  uint32_t jobCap = 0;
  // the single-grid kernels (descriptor in the kernel arguments, every tile of
  // the engine the grid's): only for a fixed engine of exactly one grid, never
  // for a pool, whose slot may be empty and whose tile space is larger
  bool one = false;
  int sweepBlocks = 0, fitBlocks = 0, centreBlocks = 0, nearBlocks[3] = {0, 0, 0}, nsNearBlocks = 0;
  ebit_schedule sched{};  // as set by the caller (0 = device default)
  ebit_schedule used{};   // resolved
  // device tables
  Inst *dinst = nullptr;
  uint32_t *tileInst = nullptr, *counts = nullptr, *errs = nullptr;
  uint2 *actList = nullptr, *nearList = nullptr, *fracList = nullptr;  // (global tile, grid)
  uint16_t *has = nullptr;
  uint8_t *nearPrev = nullptr, *tinfo = nullptr;
  uint2 *jobs = nullptr;
  unsigned long long *ctr = nullptr;
  GhfEntry *ghf = nullptr;      // cells left for the parabola fit, 4 entries per tile at most
  uint32_t *ghfCnt = nullptr;   // entry counts of the two curvature-launch parities, a line each
  uint32_t ghfPar = 0;          // parity of the next curvature launch
  int ghfBlocks = 0;
  // the fraction pass's linear fill: (first chunk, grid) per live grid (several
  // grids only) and the chunk total. Its host source is a ring of slots, each
  // rewritten only once the stream has passed that slot's last copy: a pool's
  // steps do not wait on the stream, and a copy from pageable memory may read
  // its source only when the stream reaches it.
  uint2 *fillTab = nullptr;
  static constexpr int FILL_RING = 4;
  std::vector<uint2> fillHost[FILL_RING];
  hipEvent_t fillDone[FILL_RING] = {};
  bool fillQueued[FILL_RING] = {};
  int fillNext = 0;
  uint32_t fillGrids = 0, fillTotal = 0;
  // host mirror
  GridRecords<Inst> hinst;
  GridRecords<uint8_t> live;
  GridRecords<ebit_grid> grids;
  uint32_t cur = 0, stepNo = 0;
  int slot = 1;
  // one grid: the first sweep's centre rules, run by the second sweep's launch
  const uint32_t *pendJobs = nullptr;
  SweepView pendView{};
  int pendDir = 0;
  SweepArgs pendArgs{};  // to launch them on their own when no second sweep follows
  int64_t epoch = 0, fracEpoch = -1;
  Engine() = default;
  Engine(const Engine &) = delete;
  Engine &operator=(const Engine &) = delete;
  ~Engine() {
    for (hipEvent_t ev : fillDone)
      if (ev) (void)hipEventDestroy(ev);
  }
};

namespace {

// node colours, one byte per node (row-major, (ny+1) x (nx+1)), to and from
// the device bit plane (cb_word); bits outside the grid stay 0
std::vector<uint16_t> pack_colours(const uint8_t *c, int nx, int ny) {
  std::vector<uint16_t> w(cb_words(nx, ny), 0);
  for (int y = 0; y <= ny; y++) {
    const uint8_t *row = c + (size_t)y * (nx + 1);
    for (int x0 = 0; x0 <= nx; x0 += 16) {
      uint32_t v = 0;
      for (int i = 0; i < 16 && x0 + i <= nx; i++) v |= (uint32_t)(row[x0 + i] != 0) << i;
      w[cb_word(nx, x0, y)] = (uint16_t)v;
    }
  }
  return w;
}
void unpack_colours(const std::vector<uint16_t> &w, int nx, int ny, uint8_t *c) {
  for (int y = 0; y <= ny; y++)
    for (int x = 0; x <= nx; x++) c[(size_t)y * (nx + 1) + x] = (uint8_t)((w[cb_word(nx, x, y)] >> (x & 15)) & 1u);
}

// per-grid device arrays: both state copies and the sweep scratch
void carve_grid(Inst *I, const ebit_grid &g, char *base, Carve &c) {
  const size_t nx = g.nx, ny = g.ny;
  const size_t nn = (nx + 1) * (ny + 1), nc = nx * ny, nh = nx * (ny + 1), nv = (nx + 1) * ny;
  for (int k = 0; k < 2; k++) {
    I->col[k] = c.take<uint16_t>(base, cb_words(g.nx, g.ny));
    I->hoff[k] = c.take<double>(base, nh);
    I->voff[k] = c.take<double>(base, nv);
  }
  // centre colours are single-buffered: a sweep leaves them unchanged and its
  // centre kernel, which runs after every fit has read the old values,
  // rewrites the cells it settles in place
  I->cen[0] = I->cen[1] = c.take<uint8_t>(base, nc);
  I->sp = c.take<double>(base, nn);
  I->dd = c.take<double>(base, 2 * nn);
  I->zr = c.take<uint8_t>(base, nn);
}

size_t grid_bytes(const ebit_grid &g) {
  Inst tmp;
  Carve c;
  carve_grid(&tmp, g, nullptr, c);
  return align256(c.off);
}

int validate_state(const ebit_grid *g, const ebit_state *s) {
  if (!s || !s->node_color || !s->cell_color || !s->hoff || !s->voff) return EBIT_ERR_ARG;
  const size_t nx = g->nx, ny = g->ny;
  const uint8_t *c = s->node_color;
  for (size_t k = 0; k < (nx + 1) * (ny + 1); k++)
    if (c[k] > 1) return EBIT_ERR_ARG;
  for (size_t k = 0; k < nx * ny; k++)
    if (s->cell_color[k] > 1) return EBIT_ERR_ARG;
  for (size_t j = 0; j <= ny; j++)
    for (size_t i = 0; i < nx; i++)
      if (c[j * (nx + 1) + i] != c[j * (nx + 1) + i + 1]) {
        double o = s->hoff[j * nx + i];
        if (!(o >= 0.0 && o <= 1.0)) return EBIT_ERR_ARG;
      }
  for (size_t j = 0; j < ny; j++)
    for (size_t i = 0; i <= nx; i++)
      if (c[j * (nx + 1) + i] != c[(j + 1) * (nx + 1) + i]) {
        double o = s->voff[j * (nx + 1) + i];
        if (!(o >= 0.0 && o <= 1.0)) return EBIT_ERR_ARG;
      }
  return EBIT_OK;
}

// First-fit allocator over [0, cap): tile ranges and arena bytes of the pool.
struct RangeAlloc {
  std::map<size_t, size_t> freeRuns;  // start -> length
  void init(size_t cap) {
    freeRuns.clear();
    if (cap) freeRuns[0] = cap;
  }
  bool take(size_t n, size_t align, size_t *start) {
    for (auto it = freeRuns.begin(); it != freeRuns.end(); ++it) {
      const size_t s0 = it->first, len = it->second;
      const size_t s = (s0 + align - 1) / align * align;
      if (s - s0 + n > len) continue;
      freeRuns.erase(it);
      if (s > s0) freeRuns[s0] = s - s0;
      if (s0 + len > s + n) freeRuns[s + n] = s0 + len - (s + n);
      *start = s;
      return true;
    }
    return false;
  }
  void give(size_t s, size_t n) {
    auto it = freeRuns.emplace(s, n).first;
    auto nx = std::next(it);
    if (nx != freeRuns.end() && s + n == nx->first) {
      it->second += nx->second;
      freeRuns.erase(nx);
    }
    if (it != freeRuns.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        freeRuns.erase(it);
      }
    }
  }
};

void carve_engine(Engine *e, char *base, Carve &c) {
  e->dinst = c.take<Inst>(base, e->maxGrids);
  e->errs = c.take<uint32_t>(base, e->maxGrids);
  e->tileInst = c.take<uint32_t>(base, e->ntiles);
  e->has = c.take<uint16_t>(base, e->ntiles);
  e->nearPrev = c.take<uint8_t>(base, e->ntiles);
  e->tinfo = c.take<uint8_t>(base, e->ntiles);
  e->actList = c.take<uint2>(base, e->ntiles);
  e->nearList = c.take<uint2>(base, e->ntiles);
  e->fracList = c.take<uint2>(base, e->ntiles);
  e->counts = c.take<uint32_t>(base, 2 * NSLOT);
  e->jobs = c.take<uint2>(base, e->jobCap);
  e->ctr = c.take<unsigned long long>(base, (size_t)CTR_PARTS * CTR_STRIDE);
  e->ghf = c.take<GhfEntry>(base, 4 * (size_t)e->ntiles);
  e->ghfCnt = c.take<uint32_t>(base, 2 * CNT_LINE);
  e->fillTab = c.take<uint2>(base, e->maxGrids);
}

// engine tables for ntiles tiles, maxGrids grids and jobCap fit jobs
size_t engine_bytes(uint32_t ntiles, uint32_t maxGrids, uint32_t jobCap) {
  Engine tmp;
  tmp.ntiles = ntiles;
  tmp.maxGrids = maxGrids;
  tmp.jobCap = jobCap;
  Carve c;
  carve_engine(&tmp, nullptr, c);
  return align256(c.off);
}

// Default schedule: every resident sweep and fit workgroup; 8 tiles per
// sweep workgroup at least with several grids; 5.5 of the 8 resident
// fraction-pass slots per CU for the tiles with cut cells, so that fill
// workgroups run beside them from the start and take the other slots as they
// finish (8192^2 with the fill's streaming stores: call 240 -> 192 us against
// all 8 slots; the batch of 256 grids: 679 -> 658 us per step); 6 for the
// interface consumers.
constexpr double DEF_FRAC_NEAR = 5.5, DEF_NS_NEAR = 6.0;
constexpr uint32_t DEF_MIN_CHUNK = 8;

void engine_launch_config(Engine *e) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  const ebit_schedule &s = e->sched;
  const int rs = resident_blocks(0), rf = resident_blocks(1);
  const int sp = s.sweep_per_cu ? std::min((int)s.sweep_per_cu, rs) : rs;
  const int fp = s.fit_per_cu ? std::min((int)s.fit_per_cu, rf) : rf;
  e->sweepBlocks = cus * sp;
  e->fitBlocks = cus * fp;
  e->centreBlocks = cus * resident_blocks(2);
  e->ghfBlocks = cus * 16;  // single-wavefront workgroups, one per parabola-fit entry in the usual case
  const double perCU = s.frac_near_per_cu > 0.0 ? s.frac_near_per_cu : DEF_FRAC_NEAR;
  const double nsPerCU = s.ns_near_per_cu > 0.0 ? s.ns_near_per_cu : DEF_NS_NEAR;
  const int rn = resident_blocks(5);
  e->nsNearBlocks = std::max(1, std::min((int)(cus * nsPerCU), cus * rn));
  for (int m = 0; m < 3; m++) {
    const int cap = cus * resident_blocks(3 + m);
    const int nb = std::min((int)(cus * perCU), cap);
    e->nearBlocks[m] = nb < 1 ? 1 : nb;
  }
  e->used.sweep_per_cu = (uint32_t)sp;
  e->used.fit_per_cu = (uint32_t)fp;
  e->used.sweep_min_chunk = s.sweep_min_chunk ? s.sweep_min_chunk : DEF_MIN_CHUNK;
  e->used.frac_near_per_cu = std::min(perCU, (double)resident_blocks(5));
  e->used.ns_near_per_cu = std::min(nsPerCU, (double)rn);
}

bool schedule_ok(const ebit_schedule *s) {
  return s && isfinite(s->frac_near_per_cu) && isfinite(s->ns_near_per_cu) && s->frac_near_per_cu >= 0.0 &&
         s->ns_near_per_cu >= 0.0 && s->sweep_min_chunk <= (1u << 20);
}

// The fill's chunk table of the live grids. One grid needs none (its chunks
// start at 0). The upload reads the host vector before the call returns
// (pageable source), so rebuilding it later is safe.
int engine_fill_table(Engine *e) {
  if (e->one) {
    // 16 tiles per workgroup when tile rows are whole lines, else 16 virtual
    // rows of pitch nx rounded up to 16 by 256 columns (decided in the kernel
    // from the output alignment)
    e->fillGrids = 1;
    e->fillTotal = std::max(pitch_chunks(e->hinst[0].nx, e->hinst[0].ny), (e->ntiles + 15u) / 16u);
    return EBIT_OK;
  }
  const int r = e->fillNext;
  if (!e->fillDone[r]) HIPCHK(hipEventCreateWithFlags(&e->fillDone[r], hipEventDisableTiming));
  if (e->fillQueued[r]) HIPCHK(hipEventSynchronize(e->fillDone[r]));
  e->fillQueued[r] = false;
  std::vector<uint2> &h = e->fillHost[r];
  h.clear();
  uint32_t total = 0;
  for (uint32_t k = 0; k < e->maxGrids; k++) {
    if (!e->live[k]) continue;
    h.push_back(make_uint2(total, k));
    total += pitch_chunks(e->hinst[k].nx, e->hinst[k].ny);
  }
  e->fillGrids = (uint32_t)h.size();
  e->fillTotal = total;
  if (e->fillGrids) {
    HIPCHK(hipMemcpyAsync(e->fillTab, h.data(), e->fillGrids * sizeof(uint2), hipMemcpyHostToDevice, e->stream));
    HIPCHK(hipEventRecord(e->fillDone[r], e->stream));
    e->fillQueued[r] = true;
    e->fillNext = (r + 1) % Engine::FILL_RING;
  }
  return EBIT_OK;
}

// clears every table; all tiles start unowned
int engine_reset(Engine *e) {
  HIPCHK(hipMemsetAsync(e->counts, 0, 2 * NSLOT * sizeof(uint32_t), e->stream));
  HIPCHK(hipMemsetAsync(e->ctr, 0, CTR_PARTS * CTR_STRIDE * sizeof(unsigned long long), e->stream));
  HIPCHK(hipMemsetAsync(e->errs, 0, e->maxGrids * sizeof(uint32_t), e->stream));
  HIPCHK(hipMemsetAsync(e->ghfCnt, 0, 2 * CNT_LINE * sizeof(uint32_t), e->stream));
  e->ghfPar = 0;
  HIPCHK(launch_clear_tiles(e->tileInst, e->has, e->nearPrev, e->tinfo, 0, e->ntiles, e->stream));
  e->slot = 1;
  return EBIT_OK;
}

CompactArgs compact_args(Engine *e, int afterSweep, uint32_t nextStep, int nextPhase) {
  CompactArgs a;
  a.inst = e->dinst;
  a.tileInst = e->tileInst;
  a.ntiles = e->ntiles;
  a.cur = e->cur;
  a.stepNo = nextStep;
  a.phase = nextPhase;
  a.afterSweep = afterSweep;
  a.slot = e->slot;
  a.has = e->has;
  a.nearPrev = e->nearPrev;
  a.tinfo = e->tinfo;
  a.actList = e->actList;
  a.nearList = e->nearList;
  a.fracList = e->fracList;
  a.counts = e->counts;
  a.one = e->hinst[0];
  return a;
}

int engine_compact(Engine *e, int afterSweep, uint32_t nextStep, int nextPhase) {
  e->slot ^= 1;
  const CompactArgs a = compact_args(e, afterSweep, nextStep, nextPhase);
  HIPCHK(launch_compact(e->one, a, e->stream));
  return EBIT_OK;
}

// writes grid k's descriptor, uploads its state into both copies and marks
// its tiles; the caller lists the tiles afterwards
int engine_place(Engine *e, uint32_t k, const ebit_state *s) {
  const Inst &I = e->hinst[k];
  const size_t nx = I.nx, ny = I.ny;
  const size_t nc = nx * ny, nh = nx * (ny + 1), nv = (nx + 1) * ny;
  HIPCHK(hipMemcpyAsync(e->dinst + k, &e->hinst[k], sizeof(Inst), hipMemcpyHostToDevice, e->stream));
  // the current copy from the host, the other one on the device
  const uint32_t c = e->cur, o = e->cur ^ 1u;
  const size_t ncw = cb_words(I.nx, I.ny);
  const std::vector<uint16_t> packed = pack_colours(s->node_color, I.nx, I.ny);
  HIPCHK(hipMemcpyAsync(I.col[c], packed.data(), ncw * sizeof(uint16_t), hipMemcpyHostToDevice, e->stream));
  HIPCHK(hipMemcpyAsync(I.cen[c], s->cell_color, nc, hipMemcpyHostToDevice, e->stream));
  HIPCHK(hipMemcpyAsync(I.hoff[c], s->hoff, nh * sizeof(double), hipMemcpyHostToDevice, e->stream));
  HIPCHK(hipMemcpyAsync(I.voff[c], s->voff, nv * sizeof(double), hipMemcpyHostToDevice, e->stream));
  HIPCHK(hipMemcpyAsync(I.col[o], I.col[c], ncw * sizeof(uint16_t), hipMemcpyDeviceToDevice, e->stream));
  HIPCHK(hipMemcpyAsync(I.hoff[o], I.hoff[c], nh * sizeof(double), hipMemcpyDeviceToDevice, e->stream));
  HIPCHK(hipMemcpyAsync(I.voff[o], I.voff[c], nv * sizeof(double), hipMemcpyDeviceToDevice, e->stream));
  HIPCHK(hipMemsetAsync(e->errs + k, 0, sizeof(uint32_t), e->stream));
  HIPCHK(launch_init_tiles(e->dinst, k, (uint32_t)(I.ntx * I.nty), e->cur, e->tileInst, e->has, e->nearPrev,
                           e->stream));
  // the uploads read host memory the caller may reuse after return (and the
  // packed colours, freed on return)
  HIPCHK(hipStreamSynchronize(e->stream));
  return EBIT_OK;
}

// launches the centre kernel of a first sweep whose rules no second sweep
// took over
hipError_t engine_flush_centre(Engine *e) {
  if (!e->pendJobs) return hipSuccess;
  e->pendJobs = nullptr;
  return launch_centre(e->pendDir, true, e->pendArgs, e->centreBlocks, e->stream);
}

int engine_sweep(Engine *e, int phase, const double *u, const double *v, const double *dts, double dt) {
  bool dirs[2] = {false, false};
  for (uint32_t k = 0; k < e->maxGrids; k++)
    if (e->live[k]) dirs[sweep_dir(e->hinst[k], e->stepNo, phase)] = true;
  SweepArgs a;
  a.inst = e->dinst;
  a.tileInst = e->tileInst;
  a.u = u;
  a.v = v;
  a.dts = dts;
  a.dt = dt;
  a.cur = e->cur;
  a.ntiles = e->ntiles;
  a.list = e->actList;
  a.has = e->has;
  a.jobs = e->jobs;
  // one grid swept in 8 XCD shares: a queue per share, the y sweep's regions
  // mirrored from the list's end; else one queue, of half the list. Several
  // grids: a queue per workgroup residue b % NJQ in spans of the list, the
  // y-sweeping grids' queues mirrored from the spans' end, when the spans fit
  // the list; else one queue over all of it (the x- and y-sweeping grids'
  // jobs together stay within it)
  if (e->one) {
    const uint32_t reg = (uint32_t)one_job_region(e->grids[0]);
    a.jobQ = e->sweepBlocks % (int)NJQ == 0 ? NJQ : 1u;
    a.jobRegion = a.jobQ == NJQ ? reg : NJQ * reg;
    a.jobTop = e->jobCap;
  } else {
    const size_t span = multi_job_span(e->ntiles, (uint32_t)e->sweepBlocks, e->used.sweep_min_chunk);
    const bool q = NJQ * span <= e->jobCap;
    a.jobQ = q ? NJQ : 1u;
    a.jobRegion = q ? (uint32_t)span : e->jobCap;
    a.jobTop = q ? (uint32_t)(NJQ * span) : e->jobCap;
  }
  a.minChunk = e->used.sweep_min_chunk;
  a.ctr = e->ctr;
  a.pendJobs = nullptr;
  uint32_t *cs = e->counts + NSLOT * e->slot;
  const uint32_t nextStep = phase == 0 ? e->stepNo : e->stepNo + 1;
  if (!dirs[0] && !dirs[1]) {
    HIPCHK(engine_flush_centre(e));
    e->cur ^= 1u;
    return engine_compact(e, 1, nextStep, phase == 0 ? 1 : 0);
  }
  // the compaction of the swept state rides with the last fit launch
  const int last = dirs[1] ? 1 : 0;
  e->cur ^= 1u;
  e->slot ^= 1;
  const CompactArgs c = compact_args(e, 1, nextStep, phase == 0 ? 1 : 0);
  e->cur ^= 1u;
  e->slot ^= 1;
  for (int d = 0; d < 2; d++) {
    if (!dirs[d]) continue;
    a.count = cs + (d == 0 ? CNT_ACT_X : CNT_ACT_Y);
    a.njobs = cs + (d == 0 ? CNT_JOBS_X : CNT_JOBS_Y);
    // the single grid's view, resolved here (the kernels read it from their arguments)
    // (with per-grid device dts the single-grid sweep reads lambda from dts[0])
    a.one = sweep_view(e->hinst[0], e->cur, d, u, v, dts ? 0.0 : dt / e->hinst[0].h);
    // one grid: the first sweep's centre rules ride with the second sweep (it
    // reads neither centre colours nor the first fits' results, and the
    // second fits, which read both, start after it)
    const bool fold = e->one && e->pendJobs && e->pendDir != d;
    if (fold) {
      a.pendJobs = e->pendJobs;
      a.pend = e->pendView;
    } else {
      HIPCHK(engine_flush_centre(e));
    }
    HIPCHK(launch_sweep(d, e->one, a, e->sweepBlocks, e->stream));
    a.pendJobs = nullptr;
    e->pendJobs = nullptr;
    HIPCHK(launch_fit(d, e->one, a, e->fitBlocks, d == last ? &c : nullptr, e->stream));
    if (e->one && phase == 0) {
      e->pendJobs = a.njobs;
      e->pendView = a.one;
      e->pendDir = d;
      e->pendArgs = a;
    } else {
      HIPCHK(launch_centre(d, e->one, a, e->centreBlocks, e->stream));
    }
  }
  e->cur ^= 1u;
  e->slot ^= 1;
  return EBIT_OK;
}

int engine_advect(Engine *e, const double *u, const double *v, const double *dts, double dt) {
  int rc = engine_sweep(e, 0, u, v, dts, dt);
  if (!rc) rc = engine_sweep(e, 1, u, v, dts, dt);
  if (!rc) {
    const hipError_t he = engine_flush_centre(e);
    if (he != hipSuccess) rc = device_failed(he, "engine_flush_centre", __LINE__);
  }
  e->pendJobs = nullptr;
  e->stepNo++;
  e->epoch++;
  return rc;
}

int engine_frac(Engine *e, int mode, const double *Cin, double *Cout, double *Kout) {
  FracArgs a;
  a.inst = e->dinst;
  a.tileInst = e->tileInst;
  a.ntiles = e->ntiles;
  a.cur = e->cur;
  a.Cin = Cin;
  a.Cout = Cout;
  a.Kout = Kout;
  a.tinfo = e->tinfo;
  a.list = e->fracList;
  a.count = e->counts + NSLOT * e->slot + CNT_FRAC;
  a.nearBlocks = e->nearBlocks[mode - 1];
  a.ctr = e->ctr;
  // a curvature launch appends to its parity's count (zeroed by the launch
  // before it) and zeroes the other one for the launch after it
  a.ghf = e->ghf;
  a.ghfCount = e->ghfCnt + CNT_LINE * e->ghfPar;
  a.ghfClear = e->ghfCnt + CNT_LINE * (e->ghfPar ^ 1u);
  a.fillTab = e->fillTab;
  a.fillGrids = e->fillGrids;
  a.one = e->hinst[0];
  HIPCHK(launch_frac_curv(mode, e->one, a, a.nearBlocks + (int)e->fillTotal, e->stream));
  if (mode & 2) {
    // the launch above zeroed the other parity's count: the next curvature
    // launch uses it, whatever happens to the fit launch below
    e->ghfPar ^= 1u;
    HIPCHK(launch_ghf(e->one, a, e->ghfBlocks, e->stream));
  }
  return EBIT_OK;
}

int engine_ns(Engine *e, const double *C, const double *K, const ebit_fluid *f, double *rho, double *mu, double *fx,
              double *fy) {
  if (!C || !K || !f) return EBIT_ERR_ARG;
  if (!isfinite(f->rho1) || !isfinite(f->rho2) || !isfinite(f->mu1) || !isfinite(f->mu2) || !isfinite(f->sigma))
    return EBIT_ERR_ARG;
  if (e->fracEpoch != e->epoch) return EBIT_ERR_STATE;
  NsArgs a;
  a.inst = e->dinst;
  a.tileInst = e->tileInst;
  a.ntiles = e->ntiles;
  a.cur = e->cur;
  a.C = C;
  a.K = K;
  a.rho = rho;
  a.mu = mu;
  a.fx = fx;
  a.fy = fy;
  a.rho1 = f->rho1;
  a.rho2 = f->rho2;
  a.mu1 = f->mu1;
  a.mu2 = f->mu2;
  a.sigma = f->sigma;
  a.tinfo = e->tinfo;
  a.list = e->nearList;
  a.count = e->counts + NSLOT * e->slot + CNT_NEAR;
  a.nearBlocks = e->nsNearBlocks;
  a.one = e->hinst[0];
  const bool one = e->one;
  const int fill = one ? ns_linear_blocks(e->hinst[0].nx, e->hinst[0].ny) : ns_fill_blocks(e->ntiles);
  HIPCHK(launch_ns(one, a, a.nearBlocks + fill, e->stream));
  return EBIT_OK;
}

int status_of(uint32_t bits) {
  if (bits & ERRBIT_ARG) return EBIT_ERR_ARG;
  if (bits & ERRBIT_CAP) return EBIT_ERR_NOMEM;
  if (bits & ERRBIT_CFL) return EBIT_ERR_CFL;
  if (bits & ERRBIT_DOMAIN) return EBIT_ERR_DOMAIN;
  return EBIT_OK;
}

// waits for the stream; per-grid status (optional) and the first error
int engine_errors(Engine *e, int *status) {
  std::vector<uint32_t> bits(e->maxGrids, 0);
  HIPCHK(hipMemcpyAsync(bits.data(), e->errs, e->maxGrids * sizeof(uint32_t), hipMemcpyDeviceToHost, e->stream));
  HIPCHK(hipStreamSynchronize(e->stream));
  int first = EBIT_OK;
  for (uint32_t k = 0; k < e->maxGrids; k++) {
    const int st = e->live[k] ? status_of(bits[k]) : EBIT_OK;
    if (status) status[k] = st;
    if (st && !first) first = st;
  }
  return first;
}

int engine_counters(Engine *e, ebit_counters *out) {
  unsigned long long v[CTR_PARTS * CTR_STRIDE];
  HIPCHK(hipMemcpyAsync(v, e->ctr, sizeof v, hipMemcpyDeviceToHost, e->stream));
  HIPCHK(hipStreamSynchronize(e->stream));
  int64_t *dst = (int64_t *)out;
  for (int k = 0; k < NCOUNTERS; k++) {
    unsigned long long t = 0;
    for (int p = 0; p < CTR_PARTS; p++) t += v[p * CTR_STRIDE + k];
    dst[k] = (int64_t)t;
  }
  return EBIT_OK;
}

int engine_get_state(Engine *e, uint32_t k, uint8_t *node_color, uint8_t *cell_color, double *hoff, double *voff) {
  const Inst &I = e->hinst[k];
  const size_t nx = I.nx, ny = I.ny;
  const uint32_t c = e->cur;
  std::vector<uint16_t> packed(node_color ? cb_words(I.nx, I.ny) : 0);
  if (node_color)
    HIPCHK(hipMemcpyAsync(packed.data(), I.col[c], packed.size() * sizeof(uint16_t), hipMemcpyDeviceToHost, e->stream));
  if (cell_color) HIPCHK(hipMemcpyAsync(cell_color, I.cen[c], nx * ny, hipMemcpyDeviceToHost, e->stream));
  if (hoff) HIPCHK(hipMemcpyAsync(hoff, I.hoff[c], nx * (ny + 1) * sizeof(double), hipMemcpyDeviceToHost, e->stream));
  if (voff) HIPCHK(hipMemcpyAsync(voff, I.voff[c], (nx + 1) * ny * sizeof(double), hipMemcpyDeviceToHost, e->stream));
  HIPCHK(hipStreamSynchronize(e->stream));
  if (node_color) unpack_colours(packed, I.nx, I.ny, node_color);
  return EBIT_OK;
}

void fill_inst(Inst *I, const ebit_grid &g, uint32_t tile0, uint32_t stepPar, uint32_t *err) {
  I->nx = g.nx;
  I->ny = g.ny;
  I->ntx = (g.nx + TS - 1) / TS;
  I->nty = (g.ny + TS - 1) / TS;
  I->tile0 = tile0;
  I->stepPar = stepPar;
  I->flags = ((g.flags & EBIT_SWEEP_XY) ? INST_XY : 0u) | ((g.flags & EBIT_FIT_LINE) ? INST_LINE : 0u);
  I->pad = 0;
  I->h = g.h;
  I->uoff = I->voffv = I->coff = I->koff = 0;
  I->err = err;
}

int batch_sizes(int n, const ebit_grid *grids, uint32_t *ntiles, uint32_t *jobCap, size_t *gridBytes) {
  if (n < 1 || !grids) return EBIT_ERR_ARG;
  size_t nt = 0, nj = 0, gb = 0;
  for (int k = 0; k < n; k++) {
    if (!grid_ok(&grids[k])) return EBIT_ERR_ARG;
    nt += tiles_of(grids[k]);
    nj += jobs_of(grids[k], n == 1);
    gb += grid_bytes(grids[k]);
  }
  if (nt >= 0xffffffffull) return EBIT_ERR_ARG;
  if (n > 1) nj = multi_job_cap((uint32_t)nt, nj);
  if (nj >= 0xffffffffull) return EBIT_ERR_ARG;
  *ntiles = (uint32_t)nt;
  *jobCap = (uint32_t)nj;
  *gridBytes = gb;
  return EBIT_OK;
}

// lays out and fills an engine with n fixed grids (tiles in grid order)
int engine_create_fixed(Engine *e, int n, const ebit_grid *grids, const ebit_state *inits, void *ws, size_t bytes,
                        void *stream) {
  uint32_t ntiles, jobCap;
  size_t gb;
  int rc = batch_sizes(n, grids, &ntiles, &jobCap, &gb);
  if (rc) return rc;
  if (!ws || ((uintptr_t)ws & 255) != 0 || !inits) return EBIT_ERR_ARG;
  for (int k = 0; k < n; k++) {
    rc = validate_state(&grids[k], &inits[k]);
    if (rc) return rc;
  }
  e->ntiles = ntiles;
  e->maxGrids = (uint32_t)n;
  e->one = n == 1;
  e->jobCap = jobCap;
  if (bytes < engine_bytes(ntiles, (uint32_t)n, jobCap) + gb) return EBIT_ERR_NOMEM;
  e->stream = (hipStream_t)stream;
  Carve c;
  carve_engine(e, (char *)ws, c);
  e->hinst.assign(n, Inst());
  e->live.assign(n, 1);
  e->grids.assign(grids, grids + n);
  engine_launch_config(e);
  rc = engine_reset(e);
  if (rc) return rc;
  uint32_t t0 = 0;
  for (int k = 0; k < n; k++) {
    fill_inst(&e->hinst[k], grids[k], t0, 0, e->errs + k);
    carve_grid(&e->hinst[k], grids[k], (char *)ws, c);
    t0 += tiles_of(grids[k]);
  }
  for (int k = 0; k < n; k++) {
    rc = engine_place(e, (uint32_t)k, &inits[k]);
    if (rc) return rc;
  }
  rc = engine_compact(e, 0, e->stepNo, 0);
  if (!rc) rc = engine_fill_table(e);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(e->stream));
  e->epoch++;
  return EBIT_OK;
}

}  // namespace

// single grid: an engine with one grid and the grid's own step count
struct ebit_handle {
  Engine e;
  int64_t step = 0;
};

// batch: fixed grids, velocities and fields packed by the caller
struct ebit_batch {
  Engine e;
  int n = 0;
  std::vector<size_t> uoff, voff, coff;
  size_t utot = 0, vtot = 0, ctot = 0;
};

// pool: grids come and go between steps
struct PoolGrid {
  size_t arenaOff = 0, arenaLen = 0, tile0 = 0;
  int64_t steps = 0;
};

struct ebit_pool {
  Engine e;
  char *arena = nullptr;
  size_t arenaBytes = 0;
  RangeAlloc tileAlloc, arenaAlloc;
  std::vector<PoolGrid> pg;
  double *dts = nullptr;  // device, per slot
  std::vector<double> hdts;
  bool dirty = false;  // grids added or removed since the last listing
};

namespace {
// per-grid arena bytes: state copies and scratch, then u, v, C, K
size_t pool_grid_bytes(const ebit_grid &g) {
  const size_t nx = g.nx, ny = g.ny;
  return grid_bytes(g) + align256(ny * (nx + 1) * 8) + align256((ny + 1) * nx * 8) + 2 * align256(nx * ny * 8) + 256;
}
size_t pool_table_bytes(int max_grids, uint32_t max_tiles) {
  return engine_bytes(max_tiles, (uint32_t)max_grids, (uint32_t)multi_job_cap(max_tiles, (size_t)max_tiles * JOBS_PER_TILE)) +
         align256((size_t)max_grids * sizeof(double));
}
}  // namespace

// ---------------------------------------------------------------------------
// The library's own scratch for ebit_step_static: one array per GPU, in the
// device's global memory, holding the engine tables, both state copies and the
// sweep scratch of one grid. Host code never names the array in a kernel
// argument or copy: on each device it asks once for the array's device address
// (each GPU holds its own copy at its own address) and uses that.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[EBIT_STATIC_SCRATCH_BYTES];

namespace {
constexpr int STATIC_MAX_DEVICES = 64;
struct StaticSlot {
  char *ptr = nullptr;  // device address of `scratch` on this device
  bool ready = false;
  Engine e;             // host record of the grid the scratch holds (one grid: inline)
};
StaticSlot g_static[STATIC_MAX_DEVICES];

// The device's scratch, set up on its first use with the device current.
int static_slot(StaticSlot **out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= STATIC_MAX_DEVICES) return EBIT_ERR_ARG;
  StaticSlot &S = g_static[dev];
  if (!S.ready) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || ((uintptr_t)p & 255) != 0) return EBIT_ERR_DEVICE;
    S.ptr = (char *)p;
    engine_launch_config(&S.e);
    S.ready = true;
  }
  *out = &S;
  return EBIT_OK;
}
}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
// single grid
// ---------------------------------------------------------------------------
int ebit_workspace_bytes(const ebit_grid *grid, size_t *bytes) {
  if (!grid_ok(grid) || !bytes) return EBIT_ERR_ARG;
  const size_t nj = jobs_of(*grid, true);
  if (nj >= 0xffffffffull) return EBIT_ERR_ARG;  // job list past 32-bit indices
  *bytes = engine_bytes(tiles_of(*grid), 1, (uint32_t)nj) + grid_bytes(*grid);
  return EBIT_OK;
}

int ebit_create(const ebit_grid *grid, const ebit_state *init, void *ws_dev, size_t ws_bytes, void *hip_stream,
                ebit_handle **out) {
  if (!out) return EBIT_ERR_ARG;
  *out = nullptr;
  if (!grid_ok(grid) || !ws_dev) return EBIT_ERR_ARG;
  if (((uintptr_t)ws_dev & 255) != 0) return EBIT_ERR_ARG;
  int rc = validate_state(grid, init);
  if (rc) return rc;
  size_t need = 0;
  ebit_workspace_bytes(grid, &need);
  if (ws_bytes < need) return EBIT_ERR_NOMEM;
  ebit_handle *h = new (std::nothrow) ebit_handle();
  if (!h) return EBIT_ERR_NOMEM;
  rc = engine_create_fixed(&h->e, 1, grid, init, ws_dev, ws_bytes, hip_stream);
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return EBIT_OK;
}

int ebit_advect(ebit_handle *h, const double *u_dev, const double *v_dev, double dt) {
  if (!h || !u_dev || !v_dev || !isfinite(dt)) return EBIT_ERR_ARG;
  h->e.stepNo = (uint32_t)(h->step & 1);  // the sweep order follows the grid's own step count
  const int rc = engine_advect(&h->e, u_dev, v_dev, nullptr, dt);
  h->step++;
  return rc;
}

int ebit_fraction(ebit_handle *h, double *C_dev) {
  if (!h || !C_dev) return EBIT_ERR_ARG;
  const int rc = engine_frac(&h->e, 1, nullptr, C_dev, nullptr);
  h->e.fracEpoch = h->e.epoch;
  return rc;
}

int ebit_curvature(ebit_handle *h, const double *C_dev, double *K_dev) {
  if (!h || !C_dev || !K_dev) return EBIT_ERR_ARG;
  if (h->e.fracEpoch != h->e.epoch) return EBIT_ERR_STATE;
  return engine_frac(&h->e, 2, C_dev, nullptr, K_dev);
}

int ebit_fraction_curvature(ebit_handle *h, double *C_dev, double *K_dev) {
  if (!h || !C_dev || !K_dev) return EBIT_ERR_ARG;
  const int rc = engine_frac(&h->e, 3, nullptr, C_dev, K_dev);
  h->e.fracEpoch = h->e.epoch;
  return rc;
}

int ebit_ns_fields(ebit_handle *h, const double *C_dev, const double *K_dev, const ebit_fluid *fluid, double *rho_dev,
                   double *mu_dev, double *fx_dev, double *fy_dev) {
  if (!h) return EBIT_ERR_ARG;
  return engine_ns(&h->e, C_dev, K_dev, fluid, rho_dev, mu_dev, fx_dev, fy_dev);
}

int ebit_get_state(ebit_handle *h, uint8_t *node_color, uint8_t *cell_color, double *hoff, double *voff,
                   int64_t *step) {
  if (!h) return EBIT_ERR_ARG;
  int rc = engine_get_state(&h->e, 0, node_color, cell_color, hoff, voff);
  if (rc) return rc;
  if (step) *step = h->step;
  return engine_errors(&h->e, nullptr);
}

int ebit_set_state(ebit_handle *h, const ebit_state *state, int64_t step) {
  if (!h || step < 0) return EBIT_ERR_ARG;
  int rc = validate_state(&h->e.grids[0], state);
  if (rc) return rc;
  h->step = step;
  h->e.stepNo = (uint32_t)(step & 1);
  rc = engine_place(&h->e, 0, state);  // clears the marker history of every tile of the grid
  if (rc) return rc;
  HIPCHK(hipMemsetAsync(h->e.ctr, 0, CTR_PARTS * CTR_STRIDE * sizeof(unsigned long long), h->e.stream));
  rc = engine_compact(&h->e, 0, h->e.stepNo, 0);
  if (rc) return rc;
  h->e.epoch++;
  return EBIT_OK;
}

int ebit_stats(ebit_handle *h, ebit_counters *out) {
  if (!h || !out) return EBIT_ERR_ARG;
  int rc = engine_counters(&h->e, out);
  if (rc) return rc;
  return engine_errors(&h->e, nullptr);
}

int ebit_get_schedule(const ebit_handle *h, ebit_schedule *out) {
  if (!h || !out) return EBIT_ERR_ARG;
  *out = h->e.used;
  return EBIT_OK;
}

int ebit_set_schedule(ebit_handle *h, const ebit_schedule *s) {
  if (!h || !schedule_ok(s)) return EBIT_ERR_ARG;
  h->e.sched = *s;
  engine_launch_config(&h->e);
  return EBIT_OK;
}

int ebit_stats_reset(ebit_handle *h) {
  if (!h) return EBIT_ERR_ARG;
  HIPCHK(hipMemsetAsync(h->e.ctr, 0, CTR_PARTS * CTR_STRIDE * sizeof(unsigned long long), h->e.stream));
  return EBIT_OK;
}

int ebit_sync(ebit_handle *h) {
  if (!h) return EBIT_ERR_ARG;
  return engine_errors(&h->e, nullptr);
}

int ebit_destroy(ebit_handle *h) {
  if (!h) return EBIT_ERR_ARG;
  delete h;
  return EBIT_OK;
}

// ---------------------------------------------------------------------------
// batch
// ---------------------------------------------------------------------------
int ebit_batch_workspace_bytes(int n, const ebit_grid *grids, size_t *bytes) {
  if (!bytes) return EBIT_ERR_ARG;
  uint32_t ntiles, jobCap;
  size_t gb;
  int rc = batch_sizes(n, grids, &ntiles, &jobCap, &gb);
  if (rc) return rc;
  *bytes = engine_bytes(ntiles, (uint32_t)n, jobCap) + gb;
  return EBIT_OK;
}

int ebit_batch_create(int n, const ebit_grid *grids, const ebit_state *inits, void *ws_dev, size_t ws_bytes,
                      void *hip_stream, ebit_batch **out) {
  if (!out) return EBIT_ERR_ARG;
  *out = nullptr;
  if (n < 1 || !grids || !inits) return EBIT_ERR_ARG;
  ebit_batch *b = new (std::nothrow) ebit_batch();
  if (!b) return EBIT_ERR_NOMEM;
  int rc = engine_create_fixed(&b->e, n, grids, inits, ws_dev, ws_bytes, hip_stream);
  if (rc) {
    delete b;
    return rc;
  }
  b->n = n;
  b->uoff.resize(n);
  b->voff.resize(n);
  b->coff.resize(n);
  size_t u = 0, v = 0, c = 0;
  auto up = [](size_t x) { return (x + 31) & ~(size_t)31; };  // 256-byte aligned starts
  for (int k = 0; k < n; k++) {
    const size_t nx = grids[k].nx, ny = grids[k].ny;
    b->uoff[k] = u;
    b->voff[k] = v;
    b->coff[k] = c;
    u = up(u + ny * (nx + 1));
    v = up(v + (ny + 1) * nx);
    c = up(c + ny * nx);
    Inst &I = b->e.hinst[k];
    I.uoff = b->uoff[k];
    I.voffv = b->voff[k];
    I.coff = I.koff = b->coff[k];
    const hipError_t err = hipMemcpyAsync(b->e.dinst + k, &I, sizeof(Inst), hipMemcpyHostToDevice, b->e.stream);
    if (err != hipSuccess) {
      delete b;
      return device_failed(err, "descriptor upload", __LINE__);
    }
  }
  b->utot = u;
  b->vtot = v;
  b->ctot = c;
  const hipError_t serr = hipStreamSynchronize(b->e.stream);
  if (serr != hipSuccess) {
    delete b;
    return device_failed(serr, "hipStreamSynchronize", __LINE__);
  }
  *out = b;
  return EBIT_OK;
}

int ebit_batch_layout(const ebit_batch *b, size_t *u_off, size_t *v_off, size_t *c_off, size_t *totals) {
  if (!b) return EBIT_ERR_ARG;
  for (int k = 0; k < b->n; k++) {
    if (u_off) u_off[k] = b->uoff[k];
    if (v_off) v_off[k] = b->voff[k];
    if (c_off) c_off[k] = b->coff[k];
  }
  if (totals) {
    totals[0] = b->utot;
    totals[1] = b->vtot;
    totals[2] = b->ctot;
  }
  return EBIT_OK;
}

int ebit_batch_advect(ebit_batch *b, const double *u_packed, const double *v_packed, const double *dt_dev) {
  if (!b || !u_packed || !v_packed || !dt_dev) return EBIT_ERR_ARG;
  return engine_advect(&b->e, u_packed, v_packed, dt_dev, 0.0);
}

int ebit_batch_fraction_curvature(ebit_batch *b, double *C_packed, double *K_packed) {
  if (!b || !C_packed || !K_packed) return EBIT_ERR_ARG;
  const int rc = engine_frac(&b->e, 3, nullptr, C_packed, K_packed);
  b->e.fracEpoch = b->e.epoch;
  return rc;
}

int ebit_batch_ns_fields(ebit_batch *b, const double *C_packed, const double *K_packed, const ebit_fluid *fluid,
                         double *rho_packed, double *mu_packed, double *fx_packed, double *fy_packed) {
  if (!b) return EBIT_ERR_ARG;
  return engine_ns(&b->e, C_packed, K_packed, fluid, rho_packed, mu_packed, fx_packed, fy_packed);
}

int ebit_batch_get_state(ebit_batch *b, int k, uint8_t *node_color, uint8_t *cell_color, double *hoff, double *voff,
                         int64_t *step) {
  if (!b || k < 0 || k >= b->n) return EBIT_ERR_ARG;
  int rc = engine_get_state(&b->e, (uint32_t)k, node_color, cell_color, hoff, voff);
  if (rc) return rc;
  if (step) *step = b->e.stepNo;
  return EBIT_OK;
}

int ebit_batch_stats(ebit_batch *b, ebit_counters *out) {
  if (!b || !out) return EBIT_ERR_ARG;
  return engine_counters(&b->e, out);
}

int ebit_batch_get_schedule(const ebit_batch *b, ebit_schedule *out) {
  if (!b || !out) return EBIT_ERR_ARG;
  *out = b->e.used;
  return EBIT_OK;
}

int ebit_batch_set_schedule(ebit_batch *b, const ebit_schedule *s) {
  if (!b || !schedule_ok(s)) return EBIT_ERR_ARG;
  b->e.sched = *s;
  engine_launch_config(&b->e);
  return EBIT_OK;
}

int ebit_batch_sync(ebit_batch *b, int *status) {
  if (!b) return EBIT_ERR_ARG;
  return engine_errors(&b->e, status);
}

int ebit_batch_destroy(ebit_batch *b) {
  if (!b) return EBIT_ERR_ARG;
  delete b;
  return EBIT_OK;
}

}  // extern "C"

// K captured steps of a batch. The launches of a step depend on the engine's
// host schedule (which state copy is current, which list slot, which
// parabola-fit list parity, the step's sweep order); after an even number of
// steps all of them are back where they started, so the captured launches are
// valid for every replay that starts from the same schedule.
struct ebit_graph {
  ebit_batch *b = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int ksteps = 0;
  uint32_t cur = 0, slot = 0, ghfPar = 0, stepPar = 0;
};

namespace {
bool graph_schedule_matches(const ebit_graph *g) {
  const Engine &e = g->b->e;
  return e.cur == g->cur && (uint32_t)e.slot == g->slot && e.ghfPar == g->ghfPar && (e.stepNo & 1u) == g->stepPar &&
         !e.pendJobs;
}
void graph_free(ebit_graph *g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}
}  // namespace

extern "C" {

int ebit_batch_capture(ebit_batch *b, int ksteps, const double *u_packed, const double *v_packed,
                       const double *dts_dev, double *C_packed, double *K_packed, ebit_graph **out) {
  if (!out) return EBIT_ERR_ARG;
  *out = nullptr;
  if (!b || ksteps < 2 || (ksteps & 1) || !u_packed || !v_packed || !dts_dev || !C_packed || !K_packed)
    return EBIT_ERR_ARG;
  Engine *e = &b->e;
  if (e->pendJobs) return EBIT_ERR_STATE;
  ebit_graph *g = new (std::nothrow) ebit_graph();
  if (!g) return EBIT_ERR_NOMEM;
  g->b = b;
  g->ksteps = ksteps;
  g->cur = e->cur;
  g->slot = (uint32_t)e->slot;
  g->ghfPar = e->ghfPar;
  g->stepPar = e->stepNo & 1u;
  const uint32_t stepNo0 = e->stepNo;
  const int64_t epoch0 = e->epoch, fracEpoch0 = e->fracEpoch;
  // the null stream cannot be captured: record on a stream of our own
  hipStream_t cap = nullptr;
  hipError_t he = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (he != hipSuccess) {
    delete g;
    return device_failed(he, "hipStreamCreateWithFlags", __LINE__);
  }
  const hipStream_t saved = e->stream;
  e->stream = cap;
  int rc = EBIT_OK;
  he = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (he != hipSuccess) rc = device_failed(he, "hipStreamBeginCapture", __LINE__);
  if (!rc) {
    for (int k = 0; k < ksteps && !rc; k++) {
      rc = engine_advect(e, u_packed, v_packed, dts_dev + (size_t)k * (size_t)b->n, 0.0);
      if (!rc) rc = engine_frac(e, 3, nullptr, C_packed, K_packed);
    }
    hipGraph_t graph = nullptr;
    he = hipStreamEndCapture(cap, &graph);
    if (!rc && he != hipSuccess) rc = device_failed(he, "hipStreamEndCapture", __LINE__);
    g->graph = graph;
  }
  e->stream = saved;
  (void)hipStreamDestroy(cap);
  // capturing ran nothing: the engine's step counts stay where they were
  e->stepNo = stepNo0;
  e->epoch = epoch0;
  e->fracEpoch = fracEpoch0;
  if (!rc && !graph_schedule_matches(g)) rc = EBIT_ERR_STATE;
  if (!rc) {
    he = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (he != hipSuccess) rc = device_failed(he, "hipGraphInstantiate", __LINE__);
  }
  if (rc) {
    graph_free(g);
    return rc;
  }
  *out = g;
  return EBIT_OK;
}

int ebit_graph_launch(ebit_graph *g) {
  if (!g) return EBIT_ERR_ARG;
  if (!graph_schedule_matches(g)) return EBIT_ERR_STATE;
  Engine *e = &g->b->e;
  HIPCHK(hipGraphLaunch(g->exec, e->stream));
  e->stepNo += (uint32_t)g->ksteps;
  e->epoch += g->ksteps;
  e->fracEpoch = e->epoch;
  return EBIT_OK;
}

int ebit_graph_destroy(ebit_graph *g) {
  if (!g) return EBIT_ERR_ARG;
  graph_free(g);
  return EBIT_OK;
}

// ---------------------------------------------------------------------------
// pool (served form)
// ---------------------------------------------------------------------------
int ebit_pool_workspace_bytes(int max_grids, uint32_t max_tiles, size_t arena_bytes, size_t *bytes) {
  if (!bytes || max_grids < 1 || max_tiles < 1 || max_tiles > MAX_POOL_TILES) return EBIT_ERR_ARG;
  *bytes = pool_table_bytes(max_grids, max_tiles) + align256(arena_bytes);
  return EBIT_OK;
}

int ebit_pool_grid_bytes(const ebit_grid *grid, size_t *bytes, uint32_t *tiles) {
  if (!grid_ok(grid)) return EBIT_ERR_ARG;
  if (bytes) *bytes = pool_grid_bytes(*grid);
  if (tiles) *tiles = tiles_of(*grid);
  return EBIT_OK;
}

int ebit_pool_create(int max_grids, uint32_t max_tiles, void *ws_dev, size_t ws_bytes, void *hip_stream,
                     ebit_pool **out) {
  if (!out) return EBIT_ERR_ARG;
  *out = nullptr;
  if (max_grids < 1 || max_tiles < 1 || max_tiles > MAX_POOL_TILES || !ws_dev || ((uintptr_t)ws_dev & 255) != 0)
    return EBIT_ERR_ARG;
  const size_t tb = pool_table_bytes(max_grids, max_tiles);
  if (ws_bytes < tb) return EBIT_ERR_NOMEM;
  ebit_pool *p = new (std::nothrow) ebit_pool();
  if (!p) return EBIT_ERR_NOMEM;
  Engine *e = &p->e;
  e->ntiles = max_tiles;
  e->maxGrids = (uint32_t)max_grids;
  e->one = false;
  e->jobCap = (uint32_t)multi_job_cap(max_tiles, (size_t)max_tiles * JOBS_PER_TILE);
  e->stream = (hipStream_t)hip_stream;
  Carve c;
  carve_engine(e, (char *)ws_dev, c);
  p->dts = c.take<double>((char *)ws_dev, max_grids);
  p->arena = (char *)ws_dev + tb;
  p->arenaBytes = ws_bytes - tb;
  e->hinst.assign(max_grids, Inst());
  e->live.assign(max_grids, 0);
  e->grids.assign(max_grids, ebit_grid());
  p->pg.assign(max_grids, PoolGrid());
  p->hdts.assign(max_grids, 0.0);
  p->tileAlloc.init(max_tiles);
  p->arenaAlloc.init(p->arenaBytes);
  engine_launch_config(e);
  int rc = engine_reset(e);
  if (!rc) {
    const hipError_t err = hipMemsetAsync(p->dts, 0, max_grids * sizeof(double), e->stream);
    if (err != hipSuccess) rc = device_failed(err, "hipMemsetAsync(dts)", __LINE__);
  }
  if (!rc) rc = engine_compact(e, 0, 0, 0);
  if (!rc) {
    const hipError_t err = hipStreamSynchronize(e->stream);
    if (err != hipSuccess) rc = device_failed(err, "hipStreamSynchronize", __LINE__);
  }
  if (rc) {
    delete p;
    return rc;
  }
  *out = p;
  return EBIT_OK;
}

int ebit_pool_admit(ebit_pool *p, const ebit_grid *grid, const ebit_state *init, const double *u_host,
                    const double *v_host, double dt, int *slot_out) {
  if (!p || !slot_out || !grid_ok(grid) || !u_host || !v_host || !isfinite(dt) || !init || !init->node_color ||
      !init->cell_color || !init->hoff || !init->voff)
    return EBIT_ERR_ARG;
  Engine *e = &p->e;
  int k = -1;
  for (uint32_t s = 0; s < e->maxGrids; s++)
    if (!e->live[s]) {
      k = (int)s;
      break;
    }
  if (k < 0) return EBIT_ERR_NOMEM;
  const uint32_t nt = tiles_of(*grid);
  const size_t gb = pool_grid_bytes(*grid);
  size_t t0 = 0, a0 = 0;
  if (!p->tileAlloc.take(nt, 1, &t0)) return EBIT_ERR_NOMEM;
  if (!p->arenaAlloc.take(gb, 256, &a0)) {
    p->tileAlloc.give(t0, nt);
    return EBIT_ERR_NOMEM;
  }
  PoolGrid &g = p->pg[k];
  g.arenaOff = a0;
  g.arenaLen = gb;
  g.tile0 = t0;
  g.steps = 0;
  Inst &I = e->hinst[k];
  // the grid's step 0 runs at the engine's current step
  fill_inst(&I, *grid, (uint32_t)t0, e->stepNo & 1u, e->errs + k);
  Carve c;
  c.off = a0;
  carve_grid(&I, *grid, p->arena, c);
  const size_t nx = grid->nx, ny = grid->ny;
  const size_t nn = (nx + 1) * (ny + 1), nc = nx * ny, nh = nx * (ny + 1), nv = (nx + 1) * ny;
  double *u = c.take<double>(p->arena, ny * (nx + 1));
  double *v = c.take<double>(p->arena, (ny + 1) * nx);
  double *C = c.take<double>(p->arena, nx * ny);
  double *K = c.take<double>(p->arena, nx * ny);
  const double *base = (const double *)p->arena;
  I.uoff = (size_t)(u - base);
  I.voffv = (size_t)(v - base);
  I.coff = (size_t)(C - base);
  I.koff = (size_t)(K - base);
  e->grids[k] = *grid;
  p->hdts[k] = dt;
  // Everything is enqueued on the stream, nothing waits: the caller's arrays
  // go straight to the device (the node bytes into the grid's sweep scratch,
  // free until its first sweep), and kernels pack the colours, validate the
  // state (an invalid one latches EBIT_ERR_ARG in the grid's status), fill the
  // second state copy, set the descriptor, dt and error word, and mark the
  // grid's tiles.
  uint8_t *nodeBytes = (uint8_t *)I.dd;
  uint64_t dtBits;
  memcpy(&dtBits, &dt, sizeof dtBits);
  const hipStream_t st = e->stream;
  int rc = EBIT_OK;
  hipError_t err = hipMemcpyAsync(u, u_host, nv * sizeof(double), hipMemcpyHostToDevice, st);
  if (err == hipSuccess) err = hipMemcpyAsync(v, v_host, nh * sizeof(double), hipMemcpyHostToDevice, st);
  if (err == hipSuccess) err = hipMemcpyAsync(nodeBytes, init->node_color, nn, hipMemcpyHostToDevice, st);
  if (err == hipSuccess) err = hipMemcpyAsync(I.cen[0], init->cell_color, nc, hipMemcpyHostToDevice, st);
  if (err == hipSuccess) err = hipMemcpyAsync(I.hoff[0], init->hoff, nh * sizeof(double), hipMemcpyHostToDevice, st);
  if (err == hipSuccess) err = hipMemcpyAsync(I.voff[0], init->voff, nv * sizeof(double), hipMemcpyHostToDevice, st);
  if (err != hipSuccess) rc = device_failed(err, "admission upload", __LINE__);
  if (!rc) err = launch_fill_u32(e->errs + k, 0u, 1, st);
  if (!rc && err == hipSuccess) err = launch_fill_u32((uint32_t *)(p->dts + k), (uint32_t)dtBits, 1, st);
  if (!rc && err == hipSuccess) err = launch_fill_u32((uint32_t *)(p->dts + k) + 1, (uint32_t)(dtBits >> 32), 1, st);
  if (!rc && err == hipSuccess) err = launch_put_inst(I, e->dinst + k, st);
  if (!rc && err == hipSuccess) err = launch_import_state(I, nodeBytes, I.cen[0], I.hoff[0], I.voff[0], st);
  if (!rc && err == hipSuccess)
    err = launch_init_tiles(e->dinst, (uint32_t)k, (uint32_t)(I.ntx * I.nty), e->cur, e->tileInst, e->has,
                            e->nearPrev, st);
  if (!rc && err != hipSuccess) rc = device_failed(err, "admission kernels", __LINE__);
  if (rc) {
    p->tileAlloc.give(t0, nt);
    p->arenaAlloc.give(a0, gb);
    return rc;
  }
  e->live[k] = 1;
  p->dirty = true;
  *slot_out = k;
  return EBIT_OK;
}

int ebit_pool_status(ebit_pool *p, int32_t *status_dev) {
  if (!p || !status_dev) return EBIT_ERR_ARG;
  HIPCHK(launch_status_many(p->e.errs, status_dev, p->e.maxGrids, p->e.stream));
  return EBIT_OK;
}

int ebit_pool_retire(ebit_pool *p, int slot) {
  if (!p || slot < 0 || (uint32_t)slot >= p->e.maxGrids || !p->e.live[slot]) return EBIT_ERR_ARG;
  Engine *e = &p->e;
  PoolGrid &g = p->pg[slot];
  const uint32_t nt = tiles_of(e->grids[slot]);
  HIPCHK(launch_clear_tiles(e->tileInst, e->has, e->nearPrev, e->tinfo, (uint32_t)g.tile0, nt, e->stream));
  // the tile range and arena bytes are reused only by later admissions,
  // whose uploads follow on the same stream
  p->tileAlloc.give(g.tile0, nt);
  p->arenaAlloc.give(g.arenaOff, g.arenaLen);
  e->live[slot] = 0;
  p->dirty = true;
  return EBIT_OK;
}

int ebit_pool_step(ebit_pool *p) {
  if (!p) return EBIT_ERR_ARG;
  Engine *e = &p->e;
  bool any = false;
  for (uint32_t k = 0; k < e->maxGrids; k++) any = any || e->live[k];
  if (p->dirty) {
    int rc = engine_compact(e, 0, e->stepNo, 0);
    if (!rc) rc = engine_fill_table(e);
    if (rc) return rc;
    p->dirty = false;
  }
  if (!any) return EBIT_OK;
  const double *base = (const double *)p->arena;
  int rc = engine_advect(e, base, base, p->dts, 0.0);
  if (rc) return rc;
  rc = engine_frac(e, 3, nullptr, (double *)p->arena, (double *)p->arena);
  e->fracEpoch = e->epoch;
  for (uint32_t k = 0; k < e->maxGrids; k++)
    if (e->live[k]) p->pg[k].steps++;
  return rc;
}

int ebit_pool_read(ebit_pool *p, int slot, double *C_host, double *K_host, int64_t *steps, int *status) {
  if (!p || slot < 0 || (uint32_t)slot >= p->e.maxGrids || !p->e.live[slot]) return EBIT_ERR_ARG;
  Engine *e = &p->e;
  const Inst &I = e->hinst[slot];
  const size_t n = (size_t)I.nx * I.ny;
  const double *base = (const double *)p->arena;
  if (C_host) HIPCHK(hipMemcpyAsync(C_host, base + I.coff, n * sizeof(double), hipMemcpyDeviceToHost, e->stream));
  if (K_host) HIPCHK(hipMemcpyAsync(K_host, base + I.koff, n * sizeof(double), hipMemcpyDeviceToHost, e->stream));
  uint32_t bits = 0;
  HIPCHK(hipMemcpyAsync(&bits, e->errs + slot, sizeof bits, hipMemcpyDeviceToHost, e->stream));
  HIPCHK(hipStreamSynchronize(e->stream));
  if (steps) *steps = p->pg[slot].steps;
  if (status) *status = status_of(bits);
  return EBIT_OK;
}

int ebit_pool_get_state(ebit_pool *p, int slot, uint8_t *node_color, uint8_t *cell_color, double *hoff,
                        double *voff) {
  if (!p || slot < 0 || (uint32_t)slot >= p->e.maxGrids || !p->e.live[slot]) return EBIT_ERR_ARG;
  return engine_get_state(&p->e, (uint32_t)slot, node_color, cell_color, hoff, voff);
}

int ebit_pool_stats(ebit_pool *p, ebit_counters *out) {
  if (!p || !out) return EBIT_ERR_ARG;
  return engine_counters(&p->e, out);
}

int ebit_pool_get_schedule(const ebit_pool *p, ebit_schedule *out) {
  if (!p || !out) return EBIT_ERR_ARG;
  *out = p->e.used;
  return EBIT_OK;
}

int ebit_pool_set_schedule(ebit_pool *p, const ebit_schedule *s) {
  if (!p || !schedule_ok(s)) return EBIT_ERR_ARG;
  p->e.sched = *s;
  engine_launch_config(&p->e);
  return EBIT_OK;
}

int ebit_pool_destroy(ebit_pool *p) {
  if (!p) return EBIT_ERR_ARG;
  delete p;
  return EBIT_OK;
}

int ebit_step_static(const ebit_grid *grid, uint8_t *node_color_dev, uint8_t *cell_color_dev, double *hoff_dev,
                     double *voff_dev, const double *u_dev, const double *v_dev, double dt, int64_t step,
                     double *C_dev, double *K_dev, int32_t *status_dev, void *hip_stream) {
  if (!grid_ok(grid) || !node_color_dev || !cell_color_dev || !hoff_dev || !voff_dev || !u_dev || !v_dev || !C_dev ||
      !K_dev || !status_dev || !isfinite(dt) || step < 0)
    return EBIT_ERR_ARG;
  size_t need = 0;
  if (ebit_workspace_bytes(grid, &need) != EBIT_OK) return EBIT_ERR_ARG;
  if (need > (size_t)EBIT_STATIC_SCRATCH_BYTES) return EBIT_ERR_NOMEM;
  StaticSlot *S = nullptr;
  int rc = static_slot(&S);
  if (rc) return rc;
  Engine *e = &S->e;
  hipStream_t st = (hipStream_t)hip_stream;
  // one grid laid out over the scratch exactly as over a caller's workspace
  e->stream = st;
  e->ntiles = tiles_of(*grid);
  e->maxGrids = 1;
  e->one = true;
  e->jobCap = (uint32_t)jobs_of(*grid, true);
  Carve c;
  carve_engine(e, S->ptr, c);
  e->hinst.assign(1, Inst());
  e->live.assign(1, 1);
  e->grids.assign(grid, grid + 1);
  Inst &I = e->hinst[0];
  fill_inst(&I, *grid, 0, 0, e->errs);
  carve_grid(&I, *grid, S->ptr, c);
  e->cur = 0;
  e->stepNo = (uint32_t)(step & 1);
  e->slot = 1;
  e->ghfPar = 0;
  e->pendJobs = nullptr;
  // the last call's contents stay in the scratch: clear what starts at zero
  // with kernels (no memset nodes, for callers that capture the stream)
  static_assert(sizeof(unsigned long long) == 2 * sizeof(uint32_t), "counter words");
  HIPCHK(launch_fill_u32(e->counts, 0u, 2 * NSLOT, st));
  HIPCHK(launch_fill_u32((uint32_t *)e->ctr, 0u, 2 * (size_t)CTR_PARTS * CTR_STRIDE, st));
  HIPCHK(launch_fill_u32(e->errs, 0u, 1, st));
  HIPCHK(launch_fill_u32(e->ghfCnt, 0u, 2 * CNT_LINE, st));
  HIPCHK(launch_clear_tiles(e->tileInst, e->has, e->nearPrev, e->tinfo, 0, e->ntiles, st));
  HIPCHK(launch_put_inst(I, e->dinst, st));
  HIPCHK(launch_import_state(I, node_color_dev, cell_color_dev, hoff_dev, voff_dev, st));
  HIPCHK(launch_init_tiles(e->dinst, 0, e->ntiles, 0, e->tileInst, e->has, e->nearPrev, st));
  rc = engine_compact(e, 0, e->stepNo, 0);
  if (!rc) rc = engine_fill_table(e);
  if (!rc) rc = engine_advect(e, u_dev, v_dev, nullptr, dt);
  if (!rc) rc = engine_frac(e, 3, nullptr, C_dev, K_dev);
  if (rc) return rc;
  HIPCHK(launch_export_state(I, e->cur, node_color_dev, cell_color_dev, hoff_dev, voff_dev, st));
  HIPCHK(launch_status(e->errs, status_dev, st));
  return EBIT_OK;
}

const char *ebit_device_error(void) { return g_devErr; }

const char *ebit_strerror(int code) {
  switch (code) {
    case EBIT_OK: return "ok";
    case EBIT_ERR_ARG: return "invalid argument";
    case EBIT_ERR_STATE: return "call out of order (state advanced since ebit_fraction)";
    case EBIT_ERR_CFL: return "a marker moved more than half a cell in one sweep";
    case EBIT_ERR_DOMAIN: return "a marker would leave the grid";
    case EBIT_ERR_DEVICE: return "HIP runtime error";
    case EBIT_ERR_NOMEM: return "workspace too small, or no free slot, tiles or arena space";
    default: return "unknown error";
  }
}

}  // extern "C"

static_assert(sizeof(ebit_counters) == NCOUNTERS * sizeof(int64_t), "counter layout");
