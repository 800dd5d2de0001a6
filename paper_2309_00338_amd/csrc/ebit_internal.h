// Internal definitions shared by the gfx950 kernels and the host runtime.
//
// One engine advances any number of independent grids ("instances") with one
// launch per phase. Every grid is cut into 16x16-cell tiles and the tiles of
// all grids share one global index space: grid k owns tiles
// [tile0, tile0 + ntx*nty). Kernels map a global tile (or a fit job) to its
// grid through a per-tile instance table and read the grid's geometry and
// buffers from a device array of descriptors.
#ifndef EBIT_INTERNAL_H
#define EBIT_INTERNAL_H

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ebit {

constexpr int TS = 16;             // tile edge in cells
constexpr double TIE_EPS = 1e-12;  // near-degenerate decision threshold
constexpr uint32_t NO_INST = 0xffffffffu;  // tile owned by no grid

// counter slots (same order as the public ebit_counters fields)
enum {
  C_MARKERS = 0,
  C_ANNIHILATED,
  C_THREE_LANDERS,
  C_TIES,
  C_FIT_FALLBACK,
  C_FIT_REJECT,
  C_PARITY_FALLBACK,
  C_THREE_CROSSINGS,
  C_CV_SET,
  C_CV_CONFLICT,
  C_CV_UNRESOLVED,
  C_WALL_VIOLATION,
  C_INVARIANT_FAIL,
  C_HF_FAIL,
  C_INTERFACIAL,
  C_GHF_FIT,
  C_TILES_SWEPT,   // diagnostics of the tiled schedule (no oracle counterpart)
  C_TILES_EMPTY,
  C_TILES_NEAR,
  NCOUNTERS
};

// Counters live in CTR_PARTS partitions of CTR_STRIDE 64-bit slots (one
// 256-byte line each); a workgroup adds into partition blockIdx % CTR_PARTS,
// so that the adds of thousands of workgroups do not queue on one line. The
// host sums the partitions.
constexpr int CTR_PARTS = 64;
constexpr int CTR_STRIDE = 32;
static_assert(NCOUNTERS <= CTR_STRIDE, "counters fit one partition");

// ARG: an invalid imported state; CAP: a fit-job queue ran past its region
// (the per-tile bound on queued jobs rules it out; reported as a workspace
// too small)
enum : uint32_t { ERRBIT_CFL = 1u, ERRBIT_DOMAIN = 2u, ERRBIT_ARG = 4u, ERRBIT_CAP = 8u };
enum : uint32_t { INST_XY = 1u, INST_LINE = 2u };  // x then y every step; straight-line placement

// tile info bits written by the compaction, read by the fraction pass and
// the interface consumers: TI_NEAR a cut cell in the tile or on the side of
// its left / lower neighbour that it shares (the consumers' near set),
// TI_FRAC a cut cell in the tile (the fraction pass's near set; its other
// tiles are uniform)
enum : uint8_t { TI_NEAR = 1, TI_COLOUR = 2, TI_DEAD = 4, TI_FRAC = 8 };

// Node colours are a bit plane in blocks of 16 x 16 nodes: block (bx, by)
// holds nodes x in [16 bx, 16 bx + 16), y in [16 by, 16 by + 16) as 16 words
// of 16 bits, word y & 15, bit x & 15; blocks are row-major with nx / 16 + 1
// per block row (ny / 16 + 1 block rows), and bits of nodes outside the grid
// are 0. A tile and its halo then sit in 3 x 3 blocks, 3 runs of 96 bytes.
__host__ __device__ inline int cb_nbx(int nx) { return (nx >> 4) + 1; }
__host__ __device__ inline size_t cb_words(int nx, int ny) { return (size_t)cb_nbx(nx) * (size_t)cb_nbx(ny) * 16u; }
// word of row y in the block holding node (x, y); x and y inside the grid
__host__ __device__ inline size_t cb_word(int nx, int x, int y) {
  return ((size_t)(y >> 4) * (size_t)cb_nbx(nx) + (size_t)(x >> 4)) * 16u + (size_t)(y & 15);
}

// One grid: geometry, both state copies, per-sweep scratch, and where its
// velocities and output fields sit relative to the base pointers of a call.
struct Inst {
  int32_t nx, ny, ntx, nty;
  uint32_t tile0;       // first global tile
  uint32_t stepPar;     // parity of the engine step at which the grid's step 0 ran
  uint32_t flags;       // INST_XY
  uint32_t pad;
  double h;
  uint64_t uoff, voffv;  // element offsets of u and v in the call's velocity buffers
  uint64_t coff, koff;   // element offsets of C and kappa in the call's field buffers
  uint16_t *col[2];      // node colours as a bit plane (cb_word), both copies
  uint8_t *cen[2];       // centre colours, ny x nx: one array in both entries (the centre kernel
                         // updates it in place after the fits have read the old values)
  double *hoff[2];       // H-edge offsets, (ny+1) x nx
  double *voff[2];       // V-edge offsets, ny x (nx+1)
  double *sp;            // advected aligned offsets s' of the current sweep
  double *dd;            // per unaligned edge of the current sweep: old offset t, displacement d
  uint8_t *zr;           // per unaligned edge: centre-CV results of its fit
  uint32_t *err;         // error bits of this grid
};

// One grid as one sweep sees it: the copies it reads and writes, its
// velocity for the sweep direction and lambda = dt / h. Built on the host per
// launch when an engine holds one grid, on the device per tile otherwise.
struct SweepView {
  int32_t nx, ny, ntx, pad;
  uint32_t tile0;
  double lam;
  const uint16_t *col;        // state before the sweep
  const uint8_t *cen;
  const double *hoff, *voff;
  uint16_t *ncol;             // state after the sweep
  uint8_t *ncen;
  double *nhoff, *nvoff;
  const double *vel;          // u for the x sweep, v for the y sweep
  double *sp, *dd;
  uint8_t *zr;
  uint32_t *err;
  uint32_t line;              // straight-line placement of new unaligned markers
  uint32_t pad2;
};

__host__ __device__ inline SweepView sweep_view(const Inst &I, uint32_t cur, int dir, const double *u, const double *v,
                                                double lam) {
  SweepView w;
  w.nx = I.nx;
  w.ny = I.ny;
  w.ntx = I.ntx;
  w.pad = 0;
  w.tile0 = I.tile0;
  w.lam = lam;
  w.col = I.col[cur];
  w.cen = I.cen[cur];
  w.hoff = I.hoff[cur];
  w.voff = I.voff[cur];
  w.ncol = I.col[cur ^ 1u];
  w.ncen = I.cen[cur ^ 1u];
  w.nhoff = I.hoff[cur ^ 1u];
  w.nvoff = I.voff[cur ^ 1u];
  w.vel = dir == 0 ? u + I.uoff : v + I.voffv;
  w.sp = I.sp;
  w.dd = I.dd;
  w.zr = I.zr;
  w.err = I.err;
  w.line = (I.flags & INST_LINE) ? 1u : 0u;
  w.pad2 = 0;
  return w;
}

// Fit-job queues of one sweep direction. One grid whose sweep launch is a
// multiple of 8 workgroups splits its active list into 8 shares, one per XCD
// (workgroups are dispatched round-robin over the XCDs), and the workgroups of
// share q queue their jobs on queue q, in region q of the job list. A tile
// queues at most TS * TS jobs per sweep (one per interior line it owns and
// row), so a region of TS * TS * ceil(tiles / 8) entries holds any share's
// jobs. Several grids: workgroup b queues on queue b % 8, in regions whose
// bound follows from the sweep's chunking (the runtime's multi_job_span).
constexpr uint32_t NJQ = 8;

// counts per compaction slot: active tiles of x-sweeping grids, of
// y-sweeping grids, near tiles, tiles of the fraction pass, then the NJQ
// job-queue counts of the x sweep and those of the y sweep. Each count has a
// 256-byte line of its own: every compaction workgroup and every sweep
// workgroup's job flush adds to them with returning atomics, and atomics on
// one line are served one after the other.
constexpr int CNT_LINE = 64;
enum {
  CNT_ACT_X = 0 * CNT_LINE,
  CNT_ACT_Y = 1 * CNT_LINE,
  CNT_NEAR = 2 * CNT_LINE,
  CNT_FRAC = 3 * CNT_LINE,
  CNT_JOBS_X = 4 * CNT_LINE,
  CNT_JOBS_Y = (4 + (int)NJQ) * CNT_LINE
};
constexpr int NSLOT = (4 + 2 * (int)NJQ) * CNT_LINE;

// Arguments of the kernels of one sweep direction (sweep, fit, centre). The
// x direction reads the active list and the job list from the front, the y
// direction from the back.
struct SweepArgs {
  const Inst *inst;
  const uint32_t *tileInst;  // global tile -> grid
  const double *u, *v;       // velocity base pointers of the call
  const double *dts;         // per-grid dt (device) or null: dt for every grid
  double dt;
  uint32_t cur;              // copy holding the state before this sweep (0/1)
  uint32_t ntiles;           // global tiles (length of the active list)
  const uint2 *list;         // active tiles: (global tile, grid)
  const uint32_t *count;     // active tiles of this direction
  uint16_t *has;             // per tile: where its markers sit
  uint2 *jobs;               // fit jobs: (grid, unaligned-edge index)
  uint32_t *njobs;           // job counts of this direction's queues, CNT_LINE apart
  uint32_t jobQ;             // queues in use (1 or NJQ), the same for both directions
  uint32_t jobRegion;        // entries of each queue's region
  uint32_t jobTop;           // the y direction's entry e is list slot jobTop - 1 - e
  uint32_t minChunk;         // several grids: tiles per sweep workgroup, at least
  unsigned long long *ctr;
  // one grid: the centre rules of the step's first sweep, when they are left
  // to this (second) sweep's launch; its job count (null: none) and view
  const uint32_t *pendJobs;
  SweepView one;             // the grid's view when the engine holds one grid
  SweepView pend;
};

struct CompactArgs {
  const Inst *inst;
  const uint32_t *tileInst;
  uint32_t ntiles;
  uint32_t cur;              // copy holding the current state
  uint32_t stepNo;           // engine step and phase of the next sweep
  int phase;
  int afterSweep;            // 1 after a sweep, 0 after grids were added or removed
  int slot;
  const uint16_t *has;
  uint8_t *nearPrev, *tinfo;
  uint2 *actList, *nearList, *fracList;  // (global tile, grid)
  uint32_t *counts;
  Inst one;                  // the descriptor itself when the engine holds one grid
};

// A wavefront's cells (64 consecutive cells of a near tile) whose heights
// failed in both directions, left for the parabola fit of k_ghf: the tile,
// grid * 4 + the wavefront's index in the tile, and one bit per cell.
struct GhfEntry {
  uint32_t tile, gridWave;
  unsigned long long mask;
};

struct FracArgs {
  const Inst *inst;
  const uint32_t *tileInst;
  uint32_t ntiles;           // global tiles
  uint32_t cur;              // copy holding the current state
  const double *Cin;         // base pointers of the call (C read by curvature-only)
  double *Cout, *Kout;
  const uint8_t *tinfo;
  const uint2 *list;         // near tiles: (global tile, grid)
  const uint32_t *count;
  int nearBlocks;            // workgroups [0, nearBlocks) work the near tiles
  unsigned long long *ctr;
  GhfEntry *ghf;             // cells left for the parabola fit (4 entries per tile at most)
  uint32_t *ghfCount;        // entries of this launch (zero on entry)
  uint32_t *ghfClear;        // the other launch parity's count, zeroed by this launch
  // the uniform cells' fill, pitch_chunks workgroups per grid: entry k of
  // fillTab is (first fill workgroup, grid) of the k-th grid with cells
  // (ascending first workgroups); fillGrids entries (one grid: no table)
  const uint2 *fillTab;
  uint32_t fillGrids;
  Inst one;                  // the descriptor itself when the engine holds one grid
};

// Consumers of C and kappa on the same grid: density, viscosity, surface
// tension face forces (one launch for every grid of the engine).
struct NsArgs {
  const Inst *inst;
  const uint32_t *tileInst;
  uint32_t ntiles;
  uint32_t cur;
  const double *C, *K;        // cell fields, at each grid's coff / koff
  double *rho, *mu;           // cell outputs at coff (either may be null)
  double *fx, *fy;            // face outputs at uoff / voffv (either may be null)
  double rho1, rho2, mu1, mu2, sigma;
  const uint8_t *tinfo;
  const uint2 *list;          // near tiles
  const uint32_t *count;
  int nearBlocks;
  Inst one;                   // the descriptor itself when the engine holds one grid
};

__host__ __device__ inline int sweep_dir(const Inst &I, uint32_t stepNo, int phase) {
  if (I.flags & INST_XY) return phase;
  return (int)((stepNo + I.stepPar) & 1u) ^ phase;
}

// launchers (defined with the kernels); resident_blocks(which): resident
// workgroups per CU of 0 the sweep, 1 the fit, 2 the centre kernel, 3/4/5 the
// fraction modes 1/2/3 (the y-direction kernels use the same resources; the
// fraction workgroups are half the size of the others)
int resident_blocks(int which);
// one: the engine holds a single grid (index 0)
hipError_t launch_sweep(int dir, bool one, const SweepArgs &a, int grid, hipStream_t s);
// c: the compaction that follows the sweep, run by extra workgroups of the
// fit launch (null: fits only)
hipError_t launch_fit(int dir, bool one, const SweepArgs &a, int grid, const CompactArgs *c, hipStream_t s);
hipError_t launch_centre(int dir, bool one, const SweepArgs &a, int grid, hipStream_t s);
hipError_t launch_init_tiles(const Inst *inst, uint32_t kinst, uint32_t ntiles, uint32_t cur, uint32_t *tileInst,
                             uint16_t *has, uint8_t *nearPrev, hipStream_t s);
hipError_t launch_clear_tiles(uint32_t *tileInst, uint16_t *has, uint8_t *nearPrev, uint8_t *tinfo, uint32_t tile0,
                              uint32_t ntiles, hipStream_t s);
hipError_t launch_compact(bool one, const CompactArgs &a, hipStream_t s);
hipError_t launch_frac_curv(int mode, bool one, const FracArgs &a, int grid, hipStream_t s);
// elements of C (and kappa) one per-tile fill workgroup writes (16 tiles)
constexpr uint32_t FILL_CHUNK = 4096;
// fill workgroups of one grid's uniform cells: 16 virtual rows of pitch nx
// rounded up to 16 by 256 columns each (the pitched fill of k_frac_curv)
inline uint32_t pitch_chunks(int nx, int ny) {
  const size_t P = ((size_t)nx + 15) & ~(size_t)15;
  const size_t vrows = ((size_t)nx * (size_t)ny + P - 1) / P;
  return (uint32_t)(((vrows + 15) / 16) * ((P + 255) / 256));
}
int ns_fill_blocks(uint32_t ntiles);
// workgroups of the linear uniform-part passes of k_ns for one nx x ny grid
int ns_linear_blocks(int nx, int ny);
// the parabola fit of the cells a curvature launch left (same FracArgs)
hipError_t launch_ghf(bool one, const FracArgs &a, int grid, hipStream_t s);
hipError_t launch_ns(bool one, const NsArgs &a, int grid, hipStream_t s);
// small kernels of the entry point that keeps no state between calls: a fill
// (clears tables without memset nodes), the descriptor upload, the state
// import into both copies / export of copy cur in the public layout, and the
// latched error as a public status code
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_put_inst(const Inst &I, Inst *dst, hipStream_t s);
hipError_t launch_import_state(const Inst &I, const uint8_t *node, const uint8_t *cell, const double *hoff,
                               const double *voff, hipStream_t s);
hipError_t launch_export_state(const Inst &I, uint32_t cur, uint8_t *node, uint8_t *cell, double *hoff, double *voff,
                               hipStream_t s);
hipError_t launch_status(const uint32_t *err, int32_t *status, hipStream_t s);
hipError_t launch_status_many(const uint32_t *err, int32_t *status, uint32_t n, hipStream_t s);

}  // namespace ebit

#endif
