// EBIT interface step: host runtime behind the C-ABI in include/ebit.h.
//
// The handle carves the caller's device workspace into both copies of the
// state (colours and FP64 offsets), the per-tile tables and lists, the error
// word and the counters, and enqueues the kernels on the caller's stream.
// Nothing here allocates device memory.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "ebit.h"
#include "ebit_internal.h"

using namespace ebit;

struct ebit_handle {
  ebit_grid g;
  hipStream_t stream;
  int ntx, nty, ntiles;
  int sweepBlocks[2];  // persistent grids: x and y sweeps
  int fracBlocks[3];   // fraction modes 1, 2, 3
  int fracTileBlocks[3];  // of which the fraction pass gives to near tiles
  // state copies [0], [1]
  uint8_t *col[2], *cen[2];
  double *hoff[2], *voff[2];
  int cur;  // copy holding the current state
  // tile tables
  uint16_t *has;
  uint8_t *nearPrev, *tinfo;
  uint32_t *actList, *nearList, *counts;  // counts: [act, near, jobs] x 2 slots
  double *sp, *dd;     // advected offsets / displacements of the current sweep
  uint8_t *zr;         // per unaligned edge: centre-CV results of its fit
  uint32_t *jobs;      // new unaligned markers of the current sweep
  int fitBlocks[2], centreBlocks;
  int slot;                               // counts slot written by the last compaction
  uint32_t *fracWork;  // claim counters of the fraction pass: two launches x [tiles, rows]
  int fracParity;
  uint32_t *err;
  unsigned long long *ctr;
  int64_t step;
  int64_t epoch, fracEpoch;
};

namespace {

struct Carve {
  size_t off = 0;
  template <class T>
  T *take(char *base, size_t n) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? (T *)(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

bool grid_ok(const ebit_grid *g) {
  return g && g->nx >= 4 && g->ny >= 4 && g->nx <= 65535 && g->ny <= 65535 && isfinite(g->h) && g->h > 0.0 &&
         (g->flags & ~1u) == 0;
}

void carve(ebit_handle *h, char *base, size_t *total) {
  const size_t nx = h->g.nx, ny = h->g.ny;
  const size_t nn = (nx + 1) * (ny + 1), nc = nx * ny, nh = nx * (ny + 1), nv = (nx + 1) * ny;
  Carve c;
  for (int k = 0; k < 2; k++) {
    h->col[k] = c.take<uint8_t>(base, nn);
    h->cen[k] = c.take<uint8_t>(base, nc);
    h->hoff[k] = c.take<double>(base, nh);
    h->voff[k] = c.take<double>(base, nv);
  }
  h->has = c.take<uint16_t>(base, h->ntiles);
  h->nearPrev = c.take<uint8_t>(base, h->ntiles);
  h->tinfo = c.take<uint8_t>(base, h->ntiles);
  h->actList = c.take<uint32_t>(base, h->ntiles);
  h->nearList = c.take<uint32_t>(base, h->ntiles);
  h->counts = c.take<uint32_t>(base, 6);
  h->sp = c.take<double>(base, (nx + 1) * (ny + 1));
  h->dd = c.take<double>(base, (nx + 1) * (ny + 1));
  h->zr = c.take<uint8_t>(base, (nx + 1) * (ny + 1));
  h->jobs = c.take<uint32_t>(base, (nx + 1) * (ny + 1));
  h->fracWork = c.take<uint32_t>(base, 4);
  h->err = c.take<uint32_t>(base, 1);
  h->ctr = c.take<unsigned long long>(base, NCOUNTERS);
  *total = (c.off + 255) & ~(size_t)255;
}

void tiles_of(const ebit_grid *g, int *ntx, int *nty) {
  *ntx = (g->nx + TS - 1) / TS;
  *nty = (g->ny + TS - 1) / TS;
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

#define HIPCHK(x)                          \
  do {                                     \
    if ((x) != hipSuccess) return EBIT_ERR_DEVICE; \
  } while (0)

// compaction of the current state: marker flags -> active and near lists
int compact(ebit_handle *h) {
  h->slot ^= 1;
  HIPCHK(launch_compact(h->has, h->nearPrev, h->tinfo, h->col[h->cur], h->g.nx, h->ntx, h->nty, h->actList,
                        h->nearList, h->counts, h->slot, h->stream));
  return EBIT_OK;
}

int upload(ebit_handle *h, const ebit_state *s) {
  const size_t nx = h->g.nx, ny = h->g.ny;
  const size_t nn = (nx + 1) * (ny + 1), nc = nx * ny, nh = nx * (ny + 1), nv = (nx + 1) * ny;
  for (int k = 0; k < 2; k++) {
    HIPCHK(hipMemcpyAsync(h->col[k], s->node_color, nn, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->cen[k], s->cell_color, nc, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->hoff[k], s->hoff, nh * sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->voff[k], s->voff, nv * sizeof(double), hipMemcpyHostToDevice, h->stream));
  }
  h->cur = 0;
  HIPCHK(hipMemsetAsync(h->counts, 0, 6 * sizeof(uint32_t), h->stream));
  HIPCHK(hipMemsetAsync(h->fracWork, 0, 4 * sizeof(uint32_t), h->stream));
  h->fracParity = 0;
  HIPCHK(hipMemsetAsync(h->err, 0, sizeof(uint32_t), h->stream));
  HIPCHK(hipMemsetAsync(h->ctr, 0, NCOUNTERS * sizeof(unsigned long long), h->stream));
  h->slot = 1;
  HIPCHK(launch_init_has(h->col[0], h->g.nx, h->g.ny, h->ntx, h->nty, h->has, h->nearPrev, h->stream));
  int rc = compact(h);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(h->stream));
  h->epoch++;
  return EBIT_OK;
}

int read_err(ebit_handle *h) {
  uint32_t e = 0;
  HIPCHK(hipMemcpyAsync(&e, h->err, sizeof e, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (e & ERRBIT_CFL) return EBIT_ERR_CFL;
  if (e & ERRBIT_DOMAIN) return EBIT_ERR_DOMAIN;
  return EBIT_OK;
}

int sweep(ebit_handle *h, int dir, const double *u, const double *v, double dt) {
  SweepParams p;
  const int nxt = h->cur ^ 1;
  p.nx = h->g.nx;
  p.ny = h->g.ny;
  p.ntx = h->ntx;
  p.nty = h->nty;
  p.lam = dt / h->g.h;
  p.col = h->col[h->cur];
  p.cen = h->cen[h->cur];
  p.hoff = h->hoff[h->cur];
  p.voff = h->voff[h->cur];
  p.vel = dir == 0 ? u : v;
  p.ncol = h->col[nxt];
  p.ncen = h->cen[nxt];
  p.nhoff = h->hoff[nxt];
  p.nvoff = h->voff[nxt];
  p.list = h->actList;
  p.count = h->counts + 3 * h->slot;
  p.has = h->has;
  p.err = h->err;
  p.ctr = h->ctr;
  p.sp = h->sp;
  p.dd = h->dd;
  p.jobs = h->jobs;
  p.njobs = h->counts + 3 * h->slot + 2;
  HIPCHK(launch_sweep(dir, p, h->sweepBlocks[dir], h->stream));
  FitParams f;
  f.nx = h->g.nx;
  f.ny = h->g.ny;
  f.col = h->col[h->cur];
  f.cen = h->cen[h->cur];
  f.ncol = h->col[nxt];
  f.sp = h->sp;
  f.dd = h->dd;
  f.hoff = h->hoff[h->cur];
  f.voff = h->voff[h->cur];
  f.nhoff = h->hoff[nxt];
  f.nvoff = h->voff[nxt];
  f.ncen = h->cen[nxt];
  f.zr = h->zr;
  f.jobs = h->jobs;
  f.njobs = p.njobs;
  f.ctr = h->ctr;
  HIPCHK(launch_fit(dir, f, h->fitBlocks[dir], h->stream));
  HIPCHK(launch_centre(dir, f, h->centreBlocks, h->stream));
  h->cur = nxt;
  return compact(h);
}

FracParams frac_params(ebit_handle *h, int mode, const double *Cin, double *Cout, double *Kout) {
  FracParams p;
  p.nx = h->g.nx;
  p.ny = h->g.ny;
  p.ntx = h->ntx;
  p.nty = h->nty;
  p.h = h->g.h;
  p.col = h->col[h->cur];
  p.cen = h->cen[h->cur];
  p.hoff = h->hoff[h->cur];
  p.voff = h->voff[h->cur];
  p.Cin = Cin;
  p.Cout = Cout;
  p.Kout = Kout;
  p.tinfo = h->tinfo;
  p.list = h->nearList;
  p.count = h->counts + 3 * h->slot + 1;
  p.ctr = h->ctr;
  p.tileBlocks = h->fracTileBlocks[mode - 1];
  p.work = h->fracWork + 2 * h->fracParity;
  p.workNext = h->fracWork + 2 * (h->fracParity ^ 1);
  h->fracParity ^= 1;
  p.vec = (h->g.nx % 2 == 0) && ((uintptr_t)Cout % 16 == 0) && ((uintptr_t)Kout % 16 == 0);
  return p;
}

}  // namespace

extern "C" {

int ebit_workspace_bytes(const ebit_grid *grid, size_t *bytes) {
  if (!grid_ok(grid) || !bytes) return EBIT_ERR_ARG;
  ebit_handle tmp;
  memset(&tmp, 0, sizeof tmp);
  tmp.g = *grid;
  tiles_of(grid, &tmp.ntx, &tmp.nty);
  tmp.ntiles = tmp.ntx * tmp.nty;
  carve(&tmp, nullptr, bytes);
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
  ebit_handle *h = (ebit_handle *)calloc(1, sizeof(ebit_handle));
  if (!h) return EBIT_ERR_NOMEM;
  h->g = *grid;
  h->stream = (hipStream_t)hip_stream;
  tiles_of(grid, &h->ntx, &h->nty);
  h->ntiles = h->ntx * h->nty;
  size_t tot;
  carve(h, (char *)ws_dev, &tot);
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
  for (int d = 0; d < 2; d++) {
    h->sweepBlocks[d] = cus * resident_blocks(d);
    h->fitBlocks[d] = cus * resident_blocks(5 + d);
  }
  h->centreBlocks = cus * resident_blocks(7);
  {
    double share = 0.5;
    const char *e = getenv("EBIT_FRAC_TILE_SHARE");
    if (e) share = atof(e);
    if (!(share > 0.0)) share = 0.5;
    if (share > 0.95) share = 0.95;
    for (int m = 0; m < 3; m++) {
      h->fracBlocks[m] = cus * resident_blocks(2 + m);
      h->fracTileBlocks[m] = (int)(h->fracBlocks[m] * share);
      if (h->fracTileBlocks[m] < 1) h->fracTileBlocks[m] = 1;
    }
  }
  rc = upload(h, init);
  if (rc) {
    free(h);
    return rc;
  }
  *out = h;
  return EBIT_OK;
}

int ebit_advect(ebit_handle *h, const double *u_dev, const double *v_dev, double dt) {
  if (!h || !u_dev || !v_dev || !isfinite(dt)) return EBIT_ERR_ARG;
  const int first = ((h->g.flags & EBIT_SWEEP_XY) || (h->step % 2) == 0) ? 0 : 1;
  int rc = sweep(h, first, u_dev, v_dev, dt);
  if (!rc) rc = sweep(h, 1 - first, u_dev, v_dev, dt);
  h->step++;
  h->epoch++;
  return rc;
}

int ebit_fraction(ebit_handle *h, double *C_dev) {
  if (!h || !C_dev) return EBIT_ERR_ARG;
  FracParams p = frac_params(h, 1, nullptr, C_dev, nullptr);
  HIPCHK(launch_frac_curv(1, p, h->fracBlocks[0], h->stream));
  h->fracEpoch = h->epoch;
  return EBIT_OK;
}

int ebit_curvature(ebit_handle *h, const double *C_dev, double *K_dev) {
  if (!h || !C_dev || !K_dev) return EBIT_ERR_ARG;
  if (h->fracEpoch != h->epoch) return EBIT_ERR_STATE;
  FracParams p = frac_params(h, 2, C_dev, nullptr, K_dev);
  HIPCHK(launch_frac_curv(2, p, h->fracBlocks[1], h->stream));
  return EBIT_OK;
}

int ebit_fraction_curvature(ebit_handle *h, double *C_dev, double *K_dev) {
  if (!h || !C_dev || !K_dev) return EBIT_ERR_ARG;
  FracParams p = frac_params(h, 3, nullptr, C_dev, K_dev);
  HIPCHK(launch_frac_curv(3, p, h->fracBlocks[2], h->stream));
  h->fracEpoch = h->epoch;
  return EBIT_OK;
}

int ebit_get_state(ebit_handle *h, uint8_t *node_color, uint8_t *cell_color, double *hoff, double *voff,
                   int64_t *step) {
  if (!h) return EBIT_ERR_ARG;
  const size_t nx = h->g.nx, ny = h->g.ny;
  if (node_color) HIPCHK(hipMemcpyAsync(node_color, h->col[h->cur], (nx + 1) * (ny + 1), hipMemcpyDeviceToHost, h->stream));
  if (cell_color) HIPCHK(hipMemcpyAsync(cell_color, h->cen[h->cur], nx * ny, hipMemcpyDeviceToHost, h->stream));
  if (hoff) HIPCHK(hipMemcpyAsync(hoff, h->hoff[h->cur], nx * (ny + 1) * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  if (voff) HIPCHK(hipMemcpyAsync(voff, h->voff[h->cur], (nx + 1) * ny * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  if (step) *step = h->step;
  return read_err(h);
}

int ebit_set_state(ebit_handle *h, const ebit_state *state, int64_t step) {
  if (!h || step < 0) return EBIT_ERR_ARG;
  int rc = validate_state(&h->g, state);
  if (rc) return rc;
  h->step = step;
  return upload(h, state);
}

int ebit_stats(ebit_handle *h, ebit_counters *out) {
  if (!h || !out) return EBIT_ERR_ARG;
  unsigned long long v[NCOUNTERS];
  HIPCHK(hipMemcpyAsync(v, h->ctr, sizeof v, hipMemcpyDeviceToHost, h->stream));
  int rc = read_err(h);
  int64_t *dst = (int64_t *)out;
  for (int k = 0; k < NCOUNTERS; k++) dst[k] = (int64_t)v[k];
  return rc;
}

int ebit_stats_reset(ebit_handle *h) {
  if (!h) return EBIT_ERR_ARG;
  HIPCHK(hipMemsetAsync(h->ctr, 0, NCOUNTERS * sizeof(unsigned long long), h->stream));
  return EBIT_OK;
}

int ebit_sync(ebit_handle *h) {
  if (!h) return EBIT_ERR_ARG;
  return read_err(h);
}

int ebit_destroy(ebit_handle *h) {
  if (!h) return EBIT_ERR_ARG;
  free(h);
  return EBIT_OK;
}

const char *ebit_strerror(int code) {
  switch (code) {
    case EBIT_OK: return "ok";
    case EBIT_ERR_ARG: return "invalid argument";
    case EBIT_ERR_STATE: return "call out of order (state advanced since ebit_fraction)";
    case EBIT_ERR_CFL: return "a marker moved more than half a cell in one sweep";
    case EBIT_ERR_DOMAIN: return "a marker would leave the grid";
    case EBIT_ERR_DEVICE: return "HIP runtime error";
    case EBIT_ERR_NOMEM: return "workspace too small or host allocation failed";
    default: return "unknown error";
  }
}

}  // extern "C"

static_assert(sizeof(ebit_counters) == NCOUNTERS * sizeof(int64_t), "counter layout");
