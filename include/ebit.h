/*
 * ebit.h: C-ABI of the MI355X (gfx950) EBIT interface step.
 *
 * The step is the kinematic part of the Edge-Based Interface Tracking method
 * of Pan, Long, Chirco, Scardovelli, Popinet and Zaleski (arXiv 2309.00338) on
 * a uniform 2D grid with four closed walls, in FP64:
 *   - markers on grid edges advected by explicit Euler with a bilinear
 *     velocity, one direction at a time (Sec. 2.1, Eq. Eq_marker_dis);
 *   - unaligned markers re-intersected with the grid lines by the circle fit
 *     (Sec. 2.2);
 *   - corner and centre Color Vertices updated (Sec. 2.3);
 *   - markers removed or merged by the corner colours (Sec. 2.4);
 *   - volume fraction from markers and Color Vertices, and height-function
 *     curvature of that fraction (Sec. 2.5).
 *
 * Index space. Node (i,j) sits at the integer point (i,j), 0 <= i <= nx,
 * 0 <= j <= ny; cell (i,j) is [i,i+1] x [j,j+1]. H(i,j) is the edge from node
 * (i,j) to (i+1,j); its marker sits at (i + hoff, j). V(i,j) joins (i,j) and
 * (i,j+1); its marker sits at (i, j + voff). A marker exists on an edge iff
 * the colours of its two end nodes differ (Sec. 2.4); offsets elsewhere are
 * ignored. Every array is row-major with x fastest:
 *   node_color (ny+1) x (nx+1) uint8 in {0,1}   (corner Color Vertex)
 *   cell_color  ny    x  nx    uint8 in {0,1}   (centre Color Vertex)
 *   hoff       (ny+1) x  nx    double in [0,1]
 *   voff        ny    x (nx+1) double in [0,1]
 *   u           ny    x (nx+1) double  x-face velocity at (i, j+1/2)
 *   v          (ny+1) x  nx    double  y-face velocity at (i+1/2, j)
 *   C, K        ny    x  nx    double  volume fraction, curvature
 * Colour 1 is the reference phase. Velocities and K are in physical units
 * (cell size h); offsets are in cell widths.
 *
 * Asynchrony and errors. Every call that takes a handle enqueues its work on
 * the handle's HIP stream and returns at once; nothing aborts and no C++
 * exception crosses this boundary. Argument errors are returned immediately.
 * Errors detected on the device (EBIT_ERR_CFL: some marker would move more
 * than half a cell in one sweep; EBIT_ERR_DOMAIN: a marker would leave the
 * grid; EBIT_ERR_NOMEM: a fit-job queue outgrew its part of the workspace,
 * which the sizing of ebit_workspace_bytes rules out) are latched and returned by the next ebit_sync, ebit_get_state or
 * ebit_stats call; the state is then undefined until ebit_set_state.
 *
 * Ownership. The caller owns every device buffer (workspace, u, v, C, K) and
 * keeps the workspace alive until ebit_destroy. The handle owns only a small
 * host struct. One host thread per handle at a time; handles on different
 * streams are independent.
 */
#ifndef EBIT_H
#define EBIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  EBIT_OK = 0,
  EBIT_ERR_ARG = 1,    /* bad argument (null, size, non-finite, out of range) */
  EBIT_ERR_STATE = 2,  /* call out of order (e.g. curvature of a stale C) */
  EBIT_ERR_CFL = 3,    /* a marker displacement exceeded half a cell */
  EBIT_ERR_DOMAIN = 4, /* a marker would have left the grid */
  EBIT_ERR_DEVICE = 5, /* a HIP runtime call failed */
  EBIT_ERR_NOMEM = 6   /* workspace too small / host allocation failed */
};

/* Sweep order (Sec. 2.1 splits each step into an x and a y sweep; the paper
 * does not fix their order). ALTERNATE: step n runs x then y when n is even,
 * y then x when n is odd. XY: always x then y.
 * FIT_LINE: place each new unaligned marker where the straight segment between
 * the two advected points that straddle the grid line crosses it, instead of
 * by the circle fit of Sec. 2.2 (the method's first version, the EBIT-SL rows
 * of Tables 1, 3, 4 and 5). */
enum { EBIT_SWEEP_ALTERNATE = 0u, EBIT_SWEEP_XY = 1u, EBIT_FIT_LINE = 2u };

typedef struct {
  int32_t nx, ny;  /* cells along x and y, each in [4, 65535] */
  double h;        /* physical cell size, > 0 */
  uint32_t flags;  /* EBIT_SWEEP_* | EBIT_FIT_LINE */
} ebit_grid;

/* Host-side state (Sec. 2.1-2.3): corner colours, centre colours and marker
 * offsets, laid out as in the header comment. Offsets are read only where the
 * end colours differ and must lie in [0,1] there. */
typedef struct {
  const uint8_t *node_color;
  const uint8_t *cell_color;
  const double *hoff;
  const double *voff;
} ebit_state;

/* Device counters, accumulated since create/set_state/ebit_stats_reset. */
typedef struct {
  int64_t markers;         /* markers at the start of each sweep, summed */
  int64_t annihilated;     /* aligned markers removed by pairing (Sec. 2.4) */
  int64_t three_landers;   /* edges that received three aligned markers */
  int64_t ties;            /* decisions within 1e-12 of degenerate */
  int64_t fit_fallback;    /* unaligned markers placed by the straight line */
  int64_t fit_reject;      /* circle roots discarded for leaving their edge */
  int64_t parity_fallback; /* colours and crossings disagree (mid-edge) */
  int64_t three_crossings; /* new unaligned edges crossed three times */
  int64_t cv_set;          /* centre CVs set by the aligned-marker rule */
  int64_t cv_conflict;     /* left and right rules disagreed */
  int64_t cv_unresolved;   /* 4-marker cells the rule did not reach */
  int64_t wall_violation;  /* wall-normal motion of a wall marker */
  int64_t invariant_fail;  /* lander parity differs from the colours */
  int64_t hf_fail;         /* interfacial cells with no valid height */
  int64_t interfacial;     /* cells with >= 2 markers seen by curvature */
  int64_t ghf_fit;         /* of the hf_fail cells, those given kappa by the marker parabola */
  /* schedule diagnostics (GPU tiles of 16x16 cells) */
  int64_t tiles_swept;     /* tiles swept with markers in reach */
  int64_t tiles_empty;     /* tiles swept only to carry their state over */
  int64_t tiles_near;      /* tiles given polygon/height work */
} ebit_counters;

typedef struct ebit_handle ebit_handle;

/* Launch schedule of an engine (a handle, batch or pool): how its persistent
 * kernels spread over the GPU. It decides only which workgroup handles which
 * tile or marker, never a result: states, C and kappa are bit-identical under
 * every schedule. Values are clamped to what the device can hold resident
 * (per compute unit); 0 in any field means the device's default for it.
 *   sweep_per_cu      sweep workgroups per CU (default: all resident, 16)
 *   fit_per_cu        fit workgroups per CU (default: all resident)
 *   sweep_min_chunk   several grids: tiles per sweep workgroup, at least (8)
 *   frac_near_per_cu  fraction/curvature pass: workgroups per CU that take the
 *                     tiles with cut cells, the others filling the uniform
 *                     cells beside them (5.5 of 8)
 *   ns_near_per_cu    the same split for ebit_ns_fields (6 of 8) */
typedef struct {
  uint32_t sweep_per_cu, fit_per_cu, sweep_min_chunk;
  double frac_near_per_cu, ns_near_per_cu;
} ebit_schedule;

/* The schedule in force (every field resolved, no zeros). */
int ebit_get_schedule(const ebit_handle *h, ebit_schedule *out);
/* Replace it (takes effect at the next call; EBIT_ERR_ARG for a negative or
 * non-finite field). */
int ebit_set_schedule(ebit_handle *h, const ebit_schedule *s);

/* Bytes of device workspace a grid needs (both state buffers, tile tables,
 * lists, counters, sweep scratch). Returns EBIT_ERR_ARG for an invalid grid,
 * or one whose fit-job list would pass 32-bit indices (above about
 * 46000 x 46000 cells). */
int ebit_workspace_bytes(const ebit_grid *grid, size_t *bytes);

/* Validate the host state `init`, upload it into the caller's device
 * workspace `ws_dev` (ws_bytes >= ebit_workspace_bytes) and return a handle
 * bound to `hip_stream` (a hipStream_t; NULL = default stream). Synchronous
 * with respect to the host buffers. EBIT_ERR_ARG for a bad grid, a colour not
 * in {0,1} or an offset outside [0,1] (or non-finite) on a marker edge;
 * EBIT_ERR_NOMEM if the workspace is too small. */
int ebit_create(const ebit_grid *grid, const ebit_state *init, void *ws_dev, size_t ws_bytes, void *hip_stream,
                ebit_handle **out);

/* One time step of Eq. (Eq_marker_dis) with face velocities u_dev, v_dev
 * (device, layout above) taken at t_n, as two 1D sweeps (Sec. 2.1): aligned
 * markers move along their line and flip the nodes they cross (Sec. 2.3);
 * unaligned markers are re-placed on the grid lines by the circle fit
 * (Sec. 2.2); centre colours follow rules (1)-(5) of Sec. 2.3; markers that
 * meet on one edge annihilate (Sec. 2.4). dt may be negative (a time factor
 * of the field may be folded into dt). Asynchronous; CFL/DOMAIN latch. */
int ebit_advect(ebit_handle *h, const double *u_dev, const double *v_dev, double dt);

/* Volume fraction of colour 1 in every cell (Sec. 2.5: the straight segment
 * between the cell's markers, the centre CV choosing the pairing of a
 * four-marker cell). Writes all ny*nx entries of C_dev (device). */
int ebit_fraction(ebit_handle *h, double *C_dev);

/* Height-function curvature of the fraction C_dev produced by ebit_fraction
 * on the current state (Sec. 2.5), on a 7x3 stencil oriented by the corner
 * colours. Writes all ny*nx entries of K_dev: 0 in cells with fewer than two
 * markers, else kappa (> 0 for a convex colour-1 region). Where no height is
 * valid, kappa of the least-squares parabola through the markers on the edges
 * of the 5x5 cells around the cell, in the frame of the node-colour gradient
 * (the generalised height function Sec. 2.5 refers to); NaN where that fit
 * has fewer than 3 points, a zero gradient or a near-singular system.
 * EBIT_ERR_STATE if the state advanced since ebit_fraction. */
int ebit_curvature(ebit_handle *h, const double *C_dev, double *K_dev);

/* ebit_fraction followed by ebit_curvature in one pass (same results). */
int ebit_fraction_curvature(ebit_handle *h, double *C_dev, double *K_dev);

/* Two-fluid properties and surface tension of the one-fluid Navier-Stokes
 * equations (Sec. 2.5): Eq. (physical) with the Heaviside function
 * approximated by C, and the surface-tension term sigma kappa n delta_S as a
 * continuum force on the MAC faces, sigma * kappa_f * (C_right - C_left) / h,
 * where kappa_f is the curvature of the face's two cells that carry one (two
 * or more markers and a finite kappa): their mean, the one that does, or 0.
 * Wall faces carry no force. */
typedef struct {
  double rho1, rho2;  /* density of colour 1 (the reference phase) and colour 0 */
  double mu1, mu2;    /* viscosity of colour 1 and colour 0 */
  double sigma;       /* surface tension coefficient */
} ebit_fluid;

/* rho_dev, mu_dev: ny x nx per cell; fx_dev: ny x (nx+1) on the x-faces (the
 * layout of u); fy_dev: (ny+1) x nx on the y-faces (the layout of v); any
 * output may be NULL. C_dev and K_dev must be the fraction and curvature of
 * the current state (EBIT_ERR_STATE if the state advanced since the last
 * ebit_fraction or ebit_fraction_curvature). Fully written. */
int ebit_ns_fields(ebit_handle *h, const double *C_dev, const double *K_dev, const ebit_fluid *fluid, double *rho_dev,
                   double *mu_dev, double *fx_dev, double *fy_dev);

/* Copy the current state to host buffers (any may be NULL) and the step
 * counter; waits on the stream and returns a latched device error. */
int ebit_get_state(ebit_handle *h, uint8_t *node_color, uint8_t *cell_color, double *hoff, double *voff,
                   int64_t *step);

/* Replace the state (validated as in ebit_create), clear the latched error
 * and the counters. Synchronous. */
int ebit_set_state(ebit_handle *h, const ebit_state *state, int64_t step);

/* Read the counters (waits on the stream; returns a latched device error). */
int ebit_stats(ebit_handle *h, ebit_counters *out);
int ebit_stats_reset(ebit_handle *h);

/* Wait for the handle's stream; return the latched device error, if any. */
int ebit_sync(ebit_handle *h);

/* Free the host struct; the workspace stays the caller's. */
int ebit_destroy(ebit_handle *h);

const char *ebit_strerror(int code);

/* After EBIT_ERR_DEVICE: the HIP error name and the runtime call that failed,
 * as a NUL-terminated string owned by the library (per calling thread); "" if
 * no HIP call has failed on this thread. */
const char *ebit_device_error(void);

/* ===========================================================================
 * Batched form: a fixed set of independent grids advanced together, one
 * kernel launch per phase for all of them (the tiles of all grids share one
 * work list). Each grid behaves exactly as it would under its own handle; all
 * grids take their steps together, so step n of every grid uses the same
 * sweep order (EBIT_SWEEP_ALTERNATE counts the batch's steps).
 *
 * Packed buffers. Grid k's u, v, C and K sit in shared device buffers at the
 * element offsets ebit_batch_layout reports (each start 256-byte aligned,
 * per-grid layout as in the header comment); totals[0..2] are the element
 * counts of the u, v and C/K buffers. dt is per grid, in device memory.
 * =========================================================================== */
typedef struct ebit_batch ebit_batch;

/* Workspace bytes for n grids (grids[0..n-1] as in ebit_workspace_bytes). */
int ebit_batch_workspace_bytes(int n, const ebit_grid *grids, size_t *bytes);

/* Validate and upload n initial states (inits[k] for grids[k]); synchronous
 * with respect to the host buffers. Errors as ebit_create. */
int ebit_batch_create(int n, const ebit_grid *grids, const ebit_state *inits, void *ws_dev, size_t ws_bytes,
                      void *hip_stream, ebit_batch **out);

/* Element offsets of each grid's u, v and C/K in the packed buffers (any
 * pointer may be NULL; arrays of n entries) and the buffer totals (3). */
int ebit_batch_layout(const ebit_batch *b, size_t *u_off, size_t *v_off, size_t *c_off, size_t *totals);

/* One step of every grid (as ebit_advect), grid k with dt_dev[k]. */
int ebit_batch_advect(ebit_batch *b, const double *u_packed, const double *v_packed, const double *dt_dev);

/* Fraction and curvature of every grid (as ebit_fraction_curvature). */
int ebit_batch_fraction_curvature(ebit_batch *b, double *C_packed, double *K_packed);

/* As ebit_ns_fields for every grid: rho and mu in the C/K layout, fx in the
 * u layout and fy in the v layout of ebit_batch_layout. */
int ebit_batch_ns_fields(ebit_batch *b, const double *C_packed, const double *K_packed, const ebit_fluid *fluid,
                         double *rho_packed, double *mu_packed, double *fx_packed, double *fy_packed);

/* Grid k's current state to host buffers (any may be NULL); waits. */
int ebit_batch_get_state(ebit_batch *b, int k, uint8_t *node_color, uint8_t *cell_color, double *hoff, double *voff,
                         int64_t *step);

/* Counters summed over the grids; waits. */
int ebit_batch_stats(ebit_batch *b, ebit_counters *out);

/* Waits; status[k] (n entries, may be NULL) is grid k's latched device error;
 * returns the first nonzero one. A grid in error leaves the others valid. */
int ebit_batch_sync(ebit_batch *b, int *status);
int ebit_batch_destroy(ebit_batch *b);

/* The batch's schedule (as ebit_get_schedule / ebit_set_schedule). A graph
 * captured before a change keeps the schedule it was captured with. */
int ebit_batch_get_schedule(const ebit_batch *b, ebit_schedule *out);
int ebit_batch_set_schedule(ebit_batch *b, const ebit_schedule *s);

/* K steps of the batch recorded once as a HIP graph of kernel launches and
 * replayed with one call: step k (0 <= k < ksteps) is ebit_batch_advect with
 * dt_dev = dts_dev + k*n (dts_dev: device, ksteps x n doubles, row k = the
 * grids' dt of step k), then ebit_batch_fraction_curvature into C_packed,
 * K_packed. The buffers must stay valid while the graph exists; their
 * contents are read at each replay. ksteps must be even (a step flips the
 * engine's schedule between two alternating layouts; an even count returns it
 * to where it started). Capturing runs nothing. EBIT_ERR_ARG for an odd or
 * small ksteps or a null buffer. The graph holds no memset or copy nodes. */
typedef struct ebit_graph ebit_graph;
int ebit_batch_capture(ebit_batch *b, int ksteps, const double *u_packed, const double *v_packed,
                       const double *dts_dev, double *C_packed, double *K_packed, ebit_graph **out);

/* Replay the K steps on the batch's stream (asynchronous). EBIT_ERR_STATE if
 * the batch is not at a point where the capture's schedule holds (an odd
 * number of other steps or fraction calls since the capture). */
int ebit_graph_launch(ebit_graph *g);
/* Destroy every graph of a batch before the batch itself. */
int ebit_graph_destroy(ebit_graph *g);

/* ===========================================================================
 * Served form: a pool that admits grids between steps, advances every admitted
 * grid by one step per ebit_pool_step (advection, then fraction and curvature
 * into the grid's own C and K), and retires them on request. Each grid keeps
 * its own steady face velocities and dt (uploaded at admission) and its own
 * step count (its sweep order starts from step 0 at admission). The workspace
 * holds tables for max_grids grids and max_tiles 16x16-cell tiles, then an
 * arena for the per-grid arrays; ebit_pool_grid_bytes gives one grid's arena
 * bytes and tiles, for admission control.
 * =========================================================================== */
typedef struct ebit_pool ebit_pool;

int ebit_pool_workspace_bytes(int max_grids, uint32_t max_tiles, size_t arena_bytes, size_t *bytes);
int ebit_pool_grid_bytes(const ebit_grid *grid, size_t *bytes, uint32_t *tiles);
int ebit_pool_create(int max_grids, uint32_t max_tiles, void *ws_dev, size_t ws_bytes, void *hip_stream,
                     ebit_pool **out);

/* Admit a grid: its state, u_host and v_host (host, layout above) and dt.
 * Returns its slot at once; EBIT_ERR_NOMEM when no slot, tile range or arena
 * space is free (nothing changes; admit again after a retire). Asynchronous:
 * the uploads are enqueued on the pool's stream and read the host arrays
 * later, so those must stay unchanged until the stream has passed this point
 * (the next ebit_pool_read or a synchronisation of the stream); from pinned
 * host memory the copies overlap the GPU's work, from pageable memory the HIP
 * runtime may copy before returning. The state is validated on the device: a
 * colour above 1 or an offset outside [0,1] on an edge whose end colours
 * differ latches EBIT_ERR_ARG in the grid's status (ebit_pool_read,
 * ebit_pool_status). */
int ebit_pool_admit(ebit_pool *p, const ebit_grid *grid, const ebit_state *init, const double *u_host,
                    const double *v_host, double dt, int *slot_out);

/* One step of every admitted grid, then its C and K. Asynchronous. */
int ebit_pool_step(ebit_pool *p);

/* Waits; copies the grid's latest C and K (either may be NULL) to the host,
 * with the steps it has taken and its latched device error. */
int ebit_pool_read(ebit_pool *p, int slot, double *C_host, double *K_host, int64_t *steps, int *status);
int ebit_pool_get_state(ebit_pool *p, int slot, uint8_t *node_color, uint8_t *cell_color, double *hoff,
                        double *voff);

/* Every slot's latched status (EBIT_OK, EBIT_ERR_CFL, EBIT_ERR_DOMAIN,
 * EBIT_ERR_ARG; EBIT_OK for empty slots) into status_dev (device, max_grids
 * int32), asynchronously: a caller polling many requests copies it back once
 * per step instead of waiting on the stream per request. */
int ebit_pool_status(ebit_pool *p, int32_t *status_dev);

/* Release the slot, its tiles and its arena space (asynchronous). */
int ebit_pool_retire(ebit_pool *p, int slot);
int ebit_pool_stats(ebit_pool *p, ebit_counters *out);
int ebit_pool_get_schedule(const ebit_pool *p, ebit_schedule *out);
int ebit_pool_set_schedule(ebit_pool *p, const ebit_schedule *s);
int ebit_pool_destroy(ebit_pool *p);

/* ===========================================================================
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * One whole step (as ebit_create, ebit_advect, ebit_fraction_curvature) of a
 * grid whose state lives in the caller's device buffers, in the layout of the
 * header comment: node_color_dev, cell_color_dev, hoff_dev and voff_dev are
 * read, then overwritten with the state after the step; u_dev, v_dev as in
 * ebit_advect; C_dev and K_dev are fully written as by
 * ebit_fraction_curvature. `step` is the grid's step number (its parity picks
 * the sweep order, EBIT_SWEEP_ALTERNATE). Every intermediate (engine tables,
 * both state copies, sweep scratch) lives in one array of the library's own
 * per GPU, EBIT_STATIC_SCRATCH_BYTES long, held from the library's first use
 * on that GPU until the process ends; nothing is allocated, neither by this
 * call nor by the library on its behalf. Grids whose ebit_workspace_bytes
 * exceed EBIT_STATIC_SCRATCH_BYTES (about 1056 x 1056 cells) are rejected
 * with EBIT_ERR_NOMEM before any device work.
 *
 * Asynchronous on hip_stream (NULL = default stream): the call returns after
 * enqueueing, and *status_dev (device, one int32) receives EBIT_OK,
 * EBIT_ERR_CFL, EBIT_ERR_DOMAIN, or EBIT_ERR_ARG for an invalid state (a
 * colour byte above 1, an offset outside [0,1] on an edge whose end colours
 * differ); after an error the outputs are undefined. The return value reports
 * argument errors and failed HIP calls (EBIT_ERR_DEVICE). Tables are cleared
 * by kernels, not memset nodes, so the call may be captured into a graph.
 *
 * Every call on a GPU shares that GPU's array and the library's host record
 * of it, and each call starts by clearing and reloading both: calls that
 * overlap on one GPU (from several host threads, or on several streams whose
 * work may run at once) race; serialise them.
 * =========================================================================== */
#define EBIT_STATIC_SCRATCH_BYTES (80u << 20)

int ebit_step_static(const ebit_grid *grid, uint8_t *node_color_dev, uint8_t *cell_color_dev, double *hoff_dev,
                     double *voff_dev, const double *u_dev, const double *v_dev, double dt, int64_t step,
                     double *C_dev, double *K_dev, int32_t *status_dev, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* EBIT_H */
