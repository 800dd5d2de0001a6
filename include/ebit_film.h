/*
 * ebit_film.h: C-ABI of the two-markers-per-edge interface step on MI355X
 * (gfx950), FP64.
 *
 * With one marker per edge (Sec. 2.4) two markers that land on one edge
 * annihilate, so a film of fluid thinner than a cell disappears the moment its
 * two walls share an edge. The end of Sec. 2.4 and the kinematic extension of
 * Sec. 4 name the remedy: allow two markers per edge. The paper gives no
 * algorithm for it; this library implements one reading of it:
 *   - an edge holds 0, 1 or 2 markers, an odd number iff the colours of its
 *     end nodes differ; a pair (equal end colours) is a film crossing the edge;
 *   - markers are advected as in Sec. 2.1 (each marker of a pair on its own),
 *     and a node flips once per marker that passes it;
 *   - the markers landing on an aligned edge, ordered by position, keep the
 *     middle one of an odd number and the middle two of an even number when
 *     they are at least the rupture gap delta apart (the film is thicker than
 *     delta), none otherwise; a new unaligned edge keeps its crossings by the
 *     same rule on the heights where the advected segments cross the line,
 *     each placed by the circle fit of Sec. 2.2;
 *   - the markers of a cell, in counter-clockwise order round its boundary,
 *     pair so that every segment cuts off a boundary arc whose colour differs
 *     from the centre colour (two markers: one segment; four: the pairs round
 *     the corners that differ from the centre, as in Sec. 2.3);
 *   - centre colours follow rules (1)-(5) of Sec. 2.3, the cell's left-edge
 *     markers first (lowest kept crossing first), then its right edge's;
 *   - the volume fraction is the cell minus (centre colour 1) or the sum of
 *     (centre colour 0) the regions the segments cut off.
 * With delta = +inf no film forms and the step is the one-marker method of
 * ebit.h (its ALTERNATE sweep order and circle fit).
 *
 * Index space and units are those of ebit.h. Marker arrays hold two offsets
 * per edge, ascending, of which the first `count` are meaningful:
 *   node_color (ny+1) x (nx+1) uint8 in {0,1}
 *   cell_color  ny    x  nx    uint8 in {0,1}
 *   hcount     (ny+1) x  nx    uint8 in {0,1,2}   markers on H(i,j)
 *   hoff       (ny+1) x  nx x 2 double in [0,1]   their offsets along x
 *   vcount      ny    x (nx+1) uint8 in {0,1,2}   markers on V(i,j)
 *   voff        ny    x (nx+1) x 2 double in [0,1]
 *   u, v, C as in ebit.h.
 *
 * Asynchrony, errors and ownership follow ebit.h: calls enqueue on the
 * handle's stream and return; EBIT_ERR_CFL / EBIT_ERR_DOMAIN found on the
 * device are latched and returned by the next ebit_film_sync, _get_state or
 * _stats (the state is then undefined until ebit_film_set_state). The caller
 * owns the workspace and keeps it alive until ebit_film_destroy.
 */
#ifndef EBIT_FILM_H
#define EBIT_FILM_H

#include "ebit.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Host-side film state (layout above). */
typedef struct {
  const uint8_t *node_color;
  const uint8_t *cell_color;
  const uint8_t *hcount;
  const double *hoff;
  const uint8_t *vcount;
  const double *voff;
} ebit_film_state;

/* Host buffers a state is read back into (same layout; offsets past an edge's
 * count are written as 0). */
typedef struct {
  uint8_t *node_color;
  uint8_t *cell_color;
  uint8_t *hcount;
  double *hoff;
  uint8_t *vcount;
  double *voff;
} ebit_film_out;

/* Device counters, accumulated since create or set_state. */
typedef struct {
  int64_t markers;               /* markers at the start of each sweep, summed */
  int64_t annihilated;           /* aligned landers not kept (Sec. 2.4 pairing, film rupture) */
  int64_t annihilated_unaligned; /* crossings of new unaligned edges not kept */
  int64_t three_crossings;       /* new unaligned edges crossed three times */
  int64_t parity_fail;           /* unaligned edges whose crossing count disagrees with the colours */
} ebit_film_counters;

typedef struct ebit_film ebit_film;

/* Device workspace for a grid (two state copies, sweep scratch, counters).
 * EBIT_ERR_ARG for an invalid grid (ebit.h's limits; flags must be 0). */
int ebit_film_workspace_bytes(const ebit_grid *grid, size_t *bytes);

/* A handle over the caller's workspace, loaded with `init` (validated on the
 * host: colours in {0,1}, counts of the right parity and at most 2, offsets
 * finite, in [0,1] and ascending). `delta` is the rupture gap in cell widths
 * (>= 0, +inf forbids films); `step` the step count the sweep order starts
 * from (x first on even steps). `stream` is a hipStream_t (NULL: default). */
int ebit_film_create(const ebit_grid *grid, double delta, const ebit_film_state *init, int64_t step, void *ws_dev,
                     size_t ws_bytes, void *stream, ebit_film **out);

/* One step (Sec. 2.1): an x and a y sweep in the alternating order, each
 * advecting, flipping, landing, re-intersecting and updating centre colours as
 * described above. u, v are device arrays (ebit.h layout), dt finite. */
int ebit_film_advect(ebit_film *f, const double *u_dev, const double *v_dev, double dt);

/* Volume fraction of every cell into the device array C (ny x nx). */
int ebit_film_fraction(ebit_film *f, double *C_dev);

/* Synchronise and copy the state to host buffers; returns a latched error. */
int ebit_film_get_state(ebit_film *f, const ebit_film_out *out);

/* Replace the state (validated as in create) and clear errors and counters. */
int ebit_film_set_state(ebit_film *f, const ebit_film_state *s, int64_t step);

/* Synchronise and read the counters; returns a latched error. */
int ebit_film_stats(ebit_film *f, ebit_film_counters *out);

/* Synchronise; returns a latched error. */
int ebit_film_sync(ebit_film *f);

/* Free the handle (not the workspace). */
int ebit_film_destroy(ebit_film *f);

#ifdef __cplusplus
}
#endif

#endif /* EBIT_FILM_H */
