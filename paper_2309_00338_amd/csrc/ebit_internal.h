// Internal definitions shared by the gfx950 kernels and the host runtime.
#ifndef EBIT_INTERNAL_H
#define EBIT_INTERNAL_H

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ebit {

constexpr int TS = 16;             // tile edge in cells
constexpr double TIE_EPS = 1e-12;  // near-degenerate decision threshold

// counter slots (same order as the public ebit_stats fields)
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
  C_TILES_SWEPT,   // diagnostics of the tiled schedule (no oracle counterpart)
  C_TILES_EMPTY,
  C_TILES_NEAR,
  NCOUNTERS
};

enum : uint32_t { ERRBIT_CFL = 1u, ERRBIT_DOMAIN = 2u };

struct SweepParams {
  int nx, ny, ntx, nty;
  double lam;
  const uint8_t *col;
  const uint8_t *cen;
  const double *hoff;
  const double *voff;
  const double *vel;
  uint8_t *ncol;
  uint8_t *ncen;
  double *nhoff;
  double *nvoff;
  const uint32_t *list;
  const uint32_t *count;
  uint16_t *has;  // per tile: where its markers sit (any / near a side / near a corner)
  double *sp;     // advected aligned offsets s' of present edges (aligned-edge layout)
  double *dd;     // displacements of present unaligned markers (unaligned-edge layout)
  uint32_t *jobs; // new unaligned markers for the fit kernel (unaligned-edge index)
  uint32_t *njobs;
  uint32_t *err;
  unsigned long long *ctr;
};

struct FitParams {
  int nx, ny;
  const uint8_t *col;   // old node colours
  const uint8_t *cen;   // old centre colours
  const uint8_t *ncol;  // new node colours
  const double *sp;
  const double *dd;
  const double *hoff;   // old offsets
  const double *voff;
  double *nhoff;        // new offsets
  double *nvoff;
  uint8_t *ncen;        // new centre colours
  uint8_t *zr;          // per unaligned edge: centre-CV results of its fit
  const uint32_t *jobs;
  const uint32_t *njobs;
  unsigned long long *ctr;
};

struct FracParams {
  int nx, ny, ntx, nty;
  double h;
  const uint8_t *col;
  const uint8_t *cen;
  const double *hoff;
  const double *voff;
  const double *Cin;
  double *Cout;
  double *Kout;
  const uint8_t *tinfo;  // per tile: bit 0 near, bit 1 uniform colour
  int vec;               // rows may use 16-byte stores (even nx, aligned C/K)
  int tileBlocks;        // workgroups [0, tileBlocks) claim near tiles before rows
  uint32_t *work;        // this launch's claim counters: [tiles, rows]
  uint32_t *workNext;    // the next launch's, cleared by this one
  const uint32_t *list;
  const uint32_t *count;
  unsigned long long *ctr;
};

// launchers (defined with the kernels)
// resident workgroups per CU of: 0/1 the x/y sweep, 2/3/4 fraction modes 1/2/3,
// 5/6 the x/y fit, 7 the centre kernel
int resident_blocks(int which);
hipError_t launch_sweep(int dir, const SweepParams &p, int grid, hipStream_t s);
hipError_t launch_fit(int dir, const FitParams &p, int grid, hipStream_t s);
hipError_t launch_centre(int dir, const FitParams &p, int grid, hipStream_t s);
hipError_t launch_init_has(const uint8_t *col, int nx, int ny, int ntx, int nty, uint16_t *has, uint8_t *nearPrev,
                           hipStream_t s);
hipError_t launch_compact(const uint16_t *has, uint8_t *nearPrev, uint8_t *tinfo, const uint8_t *col, int nx, int ntx,
                          int nty, uint32_t *actList, uint32_t *nearList, uint32_t *counts, int slot, hipStream_t s);
hipError_t launch_frac_curv(int mode, const FracParams &p, int grid, hipStream_t s);

}  // namespace ebit

#endif
