// Launchers of the reverse-mode (adjoint) kernels of one timestep; internal to the library.
// Planes are dense [ny][nx]; the state planes phi^n, c^n are read from the field pool (row pitch `pitch`).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.h"

namespace lbm {

// Forward intermediates of step n, as exported by the stage-export kernels (doubles, dense planes).
struct AdjFwd {
  const double *mu, *X, *Fx, *Fy, *n, *ux, *uy, *ph, *ch, *M, *Xh;
};

// Every plane an adjoint step reads or writes (T = arithmetic type, dense planes of nx * ny).
template <typename T>
struct AdjPlanes {
  const T *phi, *c;  // state at n (pitched rows)
  int pitch;
  const T *fb1, *pb1, *cb1;  // adjoint of f (9 planes), phi, c at n + 1
  T *fb, *pb, *cb;           // adjoint at n (outputs)
  // intermediate adjoints: of phi^{n+1/2}, c^{n+1/2} (K12 -> K3) and of the force (K3 -> K45)
  T *phb, *chb, *Fxb, *Fyb;
};

struct AdjModel {
  int nx, ny;
  int walls;  // LBM_WALLS_NONE or LBM_WALLS_Y
  double a, b, B0, B1, D, Gamma, gamma, omega, coef, ramp;  // ramp = min(n, t*): dA(n)/dA0
  double yper;
};

// One backward step: the adjoint at n + 1 -> the adjoint at n.  Each block adds its partial sum of
// sum_r cb1(r) * ramp * count_n(r) over its tile (the step's contribution to d/dA0) to part[tile]; part holds
// adj_blocks(nx, ny) running totals, zeroed before the first step.
template <typename T>
hipError_t launch_adjoint_step(hipStream_t s, const AdjModel& m, const AdjFwd& f, const AdjPlanes<T>& p,
                               const DropDev* drops_n, int ndrop, double* part);

// Seed of the loss x_CM^N of droplet `drop`: pass 0 writes per-block partial sums of phi over the droplet's
// nodes (phi^N >= 0, nearest centre of step N - 1) into part; pass 1 writes pb = (dx - delta) / sw on those
// nodes and 0 elsewhere, and clears fb, cb.
template <typename T>
hipError_t launch_adjoint_seed(hipStream_t s, int pass, const AdjModel& m, const T* phi, int pitch,
                               const DropDev* drops_prev, int ndrop, int drop, double delta, double sw, T* fb,
                               T* pb, T* cb, double* part);

// Blocks of the adjoint kernels: one per tile of ADJ_TILE_X x ADJ_TILE_Y nodes (at least one per 256 nodes,
// which the seed kernel's one-dimensional blocks need).
constexpr int ADJ_TILE_X = 64, ADJ_TILE_Y = 4;
inline int adj_blocks(int nx, int ny) {
  return ((nx + ADJ_TILE_X - 1) / ADJ_TILE_X) * ((ny + ADJ_TILE_Y - 1) / ADJ_TILE_Y);
}

}  // namespace lbm
