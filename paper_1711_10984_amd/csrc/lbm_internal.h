// Internal declarations shared by the kernels and the host side of the library.
// Not part of the public ABI (include/lbm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm.h"

namespace lbm {

// Tile of interior nodes processed by one workgroup of the split timestep kernels.
constexpr int TILE_X = 64;
constexpr int TILE_Y = 8;
constexpr int NTHREADS = 256;
// Sweeping kernels: a workgroup owns a strip of strip_w columns (at most FUSED_TX, so that the strip and
// its 5-column halo on each side fit the 64 lanes of a wavefront) and seg_rows rows and sweeps it row by
// row; the fused kernel runs FUSED_R rows per sweep iteration, one wavefront each.
constexpr int FUSED_LANES = 64;
constexpr int FUSED_TX = FUSED_LANES - 10;
constexpr int FUSED_R = 4;
constexpr int STRIP_W_MIN = LBM_STRIP_W_MIN;
static_assert(LBM_STRIP_W_MAX == FUSED_TX, "widest strip");
// Strip widths tried by the autotuner (LBM_TUNE_NWIDTHS of them).  Only the widest: narrower strips
// (48 columns, whose FP64 row segments are whole 128-byte lines) measured slower on the 2048^2 workloads
// in every precision.
constexpr int32_t TUNE_WIDTHS[] = {54};
static_assert(sizeof(TUNE_WIDTHS) / sizeof(TUNE_WIDTHS[0]) == LBM_TUNE_NWIDTHS, "tune width list length");
// Rows per strip segment: chosen at run time among these (the autotuner picks one per context).
constexpr int SEG_ROWS_MIN = LBM_SEG_ROWS_MIN;
constexpr int SEG_ROWS_MAX = LBM_SEG_ROWS_MAX;
constexpr int SEG_ROWS_DEFAULT = 64;
// Heights tried by the autotuner (LBM_TUNE_NROWS of them).
constexpr int32_t TUNE_ROWS[] = {16, 20, 24, 26, 28, 32, 36, 40, 44, 48, 54, 64, 80, 96, 128, 256};
static_assert(sizeof(TUNE_ROWS) / sizeof(TUNE_ROWS[0]) == LBM_TUNE_NROWS, "tune list length");
// Tilings: 0 = split-kernel tiles, 1 = fused-kernel strips.
constexpr int TILING_SPLIT = 0;
constexpr int TILING_FUSED = 1;
constexpr int MAXDROP = 256;   // droplets per instance
constexpr int MASK_WORDS = MAXDROP / 64;  // one presence bit per droplet and tile

// Per-instance description read by every kernel (device copy in the workspace).
struct InstDev {
  int32_t nx, ny, pitch, ndrop;
  int32_t tiles_x[2], tiles_y[2], tile_base[2];  // per tiling: counts and first natural index
  int32_t drop_base, seg_rows;  // seg_rows: rows per sweeping-kernel strip segment
  int64_t pstride;     // elements between consecutive planes of the pool (ny * pitch)
  int64_t off_f[2];    // element offsets of the two population buffers [9][ny][pitch], planes pstride apart
  int64_t off_phi[2];  // the two phi buffers [ny][pitch]
  int64_t off_c[2];    // the two c buffers
  int64_t off_ux, off_uy, off_n;  // velocity planes written by the LB kernel; density (diagnostics)
  int64_t part_base[2];  // per tiling: offset (doubles) of the centre-of-mass partials [tiles][ndrop][3]
  int32_t advection, walls;  // walls: LBM_WALLS_NONE or LBM_WALLS_Y
  int32_t strip_w, reserved;  // strip_w: columns owned per sweeping-kernel strip
  double yper;                // period of y in droplet distances and centres: ny, or infinite with walls
  // model parameters, derived on the host in double precision
  double a, b, B0, B1, halfB1, D, Gamma, gamma, c0, omega, coef, A0, t_star;
  double wn[3];  // rest populations w_i n0 of the three weight classes (centre, axis, diagonal)
  double n0;     // rest density
};

// Droplet table entry on the device.
struct DropDev {
  double x, y, R, Rs, ex, ey;
  int32_t active, inst;
};

// One entry of the tile list (natural order: instance, tile row, tile column).
struct TileDev {
  int32_t inst, x0, y0, t;  // t: natural tile index (partials are stored by it)
};

// Launch helpers, instantiated in lbm_kernels_f64.hip, lbm_kernels_f32.hip and lbm_kernels_f16.hip.
// T is the arithmetic (and field) type, P the population storage type (T itself, or _Float16 deviations
// from w_i n0 with T = float).  `buf` is the typed base pointer of the field pool, `parity` selects the
// current buffers.  Modes: 0 step, 1 step + stage export, 2 diagnostics only.  An export names its instance
// in dbg_inst: inst exports all LBM_NSTAGE planes, -2 - inst (export_planes()) only the first ADJ_EXPORT_PLANES
// (mu .. X^{n+1/2}), which the reverse mode reads.
constexpr int ADJ_EXPORT_PLANES = 11;
inline int export_planes(int inst, bool all) { return all ? inst : -2 - inst; }
template <typename T, typename P>
hipError_t launch_lb(hipStream_t s, int mode, int parity, int ntiles_launch, const TileDev* tiles,
                     const InstDev* inst, T* buf, double* dbg, int dbg_inst);
template <typename T>
hipError_t launch_fd(hipStream_t s, int mode, int parity, int ntiles_launch, const TileDev* tiles,
                     const InstDev* inst, T* buf, const DropDev* drops, double* part, uint64_t* mask,
                     const int64_t* step, double* dbg, int dbg_inst);
template <typename T>
hipError_t launch_cm_partials(hipStream_t s, int parity, int ntiles_launch, const TileDev* tiles,
                              const InstDev* inst, T* buf, const DropDev* drops, double* part,
                              uint64_t* mask);
hipError_t launch_reduce(hipStream_t s, int tiling, int ndrop_total, const InstDev* inst, DropDev* drops,
                         const double* part, const uint64_t* mask, int64_t* step, int increment);
// Fused timestep (one launch per step over the strip list); dbg != nullptr also exports the stage planes of
// instance dbg_inst and steps only that instance (its next state in the inactive half, and its centre-of-mass
// partials).
template <typename T, typename P>
hipError_t launch_step(hipStream_t s, int parity, int nseg_launch, const TileDev* segs, const InstDev* inst,
                       T* buf, const DropDev* drops, double* part, uint64_t* mask, const int64_t* step,
                       double* dbg, int dbg_inst);
// Same step as launch_step, computed by one 64-lane wavefront per strip segment (no workgroup barriers).
// plain: every instance is periodic in y (LBM_WALLS_NONE) and uses LBM_ADV_PAPER, which selects a kernel
// specialised for that case (the general kernel gives the same results).
template <typename T, typename P>
hipError_t launch_wave(hipStream_t s, int parity, int nseg_launch, const TileDev* segs, const InstDev* inst,
                       T* buf, const DropDev* drops, double* part, uint64_t* mask, const int64_t* step,
                       double* dbg, int dbg_inst, bool plain);
template <typename T, typename P>
hipError_t launch_obs(hipStream_t s, int parity, int ntiles_launch, const TileDev* tiles,
                      const InstDev* inst, T* buf, const DropDev* drops, double* obs_part,
                      int obs_stride);

}  // namespace lbm
