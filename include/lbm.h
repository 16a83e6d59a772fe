/*
 * lbm.h -- C ABI of the MI355X (gfx950) hybrid lattice-Boltzmann / finite-difference
 * solver for chemically driven self-propelled droplets.
 *
 * Model: Fadda, Gonnella, Lamura, Tiribocchi, "Lattice Boltzmann study of
 * chemically-driven self-propelled droplets", EPJ E (2017), arXiv:1711.10984.
 *   - order parameter phi and surfactant c obey convection-diffusion equations
 *     with chemical potentials from the free energy            (Sec. 2.1, Eqs. 1-5)
 *   - the fluid obeys Navier-Stokes + continuity through a D2Q9 BGK lattice
 *     Boltzmann scheme with a forcing term                     (Sec. 2.2, Eqs. 10-15)
 *   - phi and c are advanced by a two-step explicit finite-difference scheme
 *                                                              (Sec. 2.3, Eqs. 16-19)
 *   - surfactant production A(t) Theta(R_s - |r - r_P|) inside each active
 *     droplet and consumption -gamma (c - c0)                  (Sec. 2.1, Sec. 4)
 *   - droplet centres of mass over phi >= 0                    (Sec. 4)
 * All quantities are in lattice units (Delta x = Delta t = 1).  The lattice is periodic.
 *
 * Conventions shared by every entry point
 *   Host field arrays are row-major [ny][nx] doubles, x fastest.  Populations are
 *   [9][ny][nx] in the D2Q9 order rest, E(+x), N(+y), W(-x), S(-y), NE, NW, SW, SE.
 *   Batched contexts hold several independent lattices ("instances"); host arrays for
 *   a batch are the instances' arrays concatenated in instance order.
 *   Device memory belongs to the caller: the library carves all its buffers out of one
 *   caller-allocated workspace and never allocates or frees device memory itself
 *   (hipGraph objects and hipEvents are the only HIP objects it creates).  The HIP
 *   stream also belongs to the caller; all work is enqueued on it.  Host arrays belong
 *   to the caller and are only read or written during the call.
 *   Every function returns LBM_OK (0) or a negative error code; nothing is thrown across
 *   the ABI.  lbm_last_error() returns a thread-local description of the last failure.
 *   lbm_step() does not synchronise; device-side problems (non-finite values, B(c) <= 0)
 *   are reported by the next lbm_observables() call.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_E_INVAL -1    /* invalid argument or configuration */
#define LBM_E_NOMEM -2    /* workspace too small */
#define LBM_E_HIP -3      /* a HIP runtime call failed */
#define LBM_E_UNSTABLE -4 /* non-finite state or B(c) <= 0 somewhere (Sec. 4: B(c) > 0 is required) */
#define LBM_E_STATE -5    /* call not valid in the current state */

#define LBM_FP64 0 /* populations, fields and arithmetic in FP64 */
#define LBM_FP32 1 /* populations stored as FP32 deviations f_i - w_i n0 from the rest state, fields and
                      arithmetic in FP32; droplet sums in FP64 */
#define LBM_FP16 2 /* populations stored as FP16 deviations f_i - w_i n0 from the rest state (round to
                      nearest even), widened to FP32 on load; fields and arithmetic FP32; sums FP64 */

/* Boundaries in y (Sec. 2.2 names bounding walls, Sec. 2.3 neutral wetting at them).  LBM_WALLS_Y:
 * solid plates halfway between node rows, at y = -1/2 and y = ny - 1/2, x periodic.  Populations that
 * stream into a plate return to their node in the opposite direction (halfway bounce-back, no-slip);
 * every scalar field entering a stencil is continued across a plate by its mirror image (neutral
 * wetting, n.grad phi = 0, and no diffusive flux through the plate, n.grad mu_phi = n.grad mu_c = 0);
 * the advection stencil sees the mirrored velocity with u_y reversed (no flow through the plate);
 * droplet distances and centres are not periodic in y. */
#define LBM_WALLS_NONE 0
#define LBM_WALLS_Y 1

#define LBM_ADV_PAPER 0 /* advection half-step of Eqs. (16)-(17) as printed */
#define LBM_ADV_FLUX 1  /* conservative face-upwind flux form of the same half-step */

#define LBM_PATH_FUSED 0 /* one sweeping kernel per step (default) */
#define LBM_PATH_SPLIT 1 /* lattice-Boltzmann kernel, then finite-difference kernel (reference layout) */
#define LBM_PATH_WAVE 2  /* one sweeping kernel per step, one wavefront per strip, no workgroup barriers */

#define LBM_MAXDROP 256 /* droplets per instance */
#define LBM_NSTAGE 22   /* planes written by lbm_debug_stage */

/* Per-instance model parameters (lattice units). */
typedef struct lbm_config {
  int32_t nx, ny;     /* lattice, nx, ny >= 3; periodic in x, and in y without walls */
  int32_t precision;  /* LBM_FP64, LBM_FP32 or LBM_FP16; equal for every instance of a batch */
  int32_t advection;  /* LBM_ADV_PAPER or LBM_ADV_FLUX */
  int32_t walls;      /* LBM_WALLS_NONE or LBM_WALLS_Y */
  int32_t reserved;   /* 0 */
  double tau;         /* BGK relaxation time, > 1/2; viscosity (tau - 1/2)/3 (Eq. 15) */
  double n0;          /* initial fluid density (populations w_i n0 when none are given) */
  double a, b;        /* bulk free energy a phi^2/2 + b phi^4/4, b > 0 (Eq. 1) */
  double B0, B1;      /* gradient coupling B(c) = B0 + B1 c (Eq. 1) */
  double D;           /* surfactant mobility L(c) = D c (Eq. 4) */
  double Gamma;       /* mobility of phi multiplying the Laplacian in Eq. (18) (1 in the paper) */
  double gamma;       /* consumption rate (Sec. 2.1) */
  double A0;          /* production ramp A(n) = A0 min(n, t_star) (Sec. 4) */
  double t_star;
  double c0;          /* consumption floor c0 (Sec. 2.1) */
} lbm_config;

/* One droplet: tracked centre of mass, radius, production disk (Sec. 2.1, Sec. 4). */
typedef struct lbm_droplet {
  double x, y;   /* centre of mass r_CM; at init the centre the first CM pass starts from */
  double R, Rs;  /* droplet radius and production-disk radius */
  double ex, ey; /* unit vector: production disk centred at r_P = r_CM + (R - Rs) e */
  int32_t active; /* 1: produces surfactant; 0: passive (tracked only) */
  int32_t reserved;
} lbm_droplet;

/* Conserved sums and stability diagnostics of one instance at the current step. */
typedef struct lbm_obs {
  int64_t step;      /* n */
  double mass;       /* sum_r sum_i f_i (Eq. 11) */
  double sum_phi;    /* sum_r phi */
  double sum_c;      /* sum_r c */
  double min_B;      /* min_r B0 + B1 c (must stay > 0, Sec. 4) */
  double max_u;      /* max_r |u| */
  int32_t nonfinite; /* 1 if any population, phi or c is not finite */
  int32_t ndrop;
} lbm_obs;

typedef struct lbm_ctx lbm_ctx;

/* Bytes of device workspace a batch of `ninst` instances needs.  cfgs[ninst], ndrop[ninst]. */
int lbm_workspace_bytes(int32_t ninst, const lbm_config* cfgs, const int32_t* ndrop, size_t* bytes);

/* Create a batch and set its state at step `step` (Sec. 2).
 *   workspace: device pointer, >= lbm_workspace_bytes(), 256-byte aligned, owned by the caller and
 *              used exclusively by this context until lbm_destroy().
 *   stream:    hipStream_t owned by the caller (a non-default stream enables graph replay).
 *   phi0, c0:  host, concatenated [ny][nx] per instance.
 *   f_pre:     host, concatenated [9][ny][nx] pre-collision populations, or NULL for w_i n0.
 *   drops:     host, concatenated droplet tables (ndrop[i] each).  Initial centres of mass are one
 *              centre-of-mass pass over phi0 started from the given (x, y).
 * Errors: LBM_E_INVAL (nx, ny < 3, tau <= 1/2, b <= 0, mixed precision, too many droplets,
 * misaligned workspace), LBM_E_NOMEM (workspace too small), LBM_E_HIP. */
int lbm_init_batch(int32_t ninst, const lbm_config* cfgs, void* workspace, size_t workspace_bytes,
                   void* stream, const double* phi0, const double* c0, const double* f_pre,
                   const int32_t* ndrop, const lbm_droplet* drops, int64_t step, lbm_ctx** out);

/* Single-instance form of lbm_init_batch. */
int lbm_init(const lbm_config* cfg, void* workspace, size_t workspace_bytes, void* stream,
             const double* phi0, const double* c0, const double* f_pre, int32_t ndrop,
             const lbm_droplet* drops, int64_t step, lbm_ctx** out);

/* Advance every instance by n >= 0 timesteps n -> n+1 (Sec. 2.2-2.3, Eqs. 10-19, then the
 * centre-of-mass update of Sec. 4).  Asynchronous on the context's stream. */
int lbm_step(lbm_ctx* ctx, int64_t n);

/* Replay the timestep through hipGraphs of `steps_per_graph` steps (even, >= 2), or launch kernels
 * one by one when 0.  Default: 20 on a non-default stream, 0 on the null stream.  The two graphs (one per
 * parity of the starting step) are captured by this call; changing the path, strip height or width drops
 * them, and the next lbm_step captures them again.  lbm_step replays whole graphs while at least
 * steps_per_graph steps remain and launches the rest one by one. */
int lbm_set_graph(lbm_ctx* ctx, int32_t steps_per_graph);

/* Wait for the context's stream. */
int lbm_sync(lbm_ctx* ctx);

/* Current step counter n. */
int64_t lbm_get_step(const lbm_ctx* ctx);

/* Copy instance `inst` to host arrays (any may be NULL): pre-collision populations f_pre
 * [9][ny][nx] at time n, phi, c, and the density and velocity of Eq. (11) at time n (with half
 * the force of Eq. 14 computed from the current phi, c).  Synchronous.  Returns LBM_E_UNSTABLE
 * (after filling the arrays) if a value it returns is non-finite. */
int lbm_fields(lbm_ctx* ctx, int32_t inst, double* f_pre, double* phi, double* c, double* n, double* ux,
               double* uy);

/* Observables of instance `inst` at the current step.  drop_out (may be NULL): per droplet
 * {x_cm, y_cm, vx, vy, sum_phi}, the velocity being the phi-weighted mean of u over the
 * droplet's nodes (phi >= 0, nearest centre).  Synchronous.  Returns LBM_E_UNSTABLE (after
 * filling *obs) if a value is non-finite or B(c) <= 0. */
int lbm_observables(lbm_ctx* ctx, int32_t inst, lbm_obs* obs, double* drop_out);

/* Current droplet table of instance `inst` (ndrop entries).  Synchronous. */
int lbm_droplets(lbm_ctx* ctx, int32_t inst, lbm_droplet* out);

/* Test hook: the intermediate planes of the next step of instance `inst` as computed by the
 * production kernels, without advancing the state.  out: host [LBM_NSTAGE][ny][nx] doubles in
 * the order mu_phi, X = (B1/2)|grad phi|^2, Fx, Fy, n, ux, uy, phi^{n+1/2}, c^{n+1/2}, M
 * (bracket of Eq. 18), X^{n+1/2}, phi^{n+1}, c^{n+1}, f*_0..8 (post-collision, before
 * streaming; with FP32 arithmetic the deviation from w_i n0 plus w_i n0 in double, before the storage
 * rounding).  Instances of at most 512 x 512 nodes (LBM_E_INVAL otherwise).  Synchronous. */
int lbm_debug_stage(lbm_ctx* ctx, int32_t inst, double* out);

/* Kernel sequence used by lbm_step and lbm_debug_stage: LBM_PATH_FUSED (default), LBM_PATH_SPLIT or
 * LBM_PATH_WAVE.  All compute the same arithmetic; the split path stores u^n between its two kernels,
 * the wave path sweeps each strip with a single wavefront.  LBM_E_INVAL for another value. */
int lbm_set_path(lbm_ctx* ctx, int32_t path);
int32_t lbm_get_path(const lbm_ctx* ctx);

/* Rows per strip segment of the sweeping kernels (fused and wave paths), LBM_SEG_ROWS_MIN ..
 * LBM_SEG_ROWS_MAX (default 64; LBM_E_INVAL outside).  Taller segments recompute fewer halo rows;
 * shorter ones give more workgroups.  Synchronous. */
#define LBM_SEG_ROWS_MIN 16
#define LBM_SEG_ROWS_MAX 4096
int lbm_set_seg_rows(lbm_ctx* ctx, int32_t rows);
int32_t lbm_get_seg_rows(const lbm_ctx* ctx);

/* Columns owned per strip of the sweeping kernels, LBM_STRIP_W_MIN .. LBM_STRIP_W_MAX (default 54, the
 * most a 64-lane wavefront covers with its 5-column halo on each side; LBM_E_INVAL outside).  Only the work
 * decomposition changes: the fields are identical for every width (the centre-of-mass partial sums are
 * added in a different order).  Synchronous. */
#define LBM_STRIP_W_MIN 32
#define LBM_STRIP_W_MAX 54
int lbm_set_strip_width(lbm_ctx* ctx, int32_t width);
int32_t lbm_get_strip_width(const lbm_ctx* ctx);

/* The LBM_TUNE_NROWS segment heights tried by lbm_autotune, ascending (static array). */
#define LBM_TUNE_NROWS 16
const int32_t* lbm_tune_rows(void);
/* The LBM_TUNE_NWIDTHS strip widths tried by lbm_autotune (static array). */
#define LBM_TUNE_NWIDTHS 1
const int32_t* lbm_tune_widths(void);

/* Autotuner: time `launches` back-to-back launches of the sweeping kernel for each candidate strip width
 * and height (heights giving the same number of segments as a smaller one at that width are skipped) -- for
 * both sweeping kernels (LBM_PATH_FUSED, LBM_PATH_WAVE) and the split pair (LBM_PATH_SPLIT, no width or
 * height) when both_paths != 0, else for the current sweeping path only -- and set the path, width and
 * height of the fastest (the width is then read with lbm_get_strip_width).
 * The trial launches read the current state and write only scratch (the inactive halves of the ping-pong
 * buffers, the velocity planes and the centre-of-mass partials): the state, the droplet table and the step
 * counter are unchanged.  Called on the split path with both_paths == 0, nothing is tried.
 * rows_out, path_out (may be NULL) receive the choice; ms_out (may be NULL, 2 * LBM_TUNE_NWIDTHS *
 * LBM_TUNE_NROWS + 1 entries: [path (fused, wave)][width][height], then split) the average ms per launch
 * (per step pair for the split path) of each candidate (-1 if not tried).  Synchronous. */
int lbm_autotune(lbm_ctx* ctx, int32_t launches, int32_t both_paths, int32_t* rows_out, int32_t* path_out,
                 double* ms_out);

/* Average device time per launch (ms) of each kernel of the timestep over n eagerly launched steps,
 * measured with hipEvents on the context's stream.  Fused path: ms_out = {k_step, k_reduce, 0};
 * wave path: {k_wave, k_reduce, 0}; split path: {k_lb, k_fd, k_reduce}.  Advances the state by n steps.  Synchronous. */
int lbm_time_kernels(lbm_ctx* ctx, int64_t n, double* ms_out);

/* Device time per launch (ms) of the timestep's main kernels, without the gaps that events or host launches
 * between kernels add: `launches` back-to-back launches of each kernel, captured in a hipGraph, replayed once to
 * warm up and once between two hipEvents on the context's stream (non-default; LBM_E_STATE otherwise), total
 * time / launches.  Fused path: ms_out = {k_step, k_reduce, 0}; wave path: {k_wave, k_reduce, 0}; split path:
 * {k_lb, k_fd, k_reduce}.  Like the autotuner's trials, the launches read the current state and write only
 * scratch (the inactive halves of the ping-pong buffers, the velocity planes and the centre-of-mass partials;
 * k_reduce runs in a mode that computes the droplet sums and writes nothing): the state, the droplet table and
 * the step counter are unchanged.  Synchronous. */
int lbm_time_launches(lbm_ctx* ctx, int32_t launches, double* ms_out);

/* ---- For callers that cannot allocate ------------------------------------------------------------------
 * Code under HIP stream capture, tight serving loops and harnesses that forbid allocation can advance one
 * lattice with lbm_step_noalloc: no context, no workspace, no graph.  It calls no hipMalloc, hipFree or other
 * allocating routine and never synchronises; it only enqueues kernels on `stream` (may be NULL).  Its scratch
 * (instance description, strip list, step counter, droplet table, centre-of-mass partials and masks) is a static
 * device array of LBM_NOALLOC_SCRATCH_BYTES that each GPU holds until the process ends; lattices whose scratch
 * would not fit are rejected (LBM_E_NOMEM; e.g. 2048 x 2048 with up to 256 droplets fits).  Calls on one GPU
 * share that array: calls that overlap in time on one GPU (other streams, other threads) race; calls ordered on
 * one stream do not.
 * The caller passes the state (inputs and outputs) in device memory, each buffer 256-byte aligned, rows of nx
 * values with no padding:
 *   f[0], f[1]:   [9][ny][nx] post-collision populations stored at the emitting node, f*_i(r), so that the
 *                 pre-collision population is f_i(r) = f*_i(r - e_i) (with LBM_WALLS_Y, f*_OPP(i)(r) where r - e_i
 *                 lies behind a plate); LBM_FP64 stores doubles, LBM_FP32 the floats f*_i - (float)(w_i n0),
 *                 LBM_FP16 the _Float16 values of (float)f*_i - (float)(w_i n0);
 *   phi[0..1], c[0..1]: [ny][nx] doubles (LBM_FP64) or floats;
 *   drops:        device array of `ndrop` lbm_droplet, the current centres of mass r_CM (e.g. from
 *                 lbm_droplets), updated in place with the centres after the run.
 * The state at step `step` is read from f[0], phi[0], c[0]; after nsteps steps (Secs. 2.2-2.3 and the Sec. 4
 * centre update, the wave-path kernels of lbm_step at strip width 54 and height 40) the state at step + nsteps is
 * in index (nsteps mod 2) of each pair, and the other index holds the state one step earlier (nsteps >= 1).
 * Results equal those of lbm_step on the same state bit for bit.  Errors: LBM_E_INVAL (configuration as for
 * lbm_init, NULL or misaligned buffers, step or nsteps < 0), LBM_E_NOMEM (scratch too small), LBM_E_HIP. */
#define LBM_NOALLOC_SCRATCH_BYTES (16u << 20)
int lbm_step_noalloc(const lbm_config* cfg, void* stream, void* const f[2], void* const phi[2], void* const c[2],
                     int32_t ndrop, lbm_droplet* drops, int64_t step, int64_t nsteps);

/* ---- Reverse mode (the derivative of a droplet's displacement; Sec. 4 centre of mass) ----
 * The loss is J = x_CM(n0 + nsteps) - x_CM(n0) of droplet `drop` (minimum image in x, so |J| < nx/2), and the
 * derivatives are with respect to the production rate A0 of Sec. 4 (A(n) = A0 min(n, t_star)) and to the
 * surfactant field c at the start of the run, n0.  The adjoint is the exact transpose of the discrete step
 * (Eqs. 3, 5, 10-19) with these held fixed: the nodes inside each production disk, the upwind side chosen by
 * the sign of u in Eqs. (16)-(17) and the droplet masks (phi >= 0, nearest centre); none of them is
 * differentiable.  Contexts of one lattice (periodic, or with LBM_WALLS_Y), LBM_FP64 or LBM_FP32,
 * LBM_ADV_PAPER (LBM_E_INVAL otherwise).
 * Memory: a checkpoint of the state every `every` steps (9 population planes, phi, c), and for the interval
 * being reversed phi, c and 11 FP64 stage planes of each step, plus 26 planes of one backward step, live
 * in a caller-owned device workspace of lbm_adjoint_bytes bytes (the library allocates nothing); it must stay
 * untouched between the forward and the backward call.  An interval near sqrt(nsteps) keeps it smallest. */
int lbm_adjoint_bytes(const lbm_ctx* ctx, int64_t nsteps, int32_t every, size_t* bytes);
/* Forward pass: advances the context by nsteps steps (as lbm_step) from its current state n0, keeping a
 * checkpoint every `every` steps in ws.  J (may be NULL) receives the loss.  Synchronous. */
int lbm_adjoint_forward(lbm_ctx* ctx, void* ws, size_t bytes, int32_t drop, int64_t nsteps, int32_t every,
                        double* J);
/* Backward pass of the last lbm_adjoint_forward on this context (LBM_E_STATE if the context has stepped
 * since): recomputes each checkpoint interval, then runs the adjoint kernels from n0 + nsteps back to n0.
 * dJ_dA0 (may be NULL) receives dJ/dA0; dJ_dc0 (may be NULL, host [ny][nx], x fastest) receives dJ/dc(n0).
 * The context is left at n0 + nsteps.  May be called again.  Synchronous. */
int lbm_adjoint_backward(lbm_ctx* ctx, void* ws, size_t bytes, double* dJ_dA0, double* dJ_dc0);

/* Name of kernel `which` (0..2) of lbm_time_kernels for a path (static string, "" if none). */
const char* lbm_kernel_name(int32_t path, int32_t which);

/* Release the context (graphs, events, host bookkeeping).  The workspace is not freed. */
void lbm_destroy(lbm_ctx* ctx);

/* Description of the last error on this thread ("" if none). */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
