// Host side of the C ABI declared in include/lbm.h: workspace layout, validation, state transfer,
// launch sequencing (eager or hipGraph replay), observables and the stage-export test hook.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/lbm.h"
#include "lbm_adjoint.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// A named host range on profiler timelines (rocprofv3 --marker-trace); a plain call when no tool is attached.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

#define HIPCHK(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return fail(LBM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr size_t ALIGN = 256;
// lbm_debug_stage exports planes only for instances up to this many nodes (its scratch is sized by it).
constexpr int64_t DEBUG_MAX_NODES = 512 * 512;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// D2Q9 directions in the public order rest, E, N, W, S, NE, NW, SW, SE.
constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};  // e_OPP[k] = -e_k
constexpr double WGT[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                           1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

// Workspace layout of a batch: one typed pool for all fields, then bookkeeping arrays.
struct Layout {
  int prec = 0;
  size_t elem = 8;
  std::vector<InstDev> inst;
  std::vector<TileDev> tiles;  // split-kernel tiles in launch order (XCD-aware), padded with inst = -1
  std::vector<TileDev> segs;   // fused-kernel strips in launch order
  int ntiles = 0, nsegs = 0, ndrop_total = 0, max_nd = 0, obs_stride = 0;
  int max_segs = 0, max_seg_launch = 0, seg_rows = 0, strip_w = FUSED_TX;
  int64_t max_nodes = 0;
  size_t off_pool = 0, off_inst = 0, off_tiles = 0, off_segs = 0, off_drops = 0, off_part = 0, off_mask = 0,
         off_step = 0, off_obs = 0, off_dbg = 0, total = 0;
};

int validate(int32_t ninst, const lbm_config* cfgs, const int32_t* ndrop) {
  if (ninst <= 0 || !cfgs || !ndrop) return fail(LBM_E_INVAL, "ninst must be > 0 with configs and droplet counts");
  for (int i = 0; i < ninst; ++i) {
    const lbm_config& c = cfgs[i];
    char where[64];
    snprintf(where, sizeof where, "instance %d: ", i);
    if (c.nx < 3 || c.ny < 3) return fail(LBM_E_INVAL, std::string(where) + "nx and ny must be >= 3");
    if ((int64_t)c.nx * c.ny > (int64_t)1 << 30) return fail(LBM_E_INVAL, std::string(where) + "lattice too large");
    if (c.precision != LBM_FP64 && c.precision != LBM_FP32 && c.precision != LBM_FP16)
      return fail(LBM_E_INVAL, std::string(where) + "precision must be LBM_FP64, LBM_FP32 or LBM_FP16");
    if (c.precision != cfgs[0].precision) return fail(LBM_E_INVAL, "all instances of a batch need the same precision");
    if (c.advection != LBM_ADV_PAPER && c.advection != LBM_ADV_FLUX)
      return fail(LBM_E_INVAL, std::string(where) + "unknown advection scheme");
    if (c.walls != LBM_WALLS_NONE && c.walls != LBM_WALLS_Y)
      return fail(LBM_E_INVAL, std::string(where) + "walls must be LBM_WALLS_NONE or LBM_WALLS_Y");
    if (!(c.tau > 0.5)) return fail(LBM_E_INVAL, std::string(where) + "tau must exceed 1/2");
    if (!(c.b > 0.0)) return fail(LBM_E_INVAL, std::string(where) + "b must be positive");
    if (!(c.n0 > 0.0)) return fail(LBM_E_INVAL, std::string(where) + "n0 must be positive");
    const double vals[] = {c.a, c.B0, c.B1, c.D, c.Gamma, c.gamma, c.A0, c.t_star, c.c0};
    for (double v : vals)
      if (!std::isfinite(v)) return fail(LBM_E_INVAL, std::string(where) + "parameters must be finite");
    if (ndrop[i] < 0 || ndrop[i] > LBM_MAXDROP)
      return fail(LBM_E_INVAL, std::string(where) + "droplet count out of range [0, LBM_MAXDROP]");
  }
  return LBM_OK;
}

// Model parameters of an instance, derived in double precision (advection form, walls, Eqs. 1-19).
void set_model(const lbm_config& c, InstDev& d) {
  d.advection = c.advection;
  d.walls = c.walls;
  d.yper = c.walls ? std::numeric_limits<double>::infinity() : (double)c.ny;
  d.a = c.a;
  d.b = c.b;
  d.B0 = c.B0;
  d.B1 = c.B1;
  d.halfB1 = 0.5 * c.B1;
  d.D = c.D;
  d.Gamma = c.Gamma;
  d.gamma = c.gamma;
  d.c0 = c.c0;
  d.omega = 1.0 / c.tau;
  d.coef = 1.0 - 1.0 / (2.0 * c.tau);
  d.A0 = c.A0;
  d.t_star = c.t_star;
  d.wn[0] = WGT[0] * c.n0;
  d.wn[1] = WGT[1] * c.n0;
  d.wn[2] = WGT[5] * c.n0;
  d.n0 = c.n0;
}

void make_layout(int32_t ninst, const lbm_config* cfgs, const int32_t* ndrop, Layout& L) {
  L.prec = cfgs[0].precision;
  L.elem = L.prec == LBM_FP64 ? 8 : 4;
  const size_t row_align = ALIGN / L.elem;
  int64_t pool_elems = 0;
  int tile_base = 0, seg_base = 0, drop_base = 0;
  int64_t part_elems = 0, part_elems1 = 0;
  L.inst.resize(ninst);
  for (int i = 0; i < ninst; ++i) {
    const lbm_config& c = cfgs[i];
    InstDev& d = L.inst[i];
    memset(&d, 0, sizeof d);
    d.nx = c.nx;
    d.ny = c.ny;
    d.pitch = (int32_t)align_up((size_t)c.nx, row_align);
    d.ndrop = ndrop[i];
    d.tiles_x[TILING_SPLIT] = (c.nx + TILE_X - 1) / TILE_X;
    d.tiles_y[TILING_SPLIT] = (c.ny + TILE_Y - 1) / TILE_Y;
    d.tile_base[TILING_SPLIT] = tile_base;
    // upper bounds (narrowest strips, shortest segments); see set_segments
    d.tiles_x[TILING_FUSED] = (c.nx + STRIP_W_MIN - 1) / STRIP_W_MIN;
    d.tiles_y[TILING_FUSED] = (c.ny + SEG_ROWS_MIN - 1) / SEG_ROWS_MIN;
    d.tile_base[TILING_FUSED] = seg_base;
    d.drop_base = drop_base;
    const int64_t plane = (int64_t)c.ny * d.pitch;
    d.pstride = plane;
    // a population buffer holds 9 planes of the storage type (FP16 deviations take half a field plane)
    const int64_t fbuf = L.prec == LBM_FP16 ? (int64_t)align_up((size_t)(9 * plane / 2), row_align) : 9 * plane;
    int64_t o = pool_elems;
    d.off_f[0] = o;  o += fbuf;
    d.off_f[1] = o;  o += fbuf;
    d.off_phi[0] = o; o += plane;
    d.off_phi[1] = o; o += plane;
    d.off_c[0] = o;  o += plane;
    d.off_c[1] = o;  o += plane;
    d.off_ux = o;    o += plane;
    d.off_uy = o;    o += plane;
    d.off_n = o;     o += plane;
    pool_elems = o;
    d.part_base[TILING_SPLIT] = part_elems;
    part_elems += (int64_t)d.tiles_x[TILING_SPLIT] * d.tiles_y[TILING_SPLIT] * d.ndrop * 3;
    d.part_base[TILING_FUSED] = part_elems1;
    part_elems1 += (int64_t)d.tiles_x[TILING_FUSED] * d.tiles_y[TILING_FUSED] * d.ndrop * 3;
    set_model(c, d);
    tile_base += d.tiles_x[TILING_SPLIT] * d.tiles_y[TILING_SPLIT];
    seg_base += d.tiles_x[TILING_FUSED] * d.tiles_y[TILING_FUSED];
    drop_base += d.ndrop;
    L.max_nd = std::max(L.max_nd, (int)d.ndrop);
    L.max_nodes = std::max(L.max_nodes, (int64_t)c.nx * c.ny);
  }
  L.ntiles = tile_base;
  L.nsegs = seg_base;
  L.ndrop_total = drop_base;
  L.obs_stride = 6 + 3 * L.max_nd;
  // Work lists in launch order: workgroup b runs on XCD (b mod 8); give each XCD a contiguous run of
  // tiles (raster order within an instance) so that neighbouring tiles share that XCD's L2.
  auto build_list = [&](int tiling, int tw, int th, int count, std::vector<TileDev>& out) {
    std::vector<TileDev> natural;
    natural.reserve(count);
    for (int i = 0; i < ninst; ++i) {
      const InstDev& d = L.inst[i];
      for (int ty = 0; ty < d.tiles_y[tiling]; ++ty)
        for (int tx = 0; tx < d.tiles_x[tiling]; ++tx)
          natural.push_back(TileDev{i, tx * tw, ty * th, (int32_t)natural.size()});
    }
    const int nxcd = 8;
    const int chunk = (count + nxcd - 1) / nxcd;
    out.assign((size_t)chunk * nxcd, TileDev{-1, 0, 0, -1});
    for (int t = 0; t < count; ++t) out[(size_t)(t % chunk) * nxcd + t / chunk] = natural[t];
  };
  build_list(TILING_SPLIT, TILE_X, TILE_Y, L.ntiles, L.tiles);
  L.max_segs = L.nsegs;  // strips of the narrowest width and smallest height: sizes the strip list and partials
  L.max_seg_launch = ((L.nsegs + 7) / 8) * 8;
  (void)build_list;
  size_t off = 0;
  L.off_pool = off;  off = align_up(off + (size_t)pool_elems * L.elem, ALIGN);
  L.off_inst = off;  off = align_up(off + sizeof(InstDev) * ninst, ALIGN);
  L.off_tiles = off; off = align_up(off + sizeof(TileDev) * L.tiles.size(), ALIGN);
  L.off_segs = off;  off = align_up(off + sizeof(TileDev) * (size_t)L.max_seg_launch, ALIGN);
  L.off_drops = off; off = align_up(off + sizeof(DropDev) * std::max(1, L.ndrop_total), ALIGN);
  // the two tilings share the partials and masks (one of them is in use at a time)
  L.off_part = off;
  off = align_up(off + sizeof(double) * std::max<int64_t>(1, std::max(part_elems, part_elems1)), ALIGN);
  L.off_mask = off;
  off = align_up(off + sizeof(uint64_t) * MASK_WORDS * (size_t)std::max(L.ntiles, L.nsegs), ALIGN);
  L.off_step = off;  off = align_up(off + sizeof(int64_t), ALIGN);
  L.off_obs = off;   off = align_up(off + sizeof(double) * (size_t)L.obs_stride * L.ntiles, ALIGN);
  L.off_dbg = off;
  off = align_up(off + sizeof(double) * (size_t)LBM_NSTAGE * std::min(L.max_nodes, DEBUG_MAX_NODES), ALIGN);
  L.total = off;
}

// Whether the owned box [x0, x1] x [y0, y1] of a strip segment of instance d comes within R + 2 (minimum
// image) of a droplet centre, i.e. may hold the droplet's phi >= 0 nodes or its production disk.  Such
// segments take longer (centre-of-mass sums, disk test) and are dispatched first.
bool segment_holds_droplet(const InstDev& d, const std::vector<DropDev>& drops, int inst, int x0, int x1, int y0,
                           int y1) {
  const double xm = 0.5 * (x0 + x1), ym = 0.5 * (y0 + y1), hx = 0.5 * (x1 - x0), hy = 0.5 * (y1 - y0);
  for (const DropDev& q : drops) {
    if (q.inst != inst) continue;
    double dx = std::fabs(xm - q.x), dy = std::fabs(ym - q.y);
    if (dx > 0.5 * d.nx) dx = d.nx - dx;
    if (!d.walls && dy > 0.5 * d.ny) dy = d.ny - dy;
    dx = std::max(0.0, dx - hx);
    dy = std::max(0.0, dy - hy);
    const double r = q.R + 2.0;
    if (dx * dx + dy * dy <= r * r) return true;
  }
  return false;
}

// Sweeping-kernel strips for a strip width and segment height: per-instance counts, natural indices,
// partial offsets and the launch list.  The list is XCD-aware: workgroup b runs on XCD (b mod 8), and each
// XCD gets a contiguous run of strips in natural order (neighbouring strips share that XCD's L2); within
// its run, the strips that hold droplets (as of `drops`) are dispatched first, so that the longer-running
// ones do not end the launch.  The launch order does not change any result (partials are stored by natural
// index).  Fits in the regions sized for STRIP_W_MIN and SEG_ROWS_MIN.
void set_segments(Layout& L, int seg_rows, int strip_w, const std::vector<DropDev>& drops) {
  int base = 0;
  int64_t part = 0;
  for (auto& d : L.inst) {
    d.seg_rows = seg_rows;
    d.strip_w = strip_w;
    d.tiles_x[TILING_FUSED] = (d.nx + strip_w - 1) / strip_w;
    d.tiles_y[TILING_FUSED] = (d.ny + seg_rows - 1) / seg_rows;
    d.tile_base[TILING_FUSED] = base;
    d.part_base[TILING_FUSED] = part;
    base += d.tiles_x[TILING_FUSED] * d.tiles_y[TILING_FUSED];
    part += (int64_t)d.tiles_x[TILING_FUSED] * d.tiles_y[TILING_FUSED] * d.ndrop * 3;
  }
  L.nsegs = base;
  L.seg_rows = seg_rows;
  L.strip_w = strip_w;
  std::vector<TileDev> natural;
  natural.reserve(base);
  for (size_t i = 0; i < L.inst.size(); ++i) {
    const InstDev& d = L.inst[i];
    for (int ty = 0; ty < d.tiles_y[TILING_FUSED]; ++ty)
      for (int tx = 0; tx < d.tiles_x[TILING_FUSED]; ++tx)
        natural.push_back(TileDev{(int32_t)i, tx * strip_w, ty * seg_rows, (int32_t)natural.size()});
  }
  const int nxcd = 8;
  const int chunk = (base + nxcd - 1) / nxcd;
  L.segs.assign((size_t)chunk * nxcd, TileDev{-1, 0, 0, -1});
  std::vector<TileDev> run;
  for (int j = 0; j < nxcd; ++j) {
    run.clear();
    const int t0 = j * chunk, t1 = std::min(base, (j + 1) * chunk);
    for (int pass = 0; pass < 2; ++pass)
      for (int t = t0; t < t1; ++t) {
        const TileDev& s = natural[t];
        const InstDev& d = L.inst[s.inst];
        const bool heavy = segment_holds_droplet(d, drops, s.inst, s.x0, std::min(s.x0 + strip_w, d.nx) - 1, s.y0,
                                                 std::min(s.y0 + seg_rows, d.ny) - 1);
        if (heavy == (pass == 0)) run.push_back(s);
      }
    for (size_t k = 0; k < run.size(); ++k) L.segs[k * nxcd + j] = run[k];
  }
}


}  // namespace

struct lbm_ctx {
  Layout L;
  std::vector<lbm_config> cfg;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int parity = 0;
  int64_t step = 0;
  int graph_steps = 0;
  int path = LBM_PATH_FUSED;
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  hipGraph_t graph[2] = {nullptr, nullptr};
  // the last recorded forward pass of lbm_adjoint_forward (see lbm_adjoint_backward)
  struct {
    bool valid = false;
    int64_t n0 = 0, nsteps = 0;
    int every = 0, drop = 0;
  } adj;

  void* pool() const { return ws + L.off_pool; }
  InstDev* d_inst() const { return reinterpret_cast<InstDev*>(ws + L.off_inst); }
  TileDev* d_tiles() const { return reinterpret_cast<TileDev*>(ws + L.off_tiles); }
  TileDev* d_segs() const { return reinterpret_cast<TileDev*>(ws + L.off_segs); }
  DropDev* d_drops() const { return reinterpret_cast<DropDev*>(ws + L.off_drops); }
  double* d_part() const { return reinterpret_cast<double*>(ws + L.off_part); }
  uint64_t* d_mask() const { return reinterpret_cast<uint64_t*>(ws + L.off_mask); }
  int64_t* d_step() const { return reinterpret_cast<int64_t*>(ws + L.off_step); }
  double* d_obs() const { return reinterpret_cast<double*>(ws + L.off_obs); }
  double* d_dbg() const { return reinterpret_cast<double*>(ws + L.off_dbg); }
  int nlaunch() const { return (int)L.tiles.size(); }
  int nseglaunch() const { return (int)L.segs.size(); }
};

namespace {

// Calls f(T{}, P{}) with the arithmetic type T and the population storage type P of a precision code.
template <class F>
decltype(auto) with_types(int prec, F&& f) {
  if (prec == LBM_FP64) return f(double{}, double{});
  if (prec == LBM_FP32) return f(float{}, float{});
  return f(float{}, _Float16{});
}

// Host side of the population storage (the kernels' lb_moments / lb_collide).  FP64 stores the population.
// FP32 stores the deviation from the rest population, fp32(f - fp32(w_i n0)), read back as that deviation plus
// fp32(w_i n0).  FP16 storage keeps fp16(fp32(f) - fp32(w_i n0)), widened back as fp32(stored) + fp32(w_i n0).
template <typename T, typename P>
P host_pop_store(double f, double wn) {
  if constexpr (sizeof(T) == 8) {
    (void)wn;
    return (T)f;
  } else if constexpr (std::is_same<T, P>::value) {
    return (P)(f - (double)(float)wn);
  } else {
    return (P)((float)f - (float)wn);
  }
}
template <typename T, typename P>
double host_pop_load(P s, double wn) {
  if constexpr (sizeof(T) == 8) {
    (void)wn;
    return (double)s;
  } else if constexpr (std::is_same<T, P>::value) {
    return (double)s + (double)(float)wn;
  } else {
    return (double)((float)s + (float)wn);
  }
}

// Whether every instance is periodic in y with the printed advection (the wave kernel's specialised case).
bool all_plain(const std::vector<InstDev>& inst) {
  for (const InstDev& d : inst)
    if (d.walls != LBM_WALLS_NONE || d.advection != LBM_ADV_PAPER) return false;
  return true;
}

// The sweeping kernel of a strip path (LBM_PATH_FUSED or LBM_PATH_WAVE) over the strip list.
template <typename T, typename P>
hipError_t launch_sweep(lbm_ctx* c, int parity, double* dbg, int dbg_inst) {
  T* buf = reinterpret_cast<T*>(c->pool());
  if (c->path == LBM_PATH_WAVE)
    return launch_wave<T, P>(c->stream, parity, c->nseglaunch(), c->d_segs(), c->d_inst(), buf, c->d_drops(),
                             c->d_part(), c->d_mask(), c->d_step(), dbg, dbg_inst, all_plain(c->L.inst));
  return launch_step<T, P>(c->stream, parity, c->nseglaunch(), c->d_segs(), c->d_inst(), buf, c->d_drops(),
                           c->d_part(), c->d_mask(), c->d_step(), dbg, dbg_inst);
}

// The two tile kernels of the split path.
template <typename T, typename P>
hipError_t launch_split(lbm_ctx* c, int parity) {
  T* buf = reinterpret_cast<T*>(c->pool());
  hipError_t e = launch_lb<T, P>(c->stream, 0, parity, c->nlaunch(), c->d_tiles(), c->d_inst(), buf, nullptr, -1);
  if (e != hipSuccess) return e;
  return launch_fd<T>(c->stream, 0, parity, c->nlaunch(), c->d_tiles(), c->d_inst(), buf, c->d_drops(), c->d_part(),
                      c->d_mask(), c->d_step(), nullptr, -1);
}

template <typename T, typename P>
hipError_t enqueue_step(lbm_ctx* c, int parity) {
  hipError_t e;
  if (c->path != LBM_PATH_SPLIT) {
    e = launch_sweep<T, P>(c, parity, nullptr, -1);
    if (e != hipSuccess) return e;
    return launch_reduce(c->stream, TILING_FUSED, c->L.ndrop_total, c->d_inst(), c->d_drops(), c->d_part(),
                         c->d_mask(), c->d_step(), 1);
  }
  e = launch_split<T, P>(c, parity);
  if (e != hipSuccess) return e;
  return launch_reduce(c->stream, TILING_SPLIT, c->L.ndrop_total, c->d_inst(), c->d_drops(), c->d_part(),
                       c->d_mask(), c->d_step(), 1);
}

hipError_t enqueue_step_any(lbm_ctx* c, int parity) {
  return with_types(c->L.prec, [&](auto t, auto p) { return enqueue_step<decltype(t), decltype(p)>(c, parity); });
}

void destroy_graphs(lbm_ctx* c) {
  for (int p = 0; p < 2; ++p) {
    if (c->exec[p]) (void)hipGraphExecDestroy(c->exec[p]);
    if (c->graph[p]) (void)hipGraphDestroy(c->graph[p]);
    c->exec[p] = nullptr;
    c->graph[p] = nullptr;
  }
}

int build_graph(lbm_ctx* c, int parity) {
  HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
  hipError_t err = hipSuccess;
  for (int s = 0; s < c->graph_steps && err == hipSuccess; ++s) err = enqueue_step_any(c, (parity + s) & 1);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(c->stream, &g);
  if (err != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(LBM_E_HIP, std::string("kernel launch during capture: ") + hipGetErrorString(err));
  }
  if (e2 != hipSuccess) return fail(LBM_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
  c->graph[parity] = g;
  HIPCHK(hipGraphInstantiate(&c->exec[parity], g, nullptr, nullptr, 0));
  return LBM_OK;
}

template <typename T>
void to_device_layout(const double* src, T* dst, int nx, int ny, int pitch) {
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < pitch; ++x) dst[(size_t)y * pitch + x] = x < nx ? (T)src[(size_t)y * nx + x] : T(0);
}

template <typename T, typename P>
int upload_instance(lbm_ctx* c, int i, const double* phi0, const double* c0, const double* f_pre) {
  const InstDev& d = c->L.inst[i];
  const int nx = d.nx, ny = d.ny, pitch = d.pitch;
  const size_t plane = (size_t)d.pstride;
  std::vector<T> h(plane);
  std::vector<P> hf(plane * 9);
  T* base = reinterpret_cast<T*>(c->pool());
  to_device_layout(phi0, h.data(), nx, ny, pitch);
  HIPCHK(hipMemcpyAsync(base + d.off_phi[0], h.data(), plane * sizeof(T), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  to_device_layout(c0, h.data(), nx, ny, pitch);
  HIPCHK(hipMemcpyAsync(base + d.off_c[0], h.data(), plane * sizeof(T), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  // Stored populations are post-collision values at the emitting node: f*_i(r) = f_i(r + e_i); with walls,
  // a population streamed into a plate comes back to r reversed: f*_i(r) = f_OPP[i](r).
  P* fbase = reinterpret_cast<P*>(base + d.off_f[0]);
  const bool walls = c->cfg[i].walls != 0;
  for (int k = 0; k < 9; ++k)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        double v;
        if (f_pre) {
          const int yt = y + EY[k];
          if (walls && (yt < 0 || yt >= ny)) {
            v = f_pre[(size_t)OPP[k] * nx * ny + (size_t)y * nx + x];
          } else {
            const int xs = (x + EX[k] + nx) % nx, ys = (yt + ny) % ny;
            v = f_pre[(size_t)k * nx * ny + (size_t)ys * nx + xs];
          }
        } else {
          v = WGT[k] * c->cfg[i].n0;
        }
        hf[(size_t)k * plane + (size_t)y * pitch + x] = host_pop_store<T, P>(v, WGT[k] * c->cfg[i].n0);
      }
  HIPCHK(hipMemcpyAsync(fbase, hf.data(), 9 * plane * sizeof(P), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  // velocity / density planes start at zero; the second buffers are fully rewritten by the first step
  HIPCHK(hipMemsetAsync(base + d.off_ux, 0, 3 * plane * sizeof(T), c->stream));
  HIPCHK(hipMemsetAsync(base + d.off_f[1], 0, 9 * plane * sizeof(P), c->stream));
  HIPCHK(hipMemsetAsync(base + d.off_phi[1], 0, plane * sizeof(T), c->stream));
  HIPCHK(hipMemsetAsync(base + d.off_c[1], 0, plane * sizeof(T), c->stream));
  return LBM_OK;
}

int check_inst(lbm_ctx* c, int32_t inst) {
  if (!c) return fail(LBM_E_INVAL, "null context");
  if (inst < 0 || inst >= (int)c->L.inst.size()) return fail(LBM_E_INVAL, "instance index out of range");
  return LBM_OK;
}

// n, u planes of every instance from the current state (Eq. 11 with the force of Eq. 14).
int run_diag(lbm_ctx* c) {
  const hipError_t e = with_types(c->L.prec, [&](auto t, auto p) {
    using T = decltype(t);
    return launch_lb<T, decltype(p)>(c->stream, 2, c->parity, c->nlaunch(), c->d_tiles(), c->d_inst(),
                                     reinterpret_cast<T*>(c->pool()), nullptr, -1);
  });
  if (e != hipSuccess) return fail(LBM_E_HIP, std::string("diagnostic launch: ") + hipGetErrorString(e));
  return LBM_OK;
}

template <typename T>
int download_plane(lbm_ctx* c, int64_t off, const InstDev& d, double* out) {
  const size_t plane = (size_t)d.pstride;
  std::vector<T> h(plane);
  HIPCHK(hipMemcpyAsync(h.data(), reinterpret_cast<T*>(c->pool()) + off, plane * sizeof(T), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int y = 0; y < d.ny; ++y)
    for (int x = 0; x < d.nx; ++x) out[(size_t)y * d.nx + x] = (double)h[(size_t)y * d.pitch + x];
  return LBM_OK;
}

template <typename T, typename P>
int fields_impl(lbm_ctx* c, int inst, double* f_pre, double* phi, double* cc, double* n, double* ux,
                double* uy) {
  const InstDev& d = c->L.inst[inst];
  int rc;
  if (n || ux || uy) {
    if ((rc = run_diag(c)) != LBM_OK) return rc;
  }
  if (phi && (rc = download_plane<T>(c, d.off_phi[c->parity], d, phi)) != LBM_OK) return rc;
  if (cc && (rc = download_plane<T>(c, d.off_c[c->parity], d, cc)) != LBM_OK) return rc;
  if (n && (rc = download_plane<T>(c, d.off_n, d, n)) != LBM_OK) return rc;
  if (ux && (rc = download_plane<T>(c, d.off_ux, d, ux)) != LBM_OK) return rc;
  if (uy && (rc = download_plane<T>(c, d.off_uy, d, uy)) != LBM_OK) return rc;
  if (f_pre) {
    const size_t plane = (size_t)d.pstride;
    std::vector<P> h(9 * plane);
    HIPCHK(hipMemcpyAsync(h.data(), reinterpret_cast<P*>(reinterpret_cast<T*>(c->pool()) + d.off_f[c->parity]),
                          9 * plane * sizeof(P), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int nx = d.nx, ny = d.ny;
    const bool walls = d.walls != 0;
    for (int k = 0; k < 9; ++k)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          // pre-collision f_k(r) = f*_k(r - e_k), or with walls f*_OPP[k](r) when r - e_k is behind a plate
          const int yf = y - EY[k];
          size_t src;
          if (walls && (yf < 0 || yf >= ny)) {
            src = (size_t)OPP[k] * plane + (size_t)y * d.pitch + x;
          } else {
            const int xs = (x - EX[k] + nx) % nx, ys = (yf + ny) % ny;
            src = (size_t)k * plane + (size_t)ys * d.pitch + xs;
          }
          f_pre[(size_t)k * nx * ny + (size_t)y * nx + x] = host_pop_load<T, P>(h[src], WGT[k] * c->cfg[inst].n0);
        }
  }
  return LBM_OK;
}

// Stage planes of the next step of instance `inst` from the kernels of the current path: all LBM_NSTAGE, or only
// the first ADJ_EXPORT_PLANES (all = false).
template <typename T, typename P>
hipError_t debug_launch(lbm_ctx* c, int inst, double* dbg, bool all = true) {
  T* buf = reinterpret_cast<T*>(c->pool());
  const int di = export_planes(inst, all);
  if (c->path != LBM_PATH_SPLIT) return launch_sweep<T, P>(c, c->parity, dbg, di);
  hipError_t e = launch_lb<T, P>(c->stream, 1, c->parity, c->nlaunch(), c->d_tiles(), c->d_inst(), buf, dbg, di);
  if (e != hipSuccess) return e;
  return launch_fd<T>(c->stream, 1, c->parity, c->nlaunch(), c->d_tiles(), c->d_inst(), buf, c->d_drops(), c->d_part(),
                      c->d_mask(), c->d_step(), dbg, di);
}

// One eager step with hipEvents between its kernels: ev[0..nk] bracket nk launches.
template <typename T, typename P>
hipError_t timed_step(lbm_ctx* c, hipEvent_t* ev, int* nk) {
  T* buf = reinterpret_cast<T*>(c->pool());
  const int p = c->parity;
  hipError_t e;
  (void)hipEventRecord(ev[0], c->stream);
  if (c->path != LBM_PATH_SPLIT) {
    e = launch_sweep<T, P>(c, p, nullptr, -1);
    (void)hipEventRecord(ev[1], c->stream);
    if (e == hipSuccess)
      e = launch_reduce(c->stream, TILING_FUSED, c->L.ndrop_total, c->d_inst(), c->d_drops(), c->d_part(), c->d_mask(),
                        c->d_step(), 1);
    (void)hipEventRecord(ev[2], c->stream);
    *nk = 2;
  } else {
    e = launch_lb<T, P>(c->stream, 0, p, c->nlaunch(), c->d_tiles(), c->d_inst(), buf, nullptr, -1);
    (void)hipEventRecord(ev[1], c->stream);
    if (e == hipSuccess)
      e = launch_fd<T>(c->stream, 0, p, c->nlaunch(), c->d_tiles(), c->d_inst(), buf, c->d_drops(), c->d_part(),
                       c->d_mask(), c->d_step(), nullptr, -1);
    (void)hipEventRecord(ev[2], c->stream);
    if (e == hipSuccess)
      e = launch_reduce(c->stream, TILING_SPLIT, c->L.ndrop_total, c->d_inst(), c->d_drops(), c->d_part(), c->d_mask(),
                        c->d_step(), 1);
    (void)hipEventRecord(ev[3], c->stream);
    *nk = 3;
  }
  c->parity ^= 1;
  c->step += 1;
  return e;
}

int read_drops(lbm_ctx* c, int inst, std::vector<DropDev>& out) {
  const InstDev& d = c->L.inst[inst];
  out.resize(d.ndrop);
  if (d.ndrop == 0) return LBM_OK;
  HIPCHK(hipMemcpyAsync(out.data(), c->d_drops() + d.drop_base, sizeof(DropDev) * d.ndrop, hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

// The droplet table of every instance (device copy).
int read_all_drops(lbm_ctx* c, std::vector<DropDev>& out) {
  out.resize(c->L.ndrop_total);
  if (c->L.ndrop_total == 0) return LBM_OK;
  HIPCHK(hipMemcpyAsync(out.data(), c->d_drops(), sizeof(DropDev) * out.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

// Rebuild the strip list for a segment height and strip width (launch order from the current droplet
// centres) and upload it.
int apply_segments(lbm_ctx* c, int rows, int width) {
  HIPCHK(hipStreamSynchronize(c->stream));
  destroy_graphs(c);
  std::vector<DropDev> drops;
  int rc = read_all_drops(c, drops);
  if (rc != LBM_OK) return rc;
  set_segments(c->L, rows, width, drops);
  HIPCHK(hipMemcpyAsync(c->d_inst(), c->L.inst.data(), sizeof(InstDev) * c->L.inst.size(), hipMemcpyHostToDevice,
                        c->stream));
  HIPCHK(hipMemcpyAsync(c->d_segs(), c->L.segs.data(), sizeof(TileDev) * c->L.segs.size(), hipMemcpyHostToDevice,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

// ---- Scratch of the entry point that allocates nothing (lbm_step_noalloc) ---------------------------------
// The instance description, the strip list, the step counter, the droplet table, the centre-of-mass partials
// and the presence masks of lbm_step_noalloc live in this device array: each GPU the library runs on holds its
// own copy until the process ends.  In host code `scratch` names the symbol, not a device address; host code
// uses only the address hipGetSymbolAddress returned on the current device (g_scratch_ptr).
static __device__ __align__(256) unsigned char scratch[LBM_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
constexpr int NOALLOC_SEG_ROWS = 40;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Address of `scratch` on the current device, looked up once per device (with that device current).
int scratch_on_current_device(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(LBM_E_HIP, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(LBM_E_HIP, "hipGetSymbolAddress returned a null address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}

// Byte offsets of the regions of the scratch array for one lattice.
struct NoallocLayout {
  size_t inst, step, drops, segs, mask, part, total;
};

NoallocLayout noalloc_layout(int nsegs, int nslots, int ndrop) {
  NoallocLayout L;
  size_t off = 0;
  L.inst = off;  off = align_up(off + sizeof(InstDev), ALIGN);
  L.step = off;  off = align_up(off + sizeof(int64_t), ALIGN);
  L.drops = off; off = align_up(off + sizeof(DropDev) * (size_t)std::max(1, ndrop), ALIGN);
  L.segs = off;  off = align_up(off + sizeof(TileDev) * (size_t)nslots, ALIGN);
  L.mask = off;  off = align_up(off + sizeof(uint64_t) * MASK_WORDS * (size_t)nsegs, ALIGN);
  L.part = off;  off = align_up(off + sizeof(double) * 3 * (size_t)nsegs * (size_t)std::max(1, ndrop), ALIGN);
  L.total = off;
  return L;
}

// Fills the scratch regions: instance description, step counter, droplet table (from the caller's), the strip
// list in the XCD-aware order of set_segments (natural strip t at slot (t mod chunk) * 8 + t / chunk), and the
// presence masks cleared.
__global__ __launch_bounds__(NTHREADS) void k_noalloc_setup(InstDev inst, int64_t step, NoallocLayout L, int nsegs,
                                                            int nslots, int chunk, int ndrop,
                                                            const lbm_droplet* __restrict__ drops, char* __restrict__ s) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  if (gid == 0) {
    *reinterpret_cast<InstDev*>(s + L.inst) = inst;
    *reinterpret_cast<int64_t*>(s + L.step) = step;
  }
  const int tx = inst.tiles_x[TILING_FUSED];
  TileDev* segs = reinterpret_cast<TileDev*>(s + L.segs);
  for (int b = gid; b < nslots; b += stride) {
    const int t = (b % 8) * chunk + b / 8;
    segs[b] = t < nsegs ? TileDev{0, (t % tx) * inst.strip_w, (t / tx) * inst.seg_rows, t} : TileDev{-1, 0, 0, -1};
  }
  uint64_t* mask = reinterpret_cast<uint64_t*>(s + L.mask);
  for (int m = gid; m < nsegs * MASK_WORDS; m += stride) mask[m] = 0ull;
  DropDev* dd = reinterpret_cast<DropDev*>(s + L.drops);
  for (int k = gid; k < ndrop; k += stride) {
    const lbm_droplet q = drops[k];
    dd[k] = DropDev{q.x, q.y, q.R, q.Rs, q.ex, q.ey, q.active ? 1 : 0, 0};
  }
}

// The new centres back into the caller's droplet table.
__global__ __launch_bounds__(NTHREADS) void k_noalloc_centres(const DropDev* __restrict__ dd, int ndrop,
                                                              lbm_droplet* __restrict__ drops) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < ndrop) {
    drops[k].x = dd[k].x;
    drops[k].y = dd[k].y;
  }
}

}  // namespace

extern "C" {

int lbm_step_noalloc(const lbm_config* cfg, void* stream, void* const f[2], void* const phi[2], void* const c[2],
                     int32_t ndrop, lbm_droplet* drops, int64_t step, int64_t nsteps) {
  if (!cfg) return fail(LBM_E_INVAL, "cfg must not be NULL");
  int rc = validate(1, cfg, &ndrop);
  if (rc != LBM_OK) return rc;
  if (!f || !phi || !c) return fail(LBM_E_INVAL, "f, phi and c must not be NULL");
  void* const bufs[6] = {f[0], f[1], phi[0], phi[1], c[0], c[1]};
  for (void* b : bufs)
    if (!b || reinterpret_cast<uintptr_t>(b) % ALIGN)
      return fail(LBM_E_INVAL, "state buffers must be non-NULL and 256-byte aligned");
  if (ndrop > 0 && !drops) return fail(LBM_E_INVAL, "drops must not be NULL when ndrop > 0");
  if (step < 0 || nsteps < 0) return fail(LBM_E_INVAL, "step and nsteps must be >= 0");
  const lbm_config& cf = *cfg;
  const size_t elem = cf.precision == LBM_FP64 ? 8 : 4;
  InstDev d;
  memset(&d, 0, sizeof d);
  d.nx = cf.nx;
  d.ny = cf.ny;
  d.pitch = cf.nx;
  d.pstride = (int64_t)cf.nx * cf.ny;
  d.ndrop = ndrop;
  d.strip_w = FUSED_TX;
  d.seg_rows = NOALLOC_SEG_ROWS;
  d.tiles_x[TILING_FUSED] = (cf.nx + FUSED_TX - 1) / FUSED_TX;
  d.tiles_y[TILING_FUSED] = (cf.ny + NOALLOC_SEG_ROWS - 1) / NOALLOC_SEG_ROWS;
  // element offsets of the caller's buffers from f[0] (the pool base of the kernels); 256-byte alignment makes
  // every difference a whole number of elements
  const char* base = static_cast<const char*>(f[0]);
  auto off = [&](void* b) { return (int64_t)(static_cast<const char*>(b) - base) / (int64_t)elem; };
  d.off_f[0] = off(f[0]);
  d.off_f[1] = off(f[1]);
  d.off_phi[0] = off(phi[0]);
  d.off_phi[1] = off(phi[1]);
  d.off_c[0] = off(c[0]);
  d.off_c[1] = off(c[1]);
  set_model(cf, d);
  const int nsegs = d.tiles_x[TILING_FUSED] * d.tiles_y[TILING_FUSED];
  const int nslots = (nsegs + 7) / 8 * 8;
  const NoallocLayout L = noalloc_layout(nsegs, nslots, ndrop);
  if (L.total > LBM_NOALLOC_SCRATCH_BYTES)
    return fail(LBM_E_NOMEM, "this lattice and droplet count need " + std::to_string(L.total) +
                                 " bytes of scratch, more than LBM_NOALLOC_SCRATCH_BYTES (" +
                                 std::to_string((size_t)LBM_NOALLOC_SCRATCH_BYTES) + ")");
  void* sp = nullptr;
  if ((rc = scratch_on_current_device(&sp)) != LBM_OK) return rc;
  char* s = static_cast<char*>(sp);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int work = std::max(std::max(nslots, nsegs * MASK_WORDS), ndrop);
  hipLaunchKernelGGL(k_noalloc_setup, dim3((work + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), 0, st, d, step, L, nsegs,
                     nslots, nslots / 8, ndrop, drops, s);
  HIPCHK(hipGetLastError());
  const InstDev* di = reinterpret_cast<const InstDev*>(s + L.inst);
  const TileDev* segs = reinterpret_cast<const TileDev*>(s + L.segs);
  DropDev* dd = reinterpret_cast<DropDev*>(s + L.drops);
  double* part = reinterpret_cast<double*>(s + L.part);
  uint64_t* mask = reinterpret_cast<uint64_t*>(s + L.mask);
  int64_t* dstep = reinterpret_cast<int64_t*>(s + L.step);
  for (int64_t k = 0; k < nsteps; ++k) {
    const int parity = (int)(k & 1);
    hipError_t e = with_types(cf.precision, [&](auto t, auto p) {
      using T = decltype(t);
      return launch_wave<T, decltype(p)>(st, parity, nslots, segs, di, reinterpret_cast<T*>(const_cast<char*>(base)), dd,
                                         part, mask, dstep, nullptr, -1,
                                         cf.walls == LBM_WALLS_NONE && cf.advection == LBM_ADV_PAPER);
    });
    if (e == hipSuccess) e = launch_reduce(st, TILING_FUSED, ndrop, di, dd, part, mask, dstep, 1);
    if (e != hipSuccess) return fail(LBM_E_HIP, std::string("timestep launch: ") + hipGetErrorString(e));
  }
  if (ndrop > 0) {
    hipLaunchKernelGGL(k_noalloc_centres, dim3((ndrop + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), 0, st, dd, ndrop,
                       drops);
    HIPCHK(hipGetLastError());
  }
  return LBM_OK;
}

int lbm_workspace_bytes(int32_t ninst, const lbm_config* cfgs, const int32_t* ndrop, size_t* bytes) {
  if (!bytes) return fail(LBM_E_INVAL, "bytes must not be NULL");
  int rc = validate(ninst, cfgs, ndrop);
  if (rc != LBM_OK) return rc;
  Layout L;
  make_layout(ninst, cfgs, ndrop, L);
  *bytes = L.total;
  return LBM_OK;
}

int lbm_init_batch(int32_t ninst, const lbm_config* cfgs, void* workspace, size_t workspace_bytes, void* stream,
                   const double* phi0, const double* c0, const double* f_pre, const int32_t* ndrop,
                   const lbm_droplet* drops, int64_t step, lbm_ctx** out) {
  if (!out) return fail(LBM_E_INVAL, "out must not be NULL");
  *out = nullptr;
  int rc = validate(ninst, cfgs, ndrop);
  if (rc != LBM_OK) return rc;
  if (!workspace) return fail(LBM_E_INVAL, "workspace must not be NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % ALIGN) return fail(LBM_E_INVAL, "workspace must be 256-byte aligned");
  if (!phi0 || !c0) return fail(LBM_E_INVAL, "phi0 and c0 must not be NULL");
  if (step < 0) return fail(LBM_E_INVAL, "step must be >= 0");
  int nd_total = 0;
  for (int i = 0; i < ninst; ++i) nd_total += ndrop[i];
  if (nd_total > 0 && !drops) return fail(LBM_E_INVAL, "drops must not be NULL when droplets are requested");
  for (int k = 0; k < nd_total; ++k) {
    const lbm_droplet& d = drops[k];
    if (!std::isfinite(d.x) || !std::isfinite(d.y) || !std::isfinite(d.ex) || !std::isfinite(d.ey) ||
        !(d.R >= 0.0) || !(d.Rs >= 0.0))
      return fail(LBM_E_INVAL, "droplet table entries must be finite with R, Rs >= 0");
  }
  std::vector<DropDev> dd(std::max(1, nd_total));
  {
    int k = 0;
    for (int i = 0; i < ninst; ++i)
      for (int j = 0; j < ndrop[i]; ++j, ++k) {
        const lbm_droplet& s = drops[k];
        dd[k] = DropDev{s.x, s.y, s.R, s.Rs, s.ex, s.ey, s.active ? 1 : 0, i};
      }
  }
  lbm_ctx* c = new lbm_ctx();
  make_layout(ninst, cfgs, ndrop, c->L);
  set_segments(c->L, SEG_ROWS_DEFAULT, FUSED_TX, std::vector<DropDev>(dd.begin(), dd.begin() + nd_total));
  if (workspace_bytes < c->L.total) {
    delete c;
    return fail(LBM_E_NOMEM, "workspace smaller than lbm_workspace_bytes()");
  }
  c->cfg.assign(cfgs, cfgs + ninst);
  c->ws = static_cast<char*>(workspace);
  c->stream = static_cast<hipStream_t>(stream);
  c->step = step;
  c->graph_steps = stream ? 20 : 0;

  auto bail = [&](int code) {
    destroy_graphs(c);
    delete c;
    return code;
  };
  size_t off_field = 0;
  for (int i = 0; i < ninst; ++i) {
    const size_t n = (size_t)cfgs[i].nx * cfgs[i].ny;
    rc = with_types(c->L.prec, [&](auto t, auto p) {
      return upload_instance<decltype(t), decltype(p)>(c, i, phi0 + off_field, c0 + off_field,
                                                       f_pre ? f_pre + 9 * off_field : nullptr);
    });
    if (rc != LBM_OK) return bail(rc);
    off_field += n;
  }
  hipError_t e;
#define INIT_CHK(call)                                                                               \
  do {                                                                                               \
    e = (call);                                                                                      \
    if (e != hipSuccess) return bail(fail(LBM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e))); \
  } while (0)
  INIT_CHK(hipMemcpyAsync(c->d_inst(), c->L.inst.data(), sizeof(InstDev) * ninst, hipMemcpyHostToDevice, c->stream));
  INIT_CHK(hipMemcpyAsync(c->d_tiles(), c->L.tiles.data(), sizeof(TileDev) * c->L.tiles.size(), hipMemcpyHostToDevice,
                          c->stream));
  INIT_CHK(hipMemcpyAsync(c->d_segs(), c->L.segs.data(), sizeof(TileDev) * c->L.segs.size(), hipMemcpyHostToDevice,
                          c->stream));
  INIT_CHK(hipMemcpyAsync(c->d_drops(), dd.data(), sizeof(DropDev) * dd.size(), hipMemcpyHostToDevice, c->stream));
  INIT_CHK(hipMemcpyAsync(c->d_step(), &c->step, sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  INIT_CHK(hipMemsetAsync(c->d_mask(), 0, sizeof(uint64_t) * MASK_WORDS * std::max(c->L.ntiles, c->L.max_segs),
                          c->stream));
  // first centre-of-mass pass on phi0, started from the given centres
  INIT_CHK(with_types(c->L.prec, [&](auto t, auto) {
    using T = decltype(t);
    return launch_cm_partials<T>(c->stream, 0, c->nlaunch(), c->d_tiles(), c->d_inst(), reinterpret_cast<T*>(c->pool()),
                                 c->d_drops(), c->d_part(), c->d_mask());
  }));
  INIT_CHK(launch_reduce(c->stream, TILING_SPLIT, c->L.ndrop_total, c->d_inst(), c->d_drops(), c->d_part(),
                         c->d_mask(), c->d_step(), 0));
  INIT_CHK(hipStreamSynchronize(c->stream));
#undef INIT_CHK
  *out = c;
  g_err.clear();
  return LBM_OK;
}

int lbm_init(const lbm_config* cfg, void* workspace, size_t workspace_bytes, void* stream, const double* phi0,
             const double* c0, const double* f_pre, int32_t ndrop, const lbm_droplet* drops, int64_t step,
             lbm_ctx** out) {
  return lbm_init_batch(1, cfg, workspace, workspace_bytes, stream, phi0, c0, f_pre, &ndrop, drops, step, out);
}

int lbm_set_graph(lbm_ctx* c, int32_t steps_per_graph) {
  if (!c) return fail(LBM_E_INVAL, "null context");
  if (steps_per_graph < 0 || (steps_per_graph > 0 && (steps_per_graph % 2 != 0 || steps_per_graph < 2)))
    return fail(LBM_E_INVAL, "steps_per_graph must be 0 or an even number >= 2");
  if (steps_per_graph > 0 && !c->stream) return fail(LBM_E_STATE, "graph replay needs a non-default stream");
  destroy_graphs(c);
  c->graph_steps = steps_per_graph;
  // capture both graphs now (one per starting parity), so that no later lbm_step pays for a capture
  for (int p = 0; p < 2 && steps_per_graph > 0; ++p) {
    const int rc = build_graph(c, p);
    if (rc != LBM_OK) return rc;
  }
  return LBM_OK;
}

int lbm_step(lbm_ctx* c, int64_t n) {
  if (!c) return fail(LBM_E_INVAL, "null context");
  if (n < 0) return fail(LBM_E_INVAL, "n must be >= 0");
  Range range("lbm_step");
  int64_t left = n;
  if (c->graph_steps > 0) {
    while (left >= c->graph_steps) {
      Range replay("lbm_step graph replay");
      if (!c->exec[c->parity]) {
        int rc = build_graph(c, c->parity);
        if (rc != LBM_OK) return rc;
      }
      HIPCHK(hipGraphLaunch(c->exec[c->parity], c->stream));
      left -= c->graph_steps;
      c->step += c->graph_steps;
    }
  }
  for (; left > 0; --left) {
    hipError_t e = enqueue_step_any(c, c->parity);
    if (e != hipSuccess) return fail(LBM_E_HIP, std::string("timestep launch: ") + hipGetErrorString(e));
    c->parity ^= 1;
    c->step += 1;
  }
  return LBM_OK;
}

int lbm_sync(lbm_ctx* c) {
  if (!c) return fail(LBM_E_INVAL, "null context");
  HIPCHK(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

int64_t lbm_get_step(const lbm_ctx* c) { return c ? c->step : -1; }

int lbm_fields(lbm_ctx* c, int32_t inst, double* f_pre, double* phi, double* cc, double* n, double* ux, double* uy) {
  Range range("lbm_fields");
  int rc = check_inst(c, inst);
  if (rc != LBM_OK) return rc;
  HIPCHK(hipStreamSynchronize(c->stream));
  rc = with_types(c->L.prec, [&](auto t, auto p) {
    return fields_impl<decltype(t), decltype(p)>(c, inst, f_pre, phi, cc, n, ux, uy);
  });
  if (rc != LBM_OK) return rc;
  // a non-finite state surfaces here as well as in lbm_observables (the arrays are filled regardless)
  const size_t np = (size_t)c->L.inst[inst].nx * c->L.inst[inst].ny;
  const struct {
    const double* a;
    size_t n;
  } outs[6] = {{f_pre, 9 * np}, {phi, np}, {cc, np}, {n, np}, {ux, np}, {uy, np}};
  for (const auto& o : outs)
    if (o.a)
      for (size_t i = 0; i < o.n; ++i)
        if (!std::isfinite(o.a[i])) return fail(LBM_E_UNSTABLE, "non-finite values in the state");
  return LBM_OK;
}

int lbm_droplets(lbm_ctx* c, int32_t inst, lbm_droplet* out) {
  int rc = check_inst(c, inst);
  if (rc != LBM_OK) return rc;
  if (!out && c->L.inst[inst].ndrop > 0) return fail(LBM_E_INVAL, "out must not be NULL");
  std::vector<DropDev> dd;
  if ((rc = read_drops(c, inst, dd)) != LBM_OK) return rc;
  for (size_t k = 0; k < dd.size(); ++k)
    out[k] = lbm_droplet{dd[k].x, dd[k].y, dd[k].R, dd[k].Rs, dd[k].ex, dd[k].ey, dd[k].active, 0};
  return LBM_OK;
}

int lbm_observables(lbm_ctx* c, int32_t inst, lbm_obs* obs, double* drop_out) {
  Range range("lbm_observables");
  int rc = check_inst(c, inst);
  if (rc != LBM_OK) return rc;
  if (!obs) return fail(LBM_E_INVAL, "obs must not be NULL");
  if ((rc = run_diag(c)) != LBM_OK) return rc;
  hipError_t e = with_types(c->L.prec, [&](auto t, auto p) {
    using T = decltype(t);
    return launch_obs<T, decltype(p)>(c->stream, c->parity, c->nlaunch(), c->d_tiles(), c->d_inst(),
                                      reinterpret_cast<T*>(c->pool()), c->d_drops(), c->d_obs(), c->L.obs_stride);
  });
  if (e != hipSuccess) return fail(LBM_E_HIP, std::string("observables launch: ") + hipGetErrorString(e));
  const InstDev& d = c->L.inst[inst];
  const int nt = d.tiles_x[TILING_SPLIT] * d.tiles_y[TILING_SPLIT], S = c->L.obs_stride;
  std::vector<double> h((size_t)nt * S);
  HIPCHK(hipMemcpyAsync(h.data(), c->d_obs() + (size_t)d.tile_base[TILING_SPLIT] * S, h.size() * sizeof(double),
                        hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  std::vector<DropDev> dd;
  if ((rc = read_drops(c, inst, dd)) != LBM_OK) return rc;
  double m = 0, sp = 0, sc = 0, mb = INFINITY, mu = 0, nf = 0;
  std::vector<double> sw(d.ndrop, 0.0), su(d.ndrop, 0.0), sv(d.ndrop, 0.0);
  for (int t = 0; t < nt; ++t) {
    const double* o = &h[(size_t)t * S];
    m += o[0];
    sp += o[1];
    sc += o[2];
    mb = std::min(mb, o[3]);
    mu = std::max(mu, o[4]);
    nf = std::max(nf, o[5]);
    for (int k = 0; k < d.ndrop; ++k) {
      sw[k] += o[6 + 3 * k];
      su[k] += o[7 + 3 * k];
      sv[k] += o[8 + 3 * k];
    }
  }
  obs->step = c->step;
  obs->mass = m;
  obs->sum_phi = sp;
  obs->sum_c = sc;
  obs->min_B = mb;
  obs->max_u = mu;
  obs->nonfinite = (nf != 0.0 || !std::isfinite(m) || !std::isfinite(sp) || !std::isfinite(sc)) ? 1 : 0;
  obs->ndrop = d.ndrop;
  if (drop_out) {
    for (int k = 0; k < d.ndrop; ++k) {
      drop_out[5 * k + 0] = dd[k].x;
      drop_out[5 * k + 1] = dd[k].y;
      drop_out[5 * k + 2] = sw[k] > 0.0 ? su[k] / sw[k] : 0.0;
      drop_out[5 * k + 3] = sw[k] > 0.0 ? sv[k] / sw[k] : 0.0;
      drop_out[5 * k + 4] = sw[k];
    }
  }
  if (obs->nonfinite) return fail(LBM_E_UNSTABLE, "non-finite values in the state");
  if (!(obs->min_B > 0.0)) return fail(LBM_E_UNSTABLE, "B(c) = B0 + B1 c <= 0 somewhere (interfaces unstable)");
  return LBM_OK;
}

int lbm_debug_stage(lbm_ctx* c, int32_t inst, double* out) {
  int rc = check_inst(c, inst);
  if (rc != LBM_OK) return rc;
  if (!out) return fail(LBM_E_INVAL, "out must not be NULL");
  const InstDev& d = c->L.inst[inst];
  if ((int64_t)d.nx * d.ny > DEBUG_MAX_NODES) return fail(LBM_E_INVAL, "stage export is limited to 512 x 512 nodes");
  hipError_t e = with_types(c->L.prec,
                            [&](auto t, auto p) { return debug_launch<decltype(t), decltype(p)>(c, inst, c->d_dbg()); });
  if (e != hipSuccess) return fail(LBM_E_HIP, std::string("stage launch: ") + hipGetErrorString(e));
  const size_t n = (size_t)d.nx * d.ny;
  HIPCHK(hipMemcpyAsync(out, c->d_dbg(), sizeof(double) * LBM_NSTAGE * n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

int lbm_time_kernels(lbm_ctx* c, int64_t n, double* ms_out) {
  Range range("lbm_time_kernels");
  if (!c || !ms_out) return fail(LBM_E_INVAL, "null argument");
  if (n <= 0) return fail(LBM_E_INVAL, "n must be > 0");
  std::vector<hipEvent_t> ev((size_t)n * 4);
  for (auto& x : ev) HIPCHK(hipEventCreate(&x));
  hipError_t e = hipSuccess;
  int nk = 0;
  for (int64_t s = 0; s < n && e == hipSuccess; ++s)
    e = with_types(c->L.prec,
                   [&](auto t, auto p) { return timed_step<decltype(t), decltype(p)>(c, &ev[(size_t)s * 4], &nk); });
  hipError_t es = hipStreamSynchronize(c->stream);
  double acc[3] = {0, 0, 0};
  if (e == hipSuccess && es == hipSuccess) {
    for (int64_t s = 0; s < n; ++s)
      for (int j = 0; j < nk; ++j) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev[(size_t)s * 4 + j], ev[(size_t)s * 4 + j + 1]);
        acc[j] += ms;
      }
  }
  for (auto& x : ev) (void)hipEventDestroy(x);
  if (e != hipSuccess) return fail(LBM_E_HIP, std::string("timed launch: ") + hipGetErrorString(e));
  if (es != hipSuccess) return fail(LBM_E_HIP, std::string("timed sync: ") + hipGetErrorString(es));
  for (int j = 0; j < 3; ++j) ms_out[j] = acc[j] / (double)n;
  return LBM_OK;
}

int lbm_time_launches(lbm_ctx* c, int32_t launches, double* ms_out) {
  Range range("lbm_time_launches");
  if (!c || !ms_out) return fail(LBM_E_INVAL, "null argument");
  if (launches <= 0) return fail(LBM_E_INVAL, "launches must be > 0");
  if (!c->stream) return fail(LBM_E_STATE, "timing launches in a graph needs a non-default stream");
  ms_out[0] = ms_out[1] = ms_out[2] = 0.0;
  const bool split = c->path == LBM_PATH_SPLIT;
  // kernel k of the path over the current state, writing scratch only; the last one is the centre-of-mass
  // reduction in its mode that writes nothing
  const int nk = split ? 3 : 2;
  auto one = [&](int k) -> hipError_t {
    if (k == nk - 1)
      return launch_reduce(c->stream, split ? TILING_SPLIT : TILING_FUSED, c->L.ndrop_total, c->d_inst(), c->d_drops(),
                           c->d_part(), c->d_mask(), c->d_step(), -1);
    return with_types(c->L.prec, [&](auto t, auto p) -> hipError_t {
      using T = decltype(t);
      using P = decltype(p);
      T* buf = reinterpret_cast<T*>(c->pool());
      if (!split) return launch_sweep<T, P>(c, c->parity, nullptr, -1);
      if (k == 0) return launch_lb<T, P>(c->stream, 0, c->parity, c->nlaunch(), c->d_tiles(), c->d_inst(), buf, nullptr, -1);
      return launch_fd<T>(c->stream, 0, c->parity, c->nlaunch(), c->d_tiles(), c->d_inst(), buf, c->d_drops(),
                          c->d_part(), c->d_mask(), c->d_step(), nullptr, -1);
    });
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int rc = LBM_OK;
  for (int k = 0; k < nk && rc == LBM_OK; ++k) {
    // the launches are replayed from a graph, as lbm_step replays the timestep, so that no host launch gap
    // separates them
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed);
    for (int r = 0; r < launches && e == hipSuccess; ++r) e = one(k);
    const hipError_t ec = hipStreamEndCapture(c->stream, &g);
    if (e == hipSuccess) e = ec;
    if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(x, c->stream);  // warm-up replay
    if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
    if (e == hipSuccess) e = hipGraphLaunch(x, c->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) rc = fail(LBM_E_HIP, std::string("timed launches: ") + hipGetErrorString(e));
    ms_out[k] = (double)ms / launches;
    if (x) (void)hipGraphExecDestroy(x);
    if (g) (void)hipGraphDestroy(g);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

int lbm_set_seg_rows(lbm_ctx* c, int32_t rows) {
  if (!c) return fail(LBM_E_INVAL, "null context");
  if (rows < SEG_ROWS_MIN || rows > SEG_ROWS_MAX)
    return fail(LBM_E_INVAL, "segment height must lie in [" + std::to_string(SEG_ROWS_MIN) + ", " +
                                 std::to_string(SEG_ROWS_MAX) + "]");
  return apply_segments(c, rows, c->L.strip_w);
}

int32_t lbm_get_seg_rows(const lbm_ctx* c) { return c ? c->L.seg_rows : -1; }

int lbm_set_strip_width(lbm_ctx* c, int32_t width) {
  if (!c) return fail(LBM_E_INVAL, "null context");
  if (width < STRIP_W_MIN || width > FUSED_TX)
    return fail(LBM_E_INVAL, "strip width must lie in [" + std::to_string(STRIP_W_MIN) + ", " +
                                 std::to_string(FUSED_TX) + "]");
  return apply_segments(c, c->L.seg_rows, width);
}

int32_t lbm_get_strip_width(const lbm_ctx* c) { return c ? c->L.strip_w : -1; }

const int32_t* lbm_tune_widths(void) { return TUNE_WIDTHS; }

const int32_t* lbm_tune_rows(void) { return TUNE_ROWS; }

int lbm_autotune(lbm_ctx* c, int32_t launches, int32_t both_paths, int32_t* rows_out, int32_t* path_out,
                 double* ms_out) {
  Range range("lbm_autotune");
  if (!c) return fail(LBM_E_INVAL, "null context");
  if (launches <= 0) return fail(LBM_E_INVAL, "launches must be > 0");
  constexpr int NR = LBM_TUNE_NROWS, NW = LBM_TUNE_NWIDTHS;
  if (ms_out)
    for (int k = 0; k < 2 * NW * NR + 1; ++k) ms_out[k] = -1.0;
  if (c->path == LBM_PATH_SPLIT && !both_paths) {
    if (rows_out) *rows_out = c->L.seg_rows;
    if (path_out) *path_out = c->path;
    return LBM_OK;
  }
  const int paths[2] = {LBM_PATH_FUSED, LBM_PATH_WAVE};
  const int start_path = c->path;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int best_rows = c->L.seg_rows, best_path = c->path, best_w = c->L.strip_w;
  double best_ms = 1e300;
  int rc = LBM_OK;
  std::vector<double> cand_ms(2 * NW * NR, 1e300);
  // Heights that give the same number of strip segments as a smaller candidate are skipped.
  std::vector<bool> skip(NR, false);
  {
    std::vector<int64_t> seen;
    for (int k = 0; k < NR; ++k) {
      int64_t nseg = 0;
      for (const auto& d : c->L.inst) nseg += (d.ny + TUNE_ROWS[k] - 1) / TUNE_ROWS[k];
      skip[k] = std::find(seen.begin(), seen.end(), nseg) != seen.end();
      seen.push_back(nseg);
    }
  }
  // Trial launches read the current state and write only the inactive half of every ping-pong buffer
  // and the partials; the parity, the droplet table and the step counter are untouched.  Launches of
  // one candidate run back to back; two passes over the candidates (the first also warms clocks and
  // caches), keeping each candidate's faster pass.
  auto trial = [&](int n) -> hipError_t {
    hipError_t e = hipSuccess;
    for (int rep = 0; rep < n && e == hipSuccess; ++rep)
      e = with_types(c->L.prec,
                     [&](auto t, auto p) { return launch_sweep<decltype(t), decltype(p)>(c, c->parity, nullptr, -1); });
    return e;
  };
  for (int pass = 0; pass < 2 && rc == LBM_OK; ++pass) {
    for (int pi = 0; pi < 2 && rc == LBM_OK; ++pi) {
      if (!both_paths && paths[pi] != start_path) continue;
      c->path = paths[pi];
      for (int wi = 0; wi < NW && rc == LBM_OK; ++wi)
        for (int k = 0; k < NR; ++k) {
          if (skip[k]) continue;
          if ((rc = apply_segments(c, TUNE_ROWS[k], TUNE_WIDTHS[wi])) != LBM_OK) break;
          hipError_t e = trial(1);
          (void)hipEventRecord(e0, c->stream);
          if (e == hipSuccess) e = trial(launches);
          (void)hipEventRecord(e1, c->stream);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          if (e != hipSuccess) {
            rc = fail(LBM_E_HIP, std::string("autotune launch: ") + hipGetErrorString(e));
            break;
          }
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          double& m = cand_ms[(pi * NW + wi) * NR + k];
          m = std::min(m, (double)ms / launches);
        }
    }
  }
  for (int pi = 0; pi < 2; ++pi)
    for (int wi = 0; wi < NW; ++wi)
      for (int k = 0; k < NR; ++k) {
        const double m = cand_ms[(pi * NW + wi) * NR + k];
        if (ms_out && m < 1e299) ms_out[(pi * NW + wi) * NR + k] = m;
        if (m < best_ms) {
          best_ms = m;
          best_rows = TUNE_ROWS[k];
          best_w = TUNE_WIDTHS[wi];
          best_path = paths[pi];
        }
      }
  // the split path (two tile kernels, no strip height) competes with the step time of the sweeping kernels
  if (both_paths && rc == LBM_OK) {
    c->path = LBM_PATH_SPLIT;
    double split_ms = 1e300;
    for (int pass = 0; pass < 2 && rc == LBM_OK; ++pass) {
      hipError_t e = hipSuccess;
      auto one = [&]() {
        return with_types(c->L.prec,
                          [&](auto t, auto p) { return launch_split<decltype(t), decltype(p)>(c, c->parity); });
      };
      e = one();
      (void)hipEventRecord(e0, c->stream);
      for (int rep = 0; rep < launches && e == hipSuccess; ++rep) e = one();
      (void)hipEventRecord(e1, c->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e != hipSuccess) {
        rc = fail(LBM_E_HIP, std::string("autotune launch: ") + hipGetErrorString(e));
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      split_ms = std::min(split_ms, (double)ms / launches);
    }
    if (ms_out && split_ms < 1e299) ms_out[2 * NW * NR] = split_ms;
    if (split_ms < best_ms) {
      best_ms = split_ms;
      best_path = LBM_PATH_SPLIT;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->path = start_path;
  if (rc != LBM_OK) return rc;
  if ((rc = lbm_set_path(c, best_path)) != LBM_OK) return rc;
  if ((rc = apply_segments(c, best_rows, best_w)) != LBM_OK) return rc;
  if (rows_out) *rows_out = best_rows;
  if (path_out) *path_out = best_path;
  return LBM_OK;
}

const char* lbm_kernel_name(int32_t path, int32_t which) {
  static const char* fused[3] = {"k_step", "k_reduce", ""};
  static const char* split[3] = {"k_lb", "k_fd", "k_reduce"};
  static const char* wave[3] = {"k_wave", "k_reduce", ""};
  if (which < 0 || which > 2) return "";
  return path == LBM_PATH_SPLIT ? split[which] : path == LBM_PATH_WAVE ? wave[which] : fused[which];
}

int lbm_set_path(lbm_ctx* c, int32_t path) {
  if (!c) return fail(LBM_E_INVAL, "null context");
  if (path != LBM_PATH_FUSED && path != LBM_PATH_SPLIT && path != LBM_PATH_WAVE)
    return fail(LBM_E_INVAL, "unknown path");
  if (path != c->path) destroy_graphs(c);
  c->path = path;
  return LBM_OK;
}

int32_t lbm_get_path(const lbm_ctx* c) { return c ? c->path : -1; }

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  destroy_graphs(c);
  delete c;
}

const char* lbm_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ------------------------------------------------------------------------------------------------
// Reverse mode: checkpointed forward pass and backward sweep of the adjoint kernels.
namespace {

struct AdjLayout {
  size_t pop = 0, field = 0, dropb = 0;  // bytes of the parts of a saved state
  size_t slot = 0;   // a whole state: populations, phi, c, droplet table, step counter
  size_t sslot = 0;  // what the adjoint step reads of a recomputed state: phi, c, droplet table
  int64_t ncp = 0, nodes = 0;
  int every = 0, nb = 0;
  size_t off_cp = 0, off_seg = 0, off_final = 0, off_fwd = 0, off_adj = 0, off_part = 0, total = 0;
};

constexpr int ADJ_TMP_PLANES = 4;  // intermediate adjoints of one backward step
// The adjoint step reads the first ADJ_FWD_PLANES stage planes of the forward step (mu .. X^{n+1/2}), and the
// recompute exports only those: the record of an interval holds ADJ_FWD_PLANES planes per step.
constexpr int ADJ_FWD_PLANES = ADJ_EXPORT_PLANES;
static_assert(ADJ_FWD_PLANES <= LBM_NSTAGE, "stage planes of the adjoint's forward record");

// Up to five byte ranges (multiples of 8 bytes) copied by one launch.
struct CopyList {
  const uint64_t* src[5];
  uint64_t* dst[5];
  int64_t n[5];  // 8-byte words
  int nseg;
};

__global__ void __launch_bounds__(256) k_copy_list(CopyList L) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int s = 0; s < L.nseg; ++s)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.n[s]; i += stride)
      L.dst[s][i] = L.src[s][i];
}

struct CopyBuilder {
  CopyList L{};
  int64_t most = 0;
  void add(const void* src, void* dst, size_t bytes) {
    L.src[L.nseg] = static_cast<const uint64_t*>(src);
    L.dst[L.nseg] = static_cast<uint64_t*>(dst);
    L.n[L.nseg] = (int64_t)(bytes / 8);
    most = std::max(most, L.n[L.nseg]);
    ++L.nseg;
  }
  hipError_t launch(hipStream_t s) const {
    const int blocks = (int)std::min<int64_t>(std::max<int64_t>((most + 255) / 256, 1), 2048);
    hipLaunchKernelGGL(k_copy_list, dim3(blocks), dim3(256), 0, s, L);
    return hipGetLastError();
  }
};

int adj_check(const lbm_ctx* c, int32_t drop, int64_t nsteps, int32_t every) {
  if (!c) return fail(LBM_E_INVAL, "null context");
  if (c->L.inst.size() != 1) return fail(LBM_E_INVAL, "the adjoint takes a context of one lattice");
  const lbm_config& g = c->cfg[0];
  if (g.precision != LBM_FP64 && g.precision != LBM_FP32)
    return fail(LBM_E_INVAL, "the adjoint runs in LBM_FP64 or LBM_FP32");
  if (g.advection != LBM_ADV_PAPER) return fail(LBM_E_INVAL, "the adjoint is implemented for LBM_ADV_PAPER");
  if (drop < 0 || drop >= c->L.inst[0].ndrop) return fail(LBM_E_INVAL, "droplet index out of range");
  if (nsteps < 1 || every < 1) return fail(LBM_E_INVAL, "nsteps and checkpoint interval must be >= 1");
  return LBM_OK;
}

AdjLayout adj_layout(const lbm_ctx* c, int64_t nsteps, int every) {
  AdjLayout A;
  const InstDev& d = c->L.inst[0];
  A.nodes = (int64_t)d.nx * d.ny;
  A.nb = adj_blocks(d.nx, d.ny);
  A.every = every;
  A.ncp = (nsteps + every - 1) / every;
  A.pop = (size_t)9 * d.pstride * c->L.elem;
  A.field = (size_t)d.pstride * c->L.elem;
  A.dropb = sizeof(DropDev) * (size_t)std::max(1, (int)d.ndrop);
  A.slot = align_up(A.pop + 2 * A.field + A.dropb + sizeof(int64_t), ALIGN);
  A.sslot = align_up(2 * A.field + A.dropb, ALIGN);
  size_t off = 0;
  A.off_cp = off;    off += A.slot * (size_t)A.ncp;
  A.off_seg = off;   off += A.sslot * (size_t)every;
  A.off_final = off; off += A.slot;
  A.off_fwd = off;
  off = align_up(off + sizeof(double) * ADJ_FWD_PLANES * (size_t)every * (size_t)A.nodes, ALIGN);
  A.off_adj = off;   off = align_up(off + c->L.elem * (size_t)(22 + ADJ_TMP_PLANES) * A.nodes, ALIGN);
  A.off_part = off;  off = align_up(off + sizeof(double) * (size_t)A.nb * 2, ALIGN);  // seed sums, dA0 totals
  A.total = off;
  return A;
}

// Copy the state of the single lattice (current buffers, droplet table, step counter) to or from a whole
// slot, in one launch.
int adj_save(lbm_ctx* c, const AdjLayout& A, char* slot) {
  const InstDev& d = c->L.inst[0];
  char* pool = static_cast<char*>(c->pool());
  const size_t e = c->L.elem;
  CopyBuilder b;
  b.add(pool + d.off_f[c->parity] * e, slot, A.pop);
  b.add(pool + d.off_phi[c->parity] * e, slot + A.pop, A.field);
  b.add(pool + d.off_c[c->parity] * e, slot + A.pop + A.field, A.field);
  b.add(c->d_drops(), slot + A.pop + 2 * A.field, sizeof(DropDev) * d.ndrop);
  b.add(c->d_step(), slot + A.pop + 2 * A.field + A.dropb, sizeof(int64_t));
  HIPCHK(b.launch(c->stream));
  return LBM_OK;
}

int adj_load(lbm_ctx* c, const AdjLayout& A, const char* slot, int64_t step) {
  const InstDev& d = c->L.inst[0];
  char* pool = static_cast<char*>(c->pool());
  const size_t e = c->L.elem;
  CopyBuilder b;
  b.add(slot, pool + d.off_f[c->parity] * e, A.pop);
  b.add(slot + A.pop, pool + d.off_phi[c->parity] * e, A.field);
  b.add(slot + A.pop + A.field, pool + d.off_c[c->parity] * e, A.field);
  b.add(slot + A.pop + 2 * A.field, c->d_drops(), sizeof(DropDev) * d.ndrop);
  b.add(slot + A.pop + 2 * A.field + A.dropb, c->d_step(), sizeof(int64_t));
  HIPCHK(b.launch(c->stream));
  c->step = step;
  return LBM_OK;
}

// phi, c and the droplet table of the current state into a segment slot (what the adjoint step reads).
int adj_save_seg(lbm_ctx* c, const AdjLayout& A, char* sslot) {
  const InstDev& d = c->L.inst[0];
  char* pool = static_cast<char*>(c->pool());
  const size_t e = c->L.elem;
  CopyBuilder b;
  b.add(pool + d.off_phi[c->parity] * e, sslot, A.field);
  b.add(pool + d.off_c[c->parity] * e, sslot + A.field, A.field);
  b.add(c->d_drops(), sslot + 2 * A.field, sizeof(DropDev) * d.ndrop);
  HIPCHK(b.launch(c->stream));
  return LBM_OK;
}

const DropDev* adj_seg_drops(const AdjLayout& A, const char* sslot) {
  return reinterpret_cast<const DropDev*>(sslot + 2 * A.field);
}

template <typename T>
int adj_backward(lbm_ctx* c, const AdjLayout& A, char* w, double* dA0, double* dc0) {
  const InstDev& d = c->L.inst[0];
  const lbm_config& g = c->cfg[0];
  const int64_t n0 = c->adj.n0, N = c->adj.nsteps, M = A.nodes;
  const int every = c->adj.every, drop = c->adj.drop, nd = d.ndrop;
  int rc;
  if ((rc = adj_save(c, A, w + A.off_final)) != LBM_OK) return rc;
  // stage planes of step k0 + j of the current interval start ADJ_FWD_PLANES * j planes into the record
  double* fwd = reinterpret_cast<double*>(w + A.off_fwd);
  auto fwd_rec = [&](int64_t j) { return fwd + (size_t)ADJ_FWD_PLANES * (size_t)j * (size_t)M; };
  auto fwd_at = [&](int64_t j) {
    const double* f = fwd_rec(j);
    return AdjFwd{f + 0 * M, f + 1 * M, f + 2 * M, f + 3 * M, f + 4 * M,  f + 5 * M,
                  f + 6 * M, f + 7 * M, f + 8 * M, f + 9 * M, f + 10 * M};
  };
  T* adj = reinterpret_cast<T*>(w + A.off_adj);
  T* lam[2] = {adj, adj + 11 * M};  // adjoint state (f 9 planes, phi, c) at n and at n + 1
  T* tmp = adj + 22 * M;
  double* part = reinterpret_cast<double*>(w + A.off_part);  // seed partial sums (nb)
  double* dA0_part = part + A.nb;                             // per-block dA0 totals over all steps (nb)
  HIPCHK(hipMemsetAsync(dA0_part, 0, sizeof(double) * A.nb, c->stream));
  AdjModel m;
  m.nx = d.nx;
  m.ny = d.ny;
  m.a = g.a;
  m.b = g.b;
  m.B0 = g.B0;
  m.B1 = g.B1;
  m.D = g.D;
  m.Gamma = g.Gamma;
  m.gamma = g.gamma;
  m.omega = d.omega;
  m.coef = d.coef;
  m.yper = d.yper;
  m.walls = d.walls;
  m.ramp = 0.0;
  auto planes = [&](const char* sslot, T* in, T* out) {
    AdjPlanes<T> p;
    p.phi = reinterpret_cast<const T*>(sslot);
    p.c = reinterpret_cast<const T*>(sslot + A.field);
    p.pitch = d.pitch;
    p.fb1 = in;
    p.pb1 = in + 9 * M;
    p.cb1 = in + 10 * M;
    p.fb = out;
    p.pb = out + 9 * M;
    p.cb = out + 10 * M;
    T** t[] = {&p.phb, &p.chb, &p.Fxb, &p.Fyb};
    static_assert(sizeof(t) / sizeof(t[0]) == ADJ_TMP_PLANES, "temporary planes");
    for (int i = 0; i < ADJ_TMP_PLANES; ++i) *t[i] = tmp + (size_t)i * M;
    return p;
  };
  int cur = 1;  // lam[cur] holds the adjoint of the latest state
  bool seeded = false;
  for (int64_t s = A.ncp - 1; s >= 0; --s) {
    const int64_t k0 = s * every, k1 = std::min<int64_t>(N, k0 + every);
    // recompute the interval from its checkpoint, keeping phi, c, the droplet table and the stage planes
    // of every step
    if ((rc = adj_load(c, A, w + A.off_cp + (size_t)s * A.slot, n0 + k0)) != LBM_OK) return rc;
    for (int64_t k = k0; k < k1; ++k) {
      if ((rc = adj_save_seg(c, A, w + A.off_seg + (size_t)(k - k0) * A.sslot)) != LBM_OK) return rc;
      HIPCHK((debug_launch<T, T>(c, 0, fwd_rec(k - k0), false)));
      // the stage-export launch has also written the next state and the centre-of-mass partials, so only
      // the reduction is left of the step
      hipError_t e = launch_reduce(c->stream, c->path == LBM_PATH_SPLIT ? TILING_SPLIT : TILING_FUSED,
                                   c->L.ndrop_total, c->d_inst(), c->d_drops(), c->d_part(), c->d_mask(),
                                   c->d_step(), 1);
      if (e != hipSuccess) return fail(LBM_E_HIP, std::string("adjoint recompute: ") + hipGetErrorString(e));
      c->parity ^= 1;
      c->step += 1;
    }
    if (!seeded) {
      // loss x_CM^N - x_CM^{n0}: seed d/d phi^N over the droplet's nodes (centres of step N - 1)
      const char* last = w + A.off_seg + (size_t)(k1 - 1 - k0) * A.sslot;
      std::vector<DropDev> prev(nd), now(nd);
      HIPCHK(hipMemcpyAsync(prev.data(), adj_seg_drops(A, last), sizeof(DropDev) * nd, hipMemcpyDeviceToHost,
                            c->stream));
      HIPCHK(hipMemcpyAsync(now.data(), c->d_drops(), sizeof(DropDev) * nd, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      double dx = now[drop].x - prev[drop].x;
      if (dx >= 0.5 * d.nx) dx -= d.nx;
      if (dx < -0.5 * d.nx) dx += d.nx;
      const T* phiN = reinterpret_cast<const T*>(c->pool()) + d.off_phi[c->parity];
      HIPCHK(launch_adjoint_seed<T>(c->stream, 0, m, phiN, d.pitch, adj_seg_drops(A, last), nd, drop, 0.0, 1.0,
                                    lam[cur], lam[cur] + 9 * M, lam[cur] + 10 * M, part));
      std::vector<double> hp(A.nb);
      HIPCHK(hipMemcpyAsync(hp.data(), part, sizeof(double) * A.nb, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      double sw = 0.0;
      for (double v : hp) sw += v;
      if (!(sw > 0.0)) return fail(LBM_E_STATE, "the droplet has no nodes with phi >= 0 at the end of the run");
      HIPCHK(launch_adjoint_seed<T>(c->stream, 1, m, phiN, d.pitch, adj_seg_drops(A, last), nd, drop, dx, sw,
                                    lam[cur], lam[cur] + 9 * M, lam[cur] + 10 * M, part));
      seeded = true;
    }
    // backward through the segment, latest step first
    for (int64_t k = k1 - 1; k >= k0; --k) {
      const char* sslot = w + A.off_seg + (size_t)(k - k0) * A.sslot;
      const double tn = (double)(n0 + k);
      m.ramp = tn < g.t_star ? tn : g.t_star;
      const AdjPlanes<T> p = planes(sslot, lam[cur], lam[cur ^ 1]);
      HIPCHK(launch_adjoint_step<T>(c->stream, m, fwd_at(k - k0), p, adj_seg_drops(A, sslot), nd, dA0_part));
      cur ^= 1;
    }
  }
  // results: d/d c^{n0} and the production-rate derivative summed in a fixed order
  if (dc0) {
    std::vector<T> h((size_t)M);
    HIPCHK(hipMemcpyAsync(h.data(), lam[cur] + 10 * M, sizeof(T) * M, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < M; ++i) dc0[i] = (double)h[(size_t)i];
  }
  if (dA0) {
    std::vector<double> hp((size_t)A.nb);
    HIPCHK(hipMemcpyAsync(hp.data(), dA0_part, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    double s = 0.0;
    for (double v : hp) s += v;
    *dA0 = s;
  }
  // back to the state at the end of the forward pass
  if ((rc = adj_load(c, A, w + A.off_final, n0 + N)) != LBM_OK) return rc;
  HIPCHK(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_adjoint_bytes(const lbm_ctx* c, int64_t nsteps, int32_t every, size_t* bytes) {
  if (!c || !bytes) return fail(LBM_E_INVAL, "null argument");
  if (nsteps < 1 || every < 1) return fail(LBM_E_INVAL, "nsteps and checkpoint interval must be >= 1");
  if (c->L.inst.size() != 1) return fail(LBM_E_INVAL, "the adjoint takes a context of one lattice");
  *bytes = adj_layout(c, nsteps, every).total;
  return LBM_OK;
}

int lbm_adjoint_forward(lbm_ctx* c, void* ws, size_t bytes, int32_t drop, int64_t nsteps, int32_t every,
                        double* J) {
  Range range("lbm_adjoint_forward");
  int rc = adj_check(c, drop, nsteps, every);
  if (rc != LBM_OK) return rc;
  if (!ws) return fail(LBM_E_INVAL, "adjoint workspace must not be NULL");
  const AdjLayout A = adj_layout(c, nsteps, every);
  if (bytes < A.total) return fail(LBM_E_NOMEM, "adjoint workspace too small (see lbm_adjoint_bytes)");
  char* w = static_cast<char*>(ws);
  const InstDev& d = c->L.inst[0];
  std::vector<DropDev> dd(d.ndrop);
  HIPCHK(hipMemcpyAsync(dd.data(), c->d_drops(), sizeof(DropDev) * d.ndrop, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  const double x0 = dd[drop].x;
  c->adj.valid = false;
  c->adj.n0 = c->step;
  c->adj.nsteps = nsteps;
  c->adj.every = every;
  c->adj.drop = drop;
  for (int64_t k = 0; k < nsteps; k += every) {
    if ((rc = adj_save(c, A, w + A.off_cp + (size_t)(k / every) * A.slot)) != LBM_OK) return rc;
    if ((rc = lbm_step(c, std::min<int64_t>(every, nsteps - k))) != LBM_OK) return rc;
  }
  HIPCHK(hipMemcpyAsync(dd.data(), c->d_drops(), sizeof(DropDev) * d.ndrop, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  double dx = dd[drop].x - x0;
  if (dx >= 0.5 * d.nx) dx -= d.nx;
  if (dx < -0.5 * d.nx) dx += d.nx;
  if (J) *J = dx;
  c->adj.valid = true;
  return LBM_OK;
}

int lbm_adjoint_backward(lbm_ctx* c, void* ws, size_t bytes, double* dJ_dA0, double* dJ_dc0) {
  Range range("lbm_adjoint_backward");
  if (!c) return fail(LBM_E_INVAL, "null context");
  if (!c->adj.valid) return fail(LBM_E_STATE, "no forward pass recorded (lbm_adjoint_forward)");
  if (c->step != c->adj.n0 + c->adj.nsteps)
    return fail(LBM_E_STATE, "the context has moved since the recorded forward pass");
  if (!ws) return fail(LBM_E_INVAL, "adjoint workspace must not be NULL");
  const AdjLayout A = adj_layout(c, c->adj.nsteps, c->adj.every);
  if (bytes < A.total) return fail(LBM_E_NOMEM, "adjoint workspace too small (see lbm_adjoint_bytes)");
  char* w = static_cast<char*>(ws);
  return c->L.prec == LBM_FP64 ? adj_backward<double>(c, A, w, dJ_dA0, dJ_dc0)
                               : adj_backward<float>(c, A, w, dJ_dA0, dJ_dc0);
}

}  // extern "C"
