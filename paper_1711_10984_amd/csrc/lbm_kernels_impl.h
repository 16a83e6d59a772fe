// HIP kernels (gfx950) of the hybrid lattice-Boltzmann / finite-difference timestep of
// Fadda et al., "Lattice Boltzmann study of chemically-driven self-propelled droplets"
// (EPJ E 2017, arXiv:1711.10984), Sec. 2.
//
// One timestep n -> n+1 is three launches over a list of TILE_X x TILE_Y tiles that may span
// several independent lattices (instances) of different sizes:
//   k_lb     chemical potential mu_phi (Eq. 3), X = (B1/2)|grad phi|^2 (Eq. 5), force F (Eq. 14),
//            pull streaming + moments with half the force (Eqs. 10-11), BGK collision with the
//            equilibrium of Eq. (12) and the forcing of Eq. (13); writes f* and u^n.
//   k_fd     advection half-step (Eqs. 16-17), diffusion of phi (Eq. 18), diffusion, consumption and
//            production of c (Eq. 19); writes phi^{n+1}, c^{n+1} and per-tile centre-of-mass partials.
//   k_reduce fixed-order sum of the partials, new centres of mass (Sec. 4), step counter.
// Populations are stored post-collision (f*_i at the node that emitted them) in structure-of-arrays
// planes [9][ny][pitch]; the next step pulls f_i(r) = f*_i(r - e_i).  Every field has two buffers
// that alternate with the step parity.
//
// Floating-point expressions keep the grouping of the plain definitions (x- and y-reflection
// symmetric sums); the library is compiled without FMA contraction, so the FP64 path is IEEE
// arithmetic in a fixed order.
//
// This header holds the templated kernels; lbm_kernels_f64.hip and lbm_kernels_f32.hip instantiate them
// for one precision each, so that each translation unit gets its own floating-point contraction
// setting (none for FP64, whose arithmetic follows the plain definitions term by term; fused
// multiply-add for FP32).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lbm_internal.h"

namespace lbm {

namespace {

template <typename T>
__device__ __forceinline__ constexpr T cst(double x) {
  return static_cast<T>(x);
}

// Population storage.  P == T: the populations themselves.  P == _Float16 (with T = float): the deviation
// f_i - w_i n0 from the rest state, rounded to FP16 (round to nearest even); wn = w_i n0 in T.
template <typename T, typename P>
__device__ __forceinline__ T pop_ld(P v, T wn) {
  if constexpr (std::is_same<T, P>::value) {
    (void)wn;
    return v;
  } else {
    return T(v) + wn;
  }
}
template <typename P, typename T>
__device__ __forceinline__ P pop_st(T v, T wn) {
  if constexpr (std::is_same<T, P>::value) {
    (void)wn;
    return v;
  } else {
    return P(v - wn);
  }
}

__device__ __forceinline__ int wrap_idx(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

// Periodic wrap of an index that lies within 8 nodes of [0, n): one conditional when n >= 8.
__device__ __forceinline__ int wrap_near(int v, int n) {
  if (n >= 8) return v < 0 ? v + n : (v >= n ? v - n : v);
  return wrap_idx(v, n);
}

// Row read for row index r (within one lattice height of [0, ny)): periodic wrap, or with walls the
// mirror image across the plates at y = -1/2 and y = ny - 1/2 (row -1 reads row 0, row ny reads ny - 1).
__device__ __forceinline__ int row_of(int r, int ny, int walls) {
  if (!walls) return wrap_near(r, ny);
  const int p = 2 * ny;
  int m = r % p;
  if (m < 0) m += p;
  return m < ny ? m : p - 1 - m;
}

__device__ __forceinline__ double minimg(double d, double L) {
  if (d >= 0.5 * L) return d - L;
  if (d < -0.5 * L) return d + L;
  return d;
}

__device__ __forceinline__ double wrapd(double v, double L) {
  if (isinf(L)) return v;  // not periodic (y with walls)
  double r = fmod(v, L);
  if (r < 0.0) r += L;
  if (r >= L) r -= L;
  return r;
}

// Isotropic 9-point gradient sum_i (w_i / cs^2) e_i g(r + e_i) on an LDS tile of row stride W.
template <typename T>
__device__ __forceinline__ void grad9(const T* s, int i, int W, T& gx, T& gy) {
  const T E = s[i + 1], Wv = s[i - 1], N = s[i + W], S = s[i - W];
  const T NE = s[i + W + 1], NW = s[i + W - 1], SW = s[i - W - 1], SE = s[i - W + 1];
  gx = (T(4) * (E - Wv) + ((NE - NW) + (SE - SW))) * cst<T>(1.0 / 12.0);
  gy = (T(4) * (N - S) + ((NE - SE) + (NW - SW))) * cst<T>(1.0 / 12.0);
}

// Isotropic 9-point Laplacian sum_{i>0} (2 w_i / cs^2)(g(r + e_i) - g(r)).
template <typename T>
__device__ __forceinline__ T lap9(const T* s, int i, int W) {
  const T E = s[i + 1], Wv = s[i - 1], N = s[i + W], S = s[i - W];
  const T NE = s[i + W + 1], NW = s[i + W - 1], SW = s[i - W - 1], SE = s[i - W + 1];
  return (T(4) * ((E + Wv) + (N + S)) + ((NE + NW) + (SE + SW)) - T(20) * s[i]) * cst<T>(1.0 / 6.0);
}

// Conservative link divergence of k grad X, sum_{i>0} (2 w_i/cs^2) (k + k_i)/2 (X_i - X), with
// k = D c read from the LDS tile `cs` (stride Wc) and X from the tile `X` (stride WX).
template <typename T>
__device__ __forceinline__ T div9(const T* cs, int ic, int Wc, T D, const T* X, int iX, int WX) {
  const T k0 = D * cs[ic], X0 = X[iX];
  const T t1 = (k0 + D * cs[ic + 1]) * (X[iX + 1] - X0);
  const T t2 = (k0 + D * cs[ic + Wc]) * (X[iX + WX] - X0);
  const T t3 = (k0 + D * cs[ic - 1]) * (X[iX - 1] - X0);
  const T t4 = (k0 + D * cs[ic - Wc]) * (X[iX - WX] - X0);
  const T t5 = (k0 + D * cs[ic + Wc + 1]) * (X[iX + WX + 1] - X0);
  const T t6 = (k0 + D * cs[ic + Wc - 1]) * (X[iX + WX - 1] - X0);
  const T t7 = (k0 + D * cs[ic - Wc - 1]) * (X[iX - WX - 1] - X0);
  const T t8 = (k0 + D * cs[ic - Wc + 1]) * (X[iX - WX + 1] - X0);
  return (T(4) * ((t1 + t3) + (t2 + t4)) + ((t5 + t6) + (t7 + t8))) * cst<T>(1.0 / 12.0);
}

// Advection half-step of Eqs. (16)-(17) for the scalar tile g at index i (stride W), velocity
// tiles ux, uy of the same geometry.  mode 0: centred velocity divergence and first-order upwind
// concentration gradient; mode 1: conservative face-upwind fluxes.
template <typename T>
__device__ __forceinline__ T advect(const T* g, const T* ux, const T* uy, int i, int W, int mode) {
  const T gc = g[i];
  if (mode == 0) {
    const T divu = T(0.5) * (ux[i + 1] - ux[i - 1]) + T(0.5) * (uy[i + W] - uy[i - W]);
    const T u = ux[i], v = uy[i];
    const T dgx = u > T(0) ? gc - g[i - 1] : g[i + 1] - gc;
    const T dgy = v > T(0) ? gc - g[i - W] : g[i + W] - gc;
    return gc - ((gc * divu + u * dgx) + v * dgy);
  }
  const T uxr = T(0.5) * (ux[i] + ux[i + 1]), uxl = T(0.5) * (ux[i - 1] + ux[i]);
  const T uyt = T(0.5) * (uy[i] + uy[i + W]), uyb = T(0.5) * (uy[i - W] + uy[i]);
  const T Fr = uxr * (uxr >= T(0) ? gc : g[i + 1]);
  const T Fl = uxl * (uxl >= T(0) ? g[i - 1] : gc);
  const T Ft = uyt * (uyt >= T(0) ? gc : g[i + W]);
  const T Fb = uyb * (uyb >= T(0) ? g[i - W] : gc);
  return gc - ((Fr - Fl) + (Ft - Fb));
}

// BGK collision of Eq. (10) with the equilibrium of Eq. (12) and the forcing of Eq. (13) for one
// direction e: f* = f - omega (f - feq) + (1 - 1/(2 tau)) w [3 (e - u) + 9 (e.u) e] . F.
// wn = w n, cw = (1 - 1/(2 tau)) w, eu = e.u, eF = e.F, exu = e_x - u_x, eyu = e_y - u_y.
template <typename T>
__device__ __forceinline__ T collide1(T f, T wn, T cw, T eu, T eF, T exu, T eyu, T Fx, T Fy, T usq,
                                      T omega) {
  const T feq = wn * (((T(1) + T(3) * eu) + (T(4.5) * eu) * eu) - T(1.5) * usq);
  const T Fi = cw * (T(3) * (exu * Fx + eyu * Fy) + (T(9) * eu) * eF);
  return (f - omega * (f - feq)) + Fi;
}

// Constants of the lattice-Boltzmann part of a node: weights w_i, (1 - 1/(2 tau)) w_i, 1/tau, the rest
// populations w_i n0 in the arithmetic type, and n0.
template <typename T>
struct LbConst {
  T w0, w1, w5, cw0, cw1, cw5, omega, wr0, wr1, wr5, n0;
};

// Moments of one node (Eq. 11) from its nine stored populations pulled to it (q, in direction order): the
// density n and the velocity u = (sum f_i e_i + F/2) / n.  The node's populations are left in d for lb_collide.
// FP64 stores and takes the populations themselves and groups the sums as the oracle does, so its bits are the
// oracle's.  With FP32 arithmetic those sums would cancel: u ~ 1e-4 is a difference of populations ~ 0.1, and
// FP32 keeps only three of its digits.  FP32 and FP16 storage therefore store and work on the deviations
// d_i = f_i - w_i n0: n = n0 + dn with dn = sum d_i, and n u = sum d_i e_i + F/2, where the rest populations
// have cancelled exactly.
template <typename T, typename P>
__device__ __forceinline__ void lb_moments(const P (&q)[9], const LbConst<T>& k, T Fx, T Fy, T (&d)[9], T& dn,
                                           T& nn, T& ux, T& uy) {
  const T wr[9] = {k.wr0, k.wr1, k.wr1, k.wr1, k.wr1, k.wr5, k.wr5, k.wr5, k.wr5};
  if constexpr (sizeof(T) == 8) {
    for (int i = 0; i < 9; ++i) d[i] = pop_ld<T>(q[i], wr[i]);
    dn = T(0);
    nn = ((d[0] + (d[2] + d[4])) + (d[1] + d[3])) + ((d[5] + d[6]) + (d[7] + d[8]));
  } else {
    for (int i = 0; i < 9; ++i) d[i] = T(q[i]);
    dn = ((d[0] + (d[2] + d[4])) + (d[1] + d[3])) + ((d[5] + d[6]) + (d[7] + d[8]));
    nn = k.n0 + dn;
  }
  const T mx = (d[1] + (d[5] + d[8])) - (d[3] + (d[6] + d[7]));
  const T my = (d[2] + (d[5] + d[6])) - (d[4] + (d[7] + d[8]));
  if constexpr (sizeof(T) == 8) {
    ux = (mx + T(0.5) * Fx) / nn;
    uy = (my + T(0.5) * Fy) / nn;
  } else {  // one division
    const T rn = T(1) / nn;
    ux = (mx + T(0.5) * Fx) * rn;
    uy = (my + T(0.5) * Fy) * rn;
  }
}

// BGK collision with forcing of one node (Eqs. 10, 12, 13) after lb_moments: out receives the values to store,
// s the post-collision populations (for the stage export).  FP64 relaxes and stores the populations as the
// oracle does.  FP32 and FP16 storage relax the deviations and store d* (in FP32, or rounded to FP16); s is then
// d* + w_i n0 summed in double.  Their arithmetic is arranged for fewer instructions, with the same equations:
//   d_eq_i = w_i dn + w_i n p_i,   p_i = (3 + 4.5 e.u) e.u - 1.5 u.u
//   F_i    = 3 (1 - 1/(2 tau)) w_i h_i,   h_i = (e.F - u.F) + 3 (e.u)(e.F)
//   d*_i   = d_i + omega (d_eq_i - d_i) + F_i
// so that each moving direction costs nine operations, and u.u, u.F and the per-weight products are shared.
// A deviation d* in the storage type.  FP16 storage keeps fp16(d*) of the FP32 value d*: the empty asm makes
// d* opaque, so that the compiler cannot fuse the last FMA of d* with the conversion into one mixed-precision
// instruction that rounds only once.
template <typename P>
__device__ __forceinline__ P store_dev(float ds) {
  if constexpr (sizeof(P) == 2) asm("" : "+v"(ds));
  return P(ds);
}

template <typename T, typename P>
__device__ __forceinline__ void lb_collide(const T (&d)[9], T dn, T nn, T ux, T uy, T Fx, T Fy, const LbConst<T>& k,
                                           P (&out)[9], double (&s)[9]) {
  const T usq = ux * ux + uy * uy;
  const T wn0 = k.w0 * nn, wn1 = k.w1 * nn, wn5 = k.w5 * nn;
  if constexpr (sizeof(T) == 8) {
    const T nux = -ux, nuy = -uy, nFx = -Fx, nFy = -Fy;
    const T xp1 = T(1) - ux, xm1 = T(-1) - ux, yp1 = T(1) - uy, ym1 = T(-1) - uy;
    // direction i with w n, (1 - 1/(2 tau)) w, rest population wr, e.u, e.F, e_x - u_x, e_y - u_y
    auto one = [&](int i, T wn, T cw, T wr, T eu, T eF, T exu, T eyu) {
      const T f = collide1(d[i], wn, cw, eu, eF, exu, eyu, Fx, Fy, usq, k.omega);
      s[i] = f;
      out[i] = pop_st<P>(f, wr);
    };
    one(0, wn0, k.cw0, k.wr0, T(0), T(0), nux, nuy);
    one(1, wn1, k.cw1, k.wr1, ux, Fx, xp1, nuy);
    one(2, wn1, k.cw1, k.wr1, uy, Fy, nux, yp1);
    one(3, wn1, k.cw1, k.wr1, nux, nFx, xm1, nuy);
    one(4, wn1, k.cw1, k.wr1, nuy, nFy, nux, ym1);
    one(5, wn5, k.cw5, k.wr5, ux + uy, Fx + Fy, xp1, yp1);
    one(6, wn5, k.cw5, k.wr5, nux + uy, nFx + Fy, xm1, yp1);
    one(7, wn5, k.cw5, k.wr5, nux + nuy, nFx + nFy, xm1, ym1);
    one(8, wn5, k.cw5, k.wr5, ux - uy, Fx - Fy, xp1, ym1);
  } else {
    const T A = T(-1.5) * usq, uF = ux * Fx + uy * Fy;
    const T wd0 = k.w0 * dn, wd1 = k.w1 * dn, wd5 = k.w5 * dn;
    const T k0 = T(3) * k.cw0, k1 = T(3) * k.cw1, k5 = T(3) * k.cw5;
    auto one = [&](int i, T wd, T wn, T kc, T wr, T eu, T eF) {
      const T p = (T(3) + T(4.5) * eu) * eu + A;
      const T deq = wn * p + wd;
      const T h = (T(3) * eu) * eF + (eF - uF);
      T ds = kc * h + (k.omega * (deq - d[i]) + d[i]);
      s[i] = (double)ds + (double)wr;
      out[i] = store_dev<P>(ds);
    };
    {  // rest population: e = 0
      const T deq = wn0 * A + wd0;
      T ds = k0 * (-uF) + (k.omega * (deq - d[0]) + d[0]);
      s[0] = (double)ds + (double)k.wr0;
      out[0] = store_dev<P>(ds);
    }
    one(1, wd1, wn1, k1, k.wr1, ux, Fx);
    one(2, wd1, wn1, k1, k.wr1, uy, Fy);
    one(3, wd1, wn1, k1, k.wr1, -ux, -Fx);
    one(4, wd1, wn1, k1, k.wr1, -uy, -Fy);
    one(5, wd5, wn5, k5, k.wr5, ux + uy, Fx + Fy);
    one(6, wd5, wn5, k5, k.wr5, uy - ux, Fy - Fx);
    one(7, wd5, wn5, k5, k.wr5, -(ux + uy), -(Fx + Fy));
    one(8, wd5, wn5, k5, k.wr5, ux - uy, Fx - Fy);
  }
}

// Sum (or min/max) over the workgroup in a fixed order; every thread receives lane 0's result.
struct OpAdd {
  __device__ double operator()(double a, double b) const { return a + b; }
};
struct OpMin {
  __device__ double operator()(double a, double b) const { return fmin(a, b); }
};
struct OpMax {
  __device__ double operator()(double a, double b) const { return fmax(a, b); }
};

template <class Op>
__device__ double block_reduce(double v, double* sh, Op op) {
  for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double r = sh[0];
  for (int w = 1; w < NTHREADS / 64; ++w) r = op(r, sh[w]);
  __syncthreads();
  return r;
}

// Sum of three values over the workgroup in a fixed order (lane 0's butterfly result per wave, waves
// in order); every thread receives the result.
__device__ __forceinline__ void block_reduce3(double& a, double& b, double& c, double (*red)[3]) {
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
    c += __shfl_xor(c, o, 64);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[wv][0] = a;
    red[wv][1] = b;
    red[wv][2] = c;
  }
  __syncthreads();
  a = red[0][0];
  b = red[0][1];
  c = red[0][2];
  for (int w = 1; w < NTHREADS / 64; ++w) {
    a += red[w][0];
    b += red[w][1];
    c += red[w][2];
  }
  __syncthreads();
}

// Droplet bookkeeping of one tile: candidate lists for the nearest-centre assignment and for the
// production disks, and the deterministic per-tile sums over nodes with phi >= 0 (Sec. 4).
struct DropShared {
  int n_near, n_src;
  int near_list[MAXDROP];
  int src_list[MAXDROP];
  double mind2[MAXDROP];
  unsigned char src_flag[MAXDROP];
  double red[NTHREADS / 64];
  unsigned long long mask[MASK_WORDS];
};

// Conservative culling for the box [bx0, bx1] x [by0, by1]: a droplet is a nearest-centre candidate
// unless its distance to every node of the box exceeds the largest distance of some other droplet's
// centre to the box; a production disk is a candidate if it may reach the box.  Exact decisions are
// taken per node among the candidates, in increasing droplet index.
__device__ void cull_droplets(const InstDev& I, const DropDev* __restrict__ drops, int bx0, int bx1,
                              int by0, int by1, DropShared& sh) {
  const int tid = threadIdx.x;
  const int nd = I.ndrop;
  const double Lx = I.nx, Ly = I.yper;
  const double xm = 0.5 * (bx0 + bx1), ym = 0.5 * (by0 + by1);
  const double hx = 0.5 * (bx1 - bx0), hy = 0.5 * (by1 - by0);
  double my_min_max = 1e300;
  for (int k = tid; k < nd; k += NTHREADS) {
    const DropDev d = drops[I.drop_base + k];
    const double ddx = fabs(minimg(xm - d.x, Lx)), ddy = fabs(minimg(ym - d.y, Ly));
    const double ux = ddx + hx, uy = ddy + hy;
    my_min_max = fmin(my_min_max, ux * ux + uy * uy);
    const double lx = fmax(0.0, ddx - hx), ly = fmax(0.0, ddy - hy);
    sh.mind2[k] = lx * lx + ly * ly;
    unsigned char sf = 0;
    if (d.active) {
      const double px = d.x + (d.R - d.Rs) * d.ex, py = d.y + (d.R - d.Rs) * d.ey;
      const double sdx = fmax(0.0, fabs(minimg(xm - px, Lx)) - hx);
      const double sdy = fmax(0.0, fabs(minimg(ym - py, Ly)) - hy);
      const double rr = d.Rs + 1e-6;
      sf = (sdx * sdx + sdy * sdy <= rr * rr) ? 1 : 0;
    }
    sh.src_flag[k] = sf;
  }
  const double thr = block_reduce(my_min_max, sh.red, OpMin());
  if (tid == 0) {
    int nn = 0, ns = 0;
    const double lim = thr * (1.0 + 1e-12) + 1e-6;
    for (int k = 0; k < nd; ++k) {
      if (sh.mind2[k] <= lim) sh.near_list[nn++] = k;
      if (sh.src_flag[k]) sh.src_list[ns++] = k;
    }
    sh.n_near = nn;
    sh.n_src = ns;
  }
  __syncthreads();
}

// Index of the droplet whose centre is nearest (minimum image) to node (x, y); lowest index on ties.
__device__ __forceinline__ int nearest_drop(const InstDev& I, const DropDev* __restrict__ drops,
                                            const DropShared& sh, double x, double y) {
  int best = -1;
  double bd = 0.0;
  for (int j = 0; j < sh.n_near; ++j) {
    const int k = sh.near_list[j];
    const DropDev d = drops[I.drop_base + k];
    const double dx = minimg(x - d.x, (double)I.nx);
    const double dy = minimg(y - d.y, I.yper);
    const double d2 = dx * dx + dy * dy;
    if (best < 0 || d2 < bd) {
      best = k;
      bd = d2;
    }
  }
  return best;
}

// Number of active production disks |r - r_P| <= Rs containing node (x, y) (Sec. 2.1).
__device__ __forceinline__ int source_count(const InstDev& I, const DropDev* __restrict__ drops,
                                            const DropShared& sh, double x, double y) {
  int cnt = 0;
  for (int j = 0; j < sh.n_src; ++j) {
    const DropDev d = drops[I.drop_base + sh.src_list[j]];
    const double px = d.x + (d.R - d.Rs) * d.ex;
    const double py = d.y + (d.R - d.Rs) * d.ey;
    const double dx = minimg(x - px, (double)I.nx);
    const double dy = minimg(y - py, I.yper);
    if (dx * dx + dy * dy <= d.Rs * d.Rs) ++cnt;
  }
  return cnt;
}

constexpr int NPT = TILE_X * TILE_Y / NTHREADS;  // interior nodes per thread
static_assert(TILE_X * TILE_Y % NTHREADS == 0, "tile must be a multiple of the workgroup");

// Per-tile centre-of-mass sums {phi, phi dx, phi dy} for every droplet present in the tile, written
// as partials[t][k][3] plus a presence mask; kd[j] < 0 marks nodes that contribute nothing.
__device__ void tile_cm_sums(const InstDev& I, int t_local, int t_global, const int* kd, const double* v,
                             const double* vx, const double* vy, DropShared& sh, double* part,
                             uint64_t* mask) {
  const int tid = threadIdx.x;
  if (tid < MASK_WORDS) sh.mask[tid] = 0ull;
  __syncthreads();
  for (int j = 0; j < NPT; ++j)
    if (kd[j] >= 0) atomicOr(&sh.mask[kd[j] >> 6], 1ull << (kd[j] & 63));
  __syncthreads();
  for (int w = 0; w < MASK_WORDS; ++w) {
    unsigned long long m = sh.mask[w];
    while (m) {
      const int bit = __ffsll(m) - 1;
      m &= m - 1;
      const int k = w * 64 + bit;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0;
      for (int j = 0; j < NPT; ++j)
        if (kd[j] == k) {
          a0 += v[j];
          a1 += vx[j];
          a2 += vy[j];
        }
      const double s0 = block_reduce(a0, sh.red, OpAdd());
      const double s1 = block_reduce(a1, sh.red, OpAdd());
      const double s2 = block_reduce(a2, sh.red, OpAdd());
      if (tid == 0) {
        double* p = part + I.part_base[TILING_SPLIT] + ((int64_t)t_local * I.ndrop + k) * 3;
        p[0] = s0;
        p[1] = s1;
        p[2] = s2;
      }
    }
  }
  if (tid < MASK_WORDS) mask[(int64_t)t_global * MASK_WORDS + tid] = sh.mask[tid];
}

// ------------------------------------------------------------------------------------------------
// k_lb: mu, X, F; pull + moments; collision.  MODE 0: step, 1: step + stage planes, 2: n and u only.
// Export launches name their instance in dbg_inst: inst for all LBM_NSTAGE stage planes, -2 - inst for the
// first eleven (mu .. X^{n+1/2}) only, which is what the reverse mode reads.
__device__ __forceinline__ int export_inst(int dbg_inst) { return dbg_inst >= 0 ? dbg_inst : -2 - dbg_inst; }
__device__ __forceinline__ bool export_all(int dbg_inst) { return dbg_inst >= 0; }

template <typename T, typename P, int MODE>
__global__ __launch_bounds__(NTHREADS) void k_lb(int parity, const TileDev* __restrict__ tiles,
                                                 const InstDev* __restrict__ insts, T* __restrict__ buf,
                                                 double* __restrict__ dbg, int dbg_inst) {
  constexpr int TX = TILE_X, TY = TILE_Y;
  constexpr int W2 = TX + 4, H2 = TY + 4, W1 = TX + 2, H1 = TY + 2;
  __shared__ T s_phi[W2 * H2], s_c[W2 * H2], s_mu[W1 * H1], s_X[W1 * H1];
  __shared__ int s_col[W2], s_row[H2];

  const TileDev td = tiles[blockIdx.x];
  if (td.inst < 0) return;
  if (MODE == 1 && td.inst != export_inst(dbg_inst)) return;
  const InstDev& I = insts[td.inst];
  const int nx = I.nx, ny = I.ny, pitch = I.pitch;
  const int tid = threadIdx.x;
  const int64_t plane = I.pstride;
  const T* __restrict__ phi = buf + I.off_phi[parity];
  const T* __restrict__ cc = buf + I.off_c[parity];
  const P* __restrict__ fin = reinterpret_cast<const P*>(buf + I.off_f[parity]);
  P* __restrict__ fout = reinterpret_cast<P*>(buf + I.off_f[parity ^ 1]);
  const T wr0 = T(I.wn[0]), wr1 = T(I.wn[1]), wr5 = T(I.wn[2]);

  for (int i = tid; i < W2; i += NTHREADS) s_col[i] = wrap_idx(td.x0 + i - 2, nx);
  for (int i = tid; i < H2; i += NTHREADS) s_row[i] = row_of(td.y0 + i - 2, ny, I.walls);
  __syncthreads();
  for (int idx = tid; idx < W2 * H2; idx += NTHREADS) {
    const int ly = idx / W2, lx = idx - ly * W2;
    const int64_t g = (int64_t)s_row[ly] * pitch + s_col[lx];
    s_phi[idx] = phi[g];
    s_c[idx] = cc[g];
  }
  __syncthreads();

  // S1-S2: mu_phi (Eq. 3) and X (Eq. 5) on the tile plus a one-node ring
  const T a = T(I.a), b = T(I.b), B0 = T(I.B0), B1 = T(I.B1), halfB1 = T(I.halfB1);
  for (int idx = tid; idx < W1 * H1; idx += NTHREADS) {
    const int ly = idx / W1, lx = idx - ly * W1;
    const int i2 = (ly + 1) * W2 + (lx + 1);
    T gpx, gpy, gcx, gcy;
    grad9(s_phi, i2, W2, gpx, gpy);
    grad9(s_c, i2, W2, gcx, gcy);
    const T lp = lap9(s_phi, i2, W2);
    const T ph = s_phi[i2];
    const T B = B0 + B1 * s_c[i2];
    s_mu[idx] = ((a * ph + b * (ph * ph * ph)) - B * lp) - B1 * (gpx * gcx + gpy * gcy);
    s_X[idx] = halfB1 * (gpx * gpx + gpy * gpy);
  }
  __syncthreads();

  const T omega = T(I.omega), coef = T(I.coef);
  const T w0 = cst<T>(4.0 / 9.0), w1 = cst<T>(1.0 / 9.0), w5 = cst<T>(1.0 / 36.0);
  const T cw0 = coef * w0, cw1 = coef * w1, cw5 = coef * w5;
  const LbConst<T> lbk{w0, w1, w5, cw0, cw1, cw5, omega, wr0, wr1, wr5, T(I.n0)};
  const int64_t nplane = (int64_t)nx * ny;

  for (int idx = tid; idx < TX * TY; idx += NTHREADS) {
    const int ly = idx / TX, lx = idx - ly * TX;
    const int x = td.x0 + lx, y = td.y0 + ly;
    if (x >= nx || y >= ny) continue;
    const int i1 = (ly + 1) * W1 + (lx + 1), i2 = (ly + 2) * W2 + (lx + 2);
    // S3: F = -phi grad mu - grad c - c grad X (Eq. 14)
    T gmx, gmy, gXx, gXy, gcx, gcy;
    grad9(s_mu, i1, W1, gmx, gmy);
    grad9(s_X, i1, W1, gXx, gXy);
    grad9(s_c, i2, W2, gcx, gcy);
    const T ph = s_phi[i2], cv = s_c[i2];
    const T Fx = (-(ph * gmx) - gcx) - cv * gXx;
    const T Fy = (-(ph * gmy) - gcy) - cv * gXy;
    // S4: pull f_i(r) = f*_i(r - e_i), moments with half the force (Eq. 11)
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    const int64_t r0 = (int64_t)y * pitch, rm = (int64_t)ym * pitch, rp = (int64_t)yp * pitch;
    // with walls, the populations that would come from behind a plate are the node's own, bounced back
    const bool bb0 = I.walls && y == 0, bbn = I.walls && y == ny - 1;
    const P q[9] = {fin[r0 + x],
                    fin[plane + r0 + xm],
                    bb0 ? fin[4 * plane + r0 + x] : fin[2 * plane + rm + x],
                    fin[3 * plane + r0 + xp],
                    bbn ? fin[2 * plane + r0 + x] : fin[4 * plane + rp + x],
                    bb0 ? fin[7 * plane + r0 + x] : fin[5 * plane + rm + xm],
                    bb0 ? fin[8 * plane + r0 + x] : fin[6 * plane + rm + xp],
                    bbn ? fin[5 * plane + r0 + x] : fin[7 * plane + rp + xp],
                    bbn ? fin[6 * plane + r0 + x] : fin[8 * plane + rp + xm]};
    T d[9], dn, nn, ux, uy;
    lb_moments<T, P>(q, lbk, Fx, Fy, d, dn, nn, ux, uy);
    const int64_t o = r0 + x;
    if (MODE == 2) {
      buf[I.off_n + o] = nn;
      buf[I.off_ux + o] = ux;
      buf[I.off_uy + o] = uy;
      continue;
    }
    buf[I.off_ux + o] = ux;
    buf[I.off_uy + o] = uy;
    // S5: collision (Eqs. 10, 12, 13)
    P out[9];
    double sv[9];
    lb_collide<T, P>(d, dn, nn, ux, uy, Fx, Fy, lbk, out, sv);
    for (int i = 0; i < 9; ++i) fout[i * plane + o] = out[i];
    if (MODE == 1) {
      const int64_t q = (int64_t)y * nx + x;
      dbg[0 * nplane + q] = (double)s_mu[i1];
      dbg[1 * nplane + q] = (double)s_X[i1];
      dbg[2 * nplane + q] = (double)Fx;
      dbg[3 * nplane + q] = (double)Fy;
      dbg[4 * nplane + q] = (double)nn;
      dbg[5 * nplane + q] = (double)ux;
      dbg[6 * nplane + q] = (double)uy;
      if (export_all(dbg_inst))
        for (int i = 0; i < 9; ++i) dbg[(13 + i) * nplane + q] = sv[i];
    }
  }
}

// ------------------------------------------------------------------------------------------------
// k_fd: advection half-step, phi and c updates, centre-of-mass partials.  MODE 0: step, 1: + stages.
template <typename T, int MODE>
__global__ __launch_bounds__(NTHREADS) void k_fd(int parity, const TileDev* __restrict__ tiles,
                                                 const InstDev* __restrict__ insts, T* __restrict__ buf,
                                                 const DropDev* __restrict__ drops, double* __restrict__ part,
                                                 uint64_t* __restrict__ mask, const int64_t* __restrict__ step,
                                                 double* __restrict__ dbg, int dbg_inst) {
  constexpr int TX = TILE_X, TY = TILE_Y;
  constexpr int W3 = TX + 6, H3 = TY + 6, W2 = TX + 4, H2 = TY + 4, W1 = TX + 2, H1 = TY + 2;
  __shared__ T s_phi[W3 * H3], s_c[W3 * H3], s_ux[W3 * H3], s_uy[W3 * H3];
  __shared__ T s_ph[W2 * H2], s_ch[W2 * H2];
  __shared__ T s_M[W1 * H1], s_Xh[W1 * H1];
  __shared__ int s_col[W3], s_row[H3];
  __shared__ DropShared sh;

  const TileDev td = tiles[blockIdx.x];
  if (td.inst < 0) return;
  if (MODE == 1 && td.inst != export_inst(dbg_inst)) return;
  const InstDev& I = insts[td.inst];
  const int nx = I.nx, ny = I.ny, pitch = I.pitch;
  const int tid = threadIdx.x;
  const T* __restrict__ phi = buf + I.off_phi[parity];
  const T* __restrict__ cc = buf + I.off_c[parity];
  const T* __restrict__ gux = buf + I.off_ux;
  const T* __restrict__ guy = buf + I.off_uy;
  T* __restrict__ phi_out = buf + I.off_phi[parity ^ 1];
  T* __restrict__ c_out = buf + I.off_c[parity ^ 1];

  for (int i = tid; i < W3; i += NTHREADS) s_col[i] = wrap_idx(td.x0 + i - 3, nx);
  for (int i = tid; i < H3; i += NTHREADS) s_row[i] = row_of(td.y0 + i - 3, ny, I.walls);
  __syncthreads();
  for (int idx = tid; idx < W3 * H3; idx += NTHREADS) {
    const int ly = idx / W3, lx = idx - ly * W3;
    const int64_t g = (int64_t)s_row[ly] * pitch + s_col[lx];
    s_phi[idx] = phi[g];
    s_c[idx] = cc[g];
    s_ux[idx] = gux[g];
    // across a plate the ghost velocity is the mirror image with u_y reversed
    const int ry = td.y0 + ly - 3;
    s_uy[idx] = (I.walls && (ry < 0 || ry >= ny)) ? -guy[g] : guy[g];
  }
  __syncthreads();

  // S7: advection half-step with u^n (Eqs. 16-17) on the tile plus two rings
  const int adv = I.advection;
  for (int idx = tid; idx < W2 * H2; idx += NTHREADS) {
    const int ly = idx / W2, lx = idx - ly * W2;
    const int i3 = (ly + 1) * W3 + (lx + 1);
    s_ph[idx] = advect(s_phi, s_ux, s_uy, i3, W3, adv);
    s_ch[idx] = advect(s_c, s_ux, s_uy, i3, W3, adv);
  }
  __syncthreads();

  // S8 bracket M of Eq. (18) and S9 X^{n+1/2} on the tile plus one ring
  const T a = T(I.a), b = T(I.b), B0 = T(I.B0), B1 = T(I.B1), halfB1 = T(I.halfB1);
  for (int idx = tid; idx < W1 * H1; idx += NTHREADS) {
    const int ly = idx / W1, lx = idx - ly * W1;
    const int i2 = (ly + 1) * W2 + (lx + 1), i3 = (ly + 2) * W3 + (lx + 2);
    T gphx, gphy, gchx, gchy;
    grad9(s_ph, i2, W2, gphx, gphy);
    grad9(s_ch, i2, W2, gchx, gchy);
    const T lph = lap9(s_ph, i2, W2);
    const T pn = s_phi[i3];
    const T Bh = B0 + B1 * s_ch[i2];
    s_M[idx] = ((a * s_ph[i2] + b * (pn * pn * pn)) - Bh * lph) - B1 * (gchx * gphx + gchy * gphy);
    s_Xh[idx] = halfB1 * (gphx * gphx + gphy * gphy);
  }
  const int bx1 = min(td.x0 + TX, nx) - 1, by1 = min(td.y0 + TY, ny) - 1;
  if (I.ndrop > 0) {
    cull_droplets(I, drops, td.x0, bx1, td.y0, by1, sh);  // contains barriers
  } else {
    if (tid == 0) sh.n_near = sh.n_src = 0;
    __syncthreads();
  }

  const T Gamma = T(I.Gamma), D = T(I.D), gam = T(I.gamma), c0 = T(I.c0);
  const double tn = (double)(*step);
  const double A = I.A0 * (tn < I.t_star ? tn : I.t_star);
  const int64_t nplane = (int64_t)nx * ny;
  int kd[NPT];
  double vv[NPT], vx[NPT], vy[NPT];
  for (int j = 0; j < NPT; ++j) {
    kd[j] = -1;
    vv[j] = vx[j] = vy[j] = 0.0;
    const int idx = tid + j * NTHREADS;
    const int ly = idx / TX, lx = idx - ly * TX;
    const int x = td.x0 + lx, y = td.y0 + ly;
    if (x >= nx || y >= ny) continue;
    const int i1 = (ly + 1) * W1 + (lx + 1), i2 = (ly + 2) * W2 + (lx + 2);
    // S8: phi^{n+1} = phi^{n+1/2} + Gamma lap M (Eq. 18)
    const T phn = s_ph[i2] + Gamma * lap9(s_M, i1, W1);
    // S9: c^{n+1} (Eq. 19), log-free flux D lap c + div(D c grad X)
    const T ch = s_ch[i2];
    const T lch = lap9(s_ch, i2, W2);
    const T dv = div9(s_ch, i2, W2, D, s_Xh, i1, W1);
    const double src = A * (double)source_count(I, drops, sh, (double)x, (double)y);
    const T cn = (((ch + D * lch) + dv) - gam * (ch - c0)) + T(src);
    const int64_t o = (int64_t)y * pitch + x;
    phi_out[o] = phn;
    c_out[o] = cn;
    // S10 contributions: phi^{n+1} >= 0, nearest previous centre
    const double v = (double)phn;
    if (v >= 0.0 && I.ndrop > 0) {
      const int k = nearest_drop(I, drops, sh, (double)x, (double)y);
      const DropDev d = drops[I.drop_base + k];
      kd[j] = k;
      vv[j] = v;
      vx[j] = v * minimg((double)x - d.x, (double)nx);
      vy[j] = v * minimg((double)y - d.y, I.yper);
    }
    if (MODE == 1) {
      const int64_t q = (int64_t)y * nx + x;
      dbg[7 * nplane + q] = (double)s_ph[i2];
      dbg[8 * nplane + q] = (double)ch;
      dbg[9 * nplane + q] = (double)s_M[i1];
      dbg[10 * nplane + q] = (double)s_Xh[i1];
      if (export_all(dbg_inst)) {
        dbg[11 * nplane + q] = (double)phn;
        dbg[12 * nplane + q] = (double)cn;
      }
    }
  }
  // the stage-export mode writes the partials too: with its state writes (to the inactive half) it is a
  // whole step, which the reverse mode's recompute uses
  if (I.ndrop > 0) tile_cm_sums(I, td.t - I.tile_base[TILING_SPLIT], td.t, kd, vv, vx, vy, sh, part, mask);
}

// Centre-of-mass partials of the current phi (the first pass at initialisation).
template <typename T>
__global__ __launch_bounds__(NTHREADS) void k_cm_partials(int parity, const TileDev* __restrict__ tiles,
                                                          const InstDev* __restrict__ insts,
                                                          const T* __restrict__ buf,
                                                          const DropDev* __restrict__ drops,
                                                          double* __restrict__ part,
                                                          uint64_t* __restrict__ mask) {
  __shared__ DropShared sh;
  const TileDev td = tiles[blockIdx.x];
  if (td.inst < 0) return;
  const InstDev& I = insts[td.inst];
  if (I.ndrop == 0) return;
  const int nx = I.nx, ny = I.ny;
  const int bx1 = min(td.x0 + TILE_X, nx) - 1, by1 = min(td.y0 + TILE_Y, ny) - 1;
  cull_droplets(I, drops, td.x0, bx1, td.y0, by1, sh);
  const T* __restrict__ phi = buf + I.off_phi[parity];
  int kd[NPT];
  double vv[NPT], vx[NPT], vy[NPT];
  for (int j = 0; j < NPT; ++j) {
    kd[j] = -1;
    vv[j] = vx[j] = vy[j] = 0.0;
    const int idx = threadIdx.x + j * NTHREADS;
    const int ly = idx / TILE_X, lx = idx - ly * TILE_X;
    const int x = td.x0 + lx, y = td.y0 + ly;
    if (x >= nx || y >= ny) continue;
    const double v = (double)phi[(int64_t)y * I.pitch + x];
    if (v >= 0.0) {
      const int k = nearest_drop(I, drops, sh, (double)x, (double)y);
      const DropDev d = drops[I.drop_base + k];
      kd[j] = k;
      vv[j] = v;
      vx[j] = v * minimg((double)x - d.x, (double)nx);
      vy[j] = v * minimg((double)y - d.y, I.yper);
    }
  }
  tile_cm_sums(I, td.t - I.tile_base[TILING_SPLIT], td.t, kd, vv, vx, vy, sh, part, mask);
}

// One workgroup per droplet: fixed-order sum of the tile partials of one tiling, new centre of mass
// (Sec. 4), and the step counter.  increment 1: new centres and step + 1; 0: new centres only (the first pass);
// -1: computes the sums and writes nothing (timing).
__global__ __launch_bounds__(NTHREADS) void k_reduce(int tiling, int ndrop_total, const InstDev* __restrict__ insts,
                                                     DropDev* __restrict__ drops,
                                                     const double* __restrict__ part,
                                                     const uint64_t* __restrict__ mask,
                                                     int64_t* __restrict__ step, int increment) {
  __shared__ double red[NTHREADS / 64][3];
  const int g = blockIdx.x;
  if (g == 0 && threadIdx.x == 0 && increment > 0) *step = *step + 1;
  if (g >= ndrop_total) return;
  const DropDev d = drops[g];
  const InstDev& I = insts[d.inst];
  const int k = g - I.drop_base;
  const int ntl = I.tiles_x[tiling] * I.tiles_y[tiling];
  const int64_t tb = I.tile_base[tiling];
  const double* pb = part + I.part_base[tiling];
  // Thread t adds the partials of tiles t, t + NTHREADS, ... in increasing order; the presence bits of UNR
  // of its tiles are loaded together so that their latencies overlap.
  constexpr int UNR = 4;
  const int word = k >> 6;
  const unsigned long long bit = 1ull << (k & 63);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int base = threadIdx.x; base < ntl; base += UNR * NTHREADS) {
    unsigned long long m[UNR];
    for (int u = 0; u < UNR; ++u) {
      const int tl = base + u * NTHREADS;
      m[u] = tl < ntl ? mask[(tb + tl) * MASK_WORDS + word] : 0ull;
    }
    for (int u = 0; u < UNR; ++u)
      if (m[u] & bit) {
        const double* p = pb + ((int64_t)(base + u * NTHREADS) * I.ndrop + k) * 3;
        a0 += p[0];
        a1 += p[1];
        a2 += p[2];
      }
  }
  block_reduce3(a0, a1, a2, red);
  if (threadIdx.x == 0 && a0 > 0.0 && increment >= 0) {
    drops[g].x = wrapd(d.x + a1 / a0, (double)I.nx);
    drops[g].y = wrapd(d.y + a2 / a0, I.yper);
  }
}

// Observables of the current state from the n, u planes written by k_lb<MODE 2>:
// per-tile {mass, sum phi, sum c, min B, max |u|, nonfinite, per droplet (phi, phi ux, phi uy)}.
template <typename T, typename P>
__global__ __launch_bounds__(NTHREADS) void k_obs(int parity, const TileDev* __restrict__ tiles,
                                                  const InstDev* __restrict__ insts, const T* __restrict__ buf,
                                                  const DropDev* __restrict__ drops,
                                                  double* __restrict__ out, int stride) {
  __shared__ DropShared sh;
  const TileDev td = tiles[blockIdx.x];
  if (td.inst < 0) return;
  const InstDev& I = insts[td.inst];
  const int nx = I.nx, ny = I.ny, pitch = I.pitch;
  const int64_t plane = I.pstride;
  const int bx1 = min(td.x0 + TILE_X, nx) - 1, by1 = min(td.y0 + TILE_Y, ny) - 1;
  if (I.ndrop > 0) {
    cull_droplets(I, drops, td.x0, bx1, td.y0, by1, sh);
  } else {
    if (threadIdx.x == 0) sh.n_near = sh.n_src = 0;
    __syncthreads();
  }
  const T* __restrict__ phi = buf + I.off_phi[parity];
  const T* __restrict__ cc = buf + I.off_c[parity];
  const P* __restrict__ fst = reinterpret_cast<const P*>(buf + I.off_f[parity]);
  double m = 0.0, sp = 0.0, sc = 0.0, mb = 1e300, mu = 0.0, nf = 0.0;
  int kd[NPT];
  double vv[NPT], vx[NPT], vy[NPT];
  for (int j = 0; j < NPT; ++j) {
    kd[j] = -1;
    vv[j] = vx[j] = vy[j] = 0.0;
    const int idx = threadIdx.x + j * NTHREADS;
    const int ly = idx / TILE_X, lx = idx - ly * TILE_X;
    const int x = td.x0 + lx, y = td.y0 + ly;
    if (x >= nx || y >= ny) continue;
    const int64_t o = (int64_t)y * pitch + x;
    const double p = (double)phi[o], c = (double)cc[o];
    const double n = (double)buf[I.off_n + o];
    const double u = (double)buf[I.off_ux + o], v = (double)buf[I.off_uy + o];
    m += n;
    sp += p;
    sc += c;
    mb = fmin(mb, I.B0 + I.B1 * c);
    mu = fmax(mu, sqrt(u * u + v * v));
    bool fin = isfinite(p) && isfinite(c);
    for (int i = 0; i < 9; ++i) fin = fin && isfinite((double)fst[i * plane + o]);
    if (!fin) nf = 1.0;
    if (p >= 0.0 && I.ndrop > 0) {
      const int k = nearest_drop(I, drops, sh, (double)x, (double)y);
      kd[j] = k;
      vv[j] = p;
      vx[j] = p * u;
      vy[j] = p * v;
    }
  }
  double* o = out + (int64_t)td.t * stride;
  const double r0 = block_reduce(m, sh.red, OpAdd());
  const double r1 = block_reduce(sp, sh.red, OpAdd());
  const double r2 = block_reduce(sc, sh.red, OpAdd());
  const double r3 = block_reduce(mb, sh.red, OpMin());
  const double r4 = block_reduce(mu, sh.red, OpMax());
  const double r5 = block_reduce(nf, sh.red, OpMax());
  if (threadIdx.x == 0) {
    o[0] = r0;
    o[1] = r1;
    o[2] = r2;
    o[3] = r3;
    o[4] = r4;
    o[5] = r5;
  }
  for (int k = 0; k < I.ndrop; ++k) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int j = 0; j < NPT; ++j)
      if (kd[j] == k) {
        a0 += vv[j];
        a1 += vx[j];
        a2 += vy[j];
      }
    const double s0 = block_reduce(a0, sh.red, OpAdd());
    const double s1 = block_reduce(a1, sh.red, OpAdd());
    const double s2 = block_reduce(a2, sh.red, OpAdd());
    if (threadIdx.x == 0) {
      o[6 + 3 * k] = s0;
      o[7 + 3 * k] = s1;
      o[8 + 3 * k] = s2;
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Fused timestep.  A workgroup owns the strip [x0, x0 + FUSED_TX) x [y0, y0 + seg_rows) of one
// instance and sweeps it in y.  Lane l of every wavefront handles column x0 + l - 5 (periodic), so a
// row of 64 lanes covers the strip plus 5 halo columns on each side.  The six stages of the step are
// skewed by one row and keep their recent rows in 8-row LDS rings:
//   s0  phi^n, c^n                                   (global loads, prefetched one sweep ahead)
//   s1  mu_phi (Eq. 3), X = (B1/2)|grad phi|^2 (Eq. 5)
//   s2  F (Eq. 14), pulled f, n, u^n (Eq. 11); on owned nodes BGK + forcing (Eqs. 10, 12, 13) -> f*
//   s3  phi^{n+1/2}, c^{n+1/2} (Eqs. 16-17)
//   s4  M, the bracket of Eq. (18), and X^{n+1/2}
//   s5  phi^{n+1} (Eq. 18), c^{n+1} (Eq. 19) on owned nodes; centre-of-mass contributions (Sec. 4)
// Each sweep iteration advances every stage by FUSED_R rows (one wavefront per row).  Stage s needs rows
// r-1..r+1 of stage s-1, which the one-row skew provides without recomputing any row in y; only the
// 5 halo columns per side are computed twice (by both neighbouring strips).
// Nearest-centre candidates of a segment whose centre-of-mass sums the sweeping kernels accumulate per lane
// (or per thread) across rows; further candidates (rare) are reduced row by row.
constexpr int CM_SLOTS = 4;
constexpr int RING = 8;

struct FusedShared {
  unsigned long long near_mask[MASK_WORDS], src_mask[MASK_WORDS], seg_mask[MASK_WORDS], it_mask[MASK_WORDS];
  double red[NTHREADS / 64][3];
  // centre-of-mass sums of the segment's first nearest-centre candidate, per thread across iterations
  double slot[3][NTHREADS];
};

// 9-point stencils on three LDS rows: up = row r+1 (N), mid = row r, dn = row r-1 (S); lane l.
template <typename T>
__device__ __forceinline__ void grad9r(const T* up, const T* mid, const T* dn, int l, T& gx, T& gy) {
  const T E = mid[l + 1], Wv = mid[l - 1], N = up[l], S = dn[l];
  const T NE = up[l + 1], NW = up[l - 1], SW = dn[l - 1], SE = dn[l + 1];
  gx = (T(4) * (E - Wv) + ((NE - NW) + (SE - SW))) * cst<T>(1.0 / 12.0);
  gy = (T(4) * (N - S) + ((NE - SE) + (NW - SW))) * cst<T>(1.0 / 12.0);
}

template <typename T>
__device__ __forceinline__ T lap9r(const T* up, const T* mid, const T* dn, int l) {
  const T E = mid[l + 1], Wv = mid[l - 1], N = up[l], S = dn[l];
  const T NE = up[l + 1], NW = up[l - 1], SW = dn[l - 1], SE = dn[l + 1];
  return (T(4) * ((E + Wv) + (N + S)) + ((NE + NW) + (SE + SW)) - T(20) * mid[l]) * cst<T>(1.0 / 6.0);
}

template <typename T>
__device__ __forceinline__ T div9r(const T* cu, const T* cm, const T* cd, T D, const T* Xu, const T* Xm,
                                   const T* Xd, int l) {
  const T k0 = D * cm[l], X0 = Xm[l];
  const T t1 = (k0 + D * cm[l + 1]) * (Xm[l + 1] - X0);
  const T t2 = (k0 + D * cu[l]) * (Xu[l] - X0);
  const T t3 = (k0 + D * cm[l - 1]) * (Xm[l - 1] - X0);
  const T t4 = (k0 + D * cd[l]) * (Xd[l] - X0);
  const T t5 = (k0 + D * cu[l + 1]) * (Xu[l + 1] - X0);
  const T t6 = (k0 + D * cu[l - 1]) * (Xu[l - 1] - X0);
  const T t7 = (k0 + D * cd[l - 1]) * (Xd[l - 1] - X0);
  const T t8 = (k0 + D * cd[l + 1]) * (Xd[l + 1] - X0);
  return (T(4) * ((t1 + t3) + (t2 + t4)) + ((t5 + t6) + (t7 + t8))) * cst<T>(1.0 / 12.0);
}

// Advection half-step of Eqs. (16)-(17) at one lane: scalar g (centre, east, west, north, south),
// velocity x-component at the centre and its east/west neighbours, y-component at the centre and its
// north/south neighbours.
template <typename T>
__device__ __forceinline__ T advect_n(T gc, T ge, T gw, T gn, T gs, T uc, T ue, T uw, T vc, T vn, T vs, int mode) {
  if (mode == 0) {
    const T divu = T(0.5) * (ue - uw) + T(0.5) * (vn - vs);
    const T dgx = uc > T(0) ? gc - gw : ge - gc;
    const T dgy = vc > T(0) ? gc - gs : gn - gc;
    return gc - ((gc * divu + uc * dgx) + vc * dgy);
  }
  const T uxr = T(0.5) * (uc + ue), uxl = T(0.5) * (uw + uc);
  const T uyt = T(0.5) * (vc + vn), uyb = T(0.5) * (vs + vc);
  const T Fr = uxr * (uxr >= T(0) ? gc : ge);
  const T Fl = uxl * (uxl >= T(0) ? gw : gc);
  const T Ft = uyt * (uyt >= T(0) ? gc : gn);
  const T Fb = uyb * (uyb >= T(0) ? gs : gc);
  return gc - ((Fr - Fl) + (Ft - Fb));
}

// DBG: also export the stage planes of instance dbg_inst (the other instances are skipped).  The state writes and
// the centre-of-mass partials are those of a step either way: they go to the inactive half, so an export leaves
// the state as it was, and followed by the reduction it is a whole step (the reverse mode's recompute).
template <typename T, typename P, bool DBG>
__global__ __launch_bounds__(NTHREADS) void k_step(int parity, const TileDev* __restrict__ segs,
                                                   const InstDev* __restrict__ insts, T* __restrict__ buf,
                                                   const DropDev* __restrict__ drops, double* __restrict__ part,
                                                   uint64_t* __restrict__ mask, const int64_t* __restrict__ step,
                                                   double* __restrict__ dbg, int dbg_inst) {
  constexpr int L = FUSED_LANES;
  __shared__ T r_phi[RING][L], r_c[RING][L], r_mu[RING][L], r_X[RING][L], r_ux[RING][L], r_uy[RING][L];
  __shared__ T r_ph[RING][L], r_ch[RING][L], r_M[RING][L], r_Xh[RING][L];
  __shared__ FusedShared sh;

  const TileDev sd = segs[blockIdx.x];
  if (sd.inst < 0) return;
  if (DBG && sd.inst != export_inst(dbg_inst)) return;
  const InstDev& I = insts[sd.inst];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nx = I.nx, ny = I.ny, pitch = I.pitch, nd = I.ndrop;
  const int x0 = sd.x0, y0 = sd.y0;
  const int yend = min(y0 + I.seg_rows, ny);
  const int xend = min(x0 + I.strip_w, nx);
  const int col = lane - 5;                   // column offset of this lane
  const int gx = wrap_idx(x0 + col, nx);      // periodic global column
  const int gxm = gx == 0 ? nx - 1 : gx - 1, gxp = gx == nx - 1 ? 0 : gx + 1;
  const bool own_col = col >= 0 && col < I.strip_w && x0 + col < nx;
  const int64_t plane = I.pstride;
  const T* __restrict__ phi_in = buf + I.off_phi[parity];
  const T* __restrict__ c_in = buf + I.off_c[parity];
  const P* __restrict__ fin = reinterpret_cast<const P*>(buf + I.off_f[parity]);
  P* __restrict__ fout = reinterpret_cast<P*>(buf + I.off_f[parity ^ 1]);
  const T wr0 = T(I.wn[0]), wr1 = T(I.wn[1]), wr5 = T(I.wn[2]);
  T* __restrict__ phi_out = buf + I.off_phi[parity ^ 1];
  T* __restrict__ c_out = buf + I.off_c[parity ^ 1];
  const int64_t nplane = (int64_t)nx * ny;

  // --- droplet culling for the owned box [x0, xend) x [y0, yend); thread k handles droplet k
  if (nd > 0) {
    const double Lx = nx, Ly = I.yper;
    const double xm = 0.5 * (x0 + xend - 1), ym = 0.5 * (y0 + yend - 1);
    const double hx = 0.5 * (xend - 1 - x0), hy = 0.5 * (yend - 1 - y0);
    double maxd2 = 1e300, mind2 = 1e300;
    bool srcf = false;
    if (tid < nd) {
      const DropDev d = drops[I.drop_base + tid];
      const double ddx = fabs(minimg(xm - d.x, Lx)), ddy = fabs(minimg(ym - d.y, Ly));
      const double ux = ddx + hx, uy = ddy + hy;
      maxd2 = ux * ux + uy * uy;
      const double lx = fmax(0.0, ddx - hx), ly = fmax(0.0, ddy - hy);
      mind2 = lx * lx + ly * ly;
      if (d.active) {
        const double px = d.x + (d.R - d.Rs) * d.ex, py = d.y + (d.R - d.Rs) * d.ey;
        const double sdx = fmax(0.0, fabs(minimg(xm - px, Lx)) - hx);
        const double sdy = fmax(0.0, fabs(minimg(ym - py, Ly)) - hy);
        const double rr = d.Rs + 1e-6;
        srcf = sdx * sdx + sdy * sdy <= rr * rr;
      }
    }
    double thr = maxd2;
    for (int o = 32; o > 0; o >>= 1) thr = fmin(thr, __shfl_xor(thr, o, 64));
    if (lane == 0) sh.red[wv][0] = thr;
    __syncthreads();
    thr = fmin(fmin(sh.red[0][0], sh.red[1][0]), fmin(sh.red[2][0], sh.red[3][0]));
    const double lim = thr * (1.0 + 1e-12) + 1e-6;
    const unsigned long long nb = __ballot(tid < nd && mind2 <= lim);
    const unsigned long long sb = __ballot(srcf);
    if (lane == 0) {
      sh.near_mask[wv] = nb;
      sh.src_mask[wv] = sb;
      sh.seg_mask[wv] = 0ull;
    }
    __syncthreads();
  }
  // the first candidate (lowest droplet index) owns the per-thread slot; ncand candidates in all
  int cand0 = -1, ncand = 0;
  if (nd > 0) {
    for (int w = MASK_WORDS - 1; w >= 0; --w) {
      const unsigned long long m = sh.near_mask[w];
      if (m) cand0 = w * 64 + __ffsll(m) - 1;
      ncand += __popcll(m);
    }
    cand0 = __builtin_amdgcn_readfirstlane(cand0);
    ncand = __builtin_amdgcn_readfirstlane(ncand);
  }
  sh.slot[0][tid] = sh.slot[1][tid] = sh.slot[2][tid] = 0.0;
  bool met0 = false;
  const int t_local = sd.t - I.tile_base[TILING_FUSED];
  double* const part_t = part + I.part_base[TILING_FUSED] + (int64_t)t_local * nd * 3;
  const double tn = (double)(*step);
  const double A = I.A0 * (tn < I.t_star ? tn : I.t_star);

  const T a = T(I.a), b = T(I.b), B0 = T(I.B0), B1 = T(I.B1), halfB1 = T(I.halfB1);
  const T omega = T(I.omega), coef = T(I.coef);
  const T w0 = cst<T>(4.0 / 9.0), w1 = cst<T>(1.0 / 9.0), w5 = cst<T>(1.0 / 36.0);
  const T cw0 = coef * w0, cw1 = coef * w1, cw5 = coef * w5;
  const LbConst<T> lbk{w0, w1, w5, cw0, cw1, cw5, omega, wr0, wr1, wr5, T(I.n0)};
  const T Gamma = T(I.Gamma), D = T(I.D), gam = T(I.gamma), c0 = T(I.c0);
  const int adv = I.advection;

  // stage row validity windows: stage s computes rows [y0 - (5 - s), yend + (5 - s))
  const bool l1 = lane >= 1 && lane < L - 1, l2 = lane >= 2 && lane < L - 2, l3 = lane >= 3 && lane < L - 3;
  const bool l4 = lane >= 4 && lane < L - 4;
  const int H = yend - y0;
  const int nit = (H + 6 + FUSED_R - 1) / FUSED_R + 1;

  // prefetch registers: phi, c of the stage-0 row and the pulled populations of the stage-2 row
  T pf_phi = T(0), pf_c = T(0);
  P pf[9];
  for (int i = 0; i < 9; ++i) pf[i] = P(0);
  const int walls = I.walls;
  auto load_s0 = [&](int it) {
    const int r = y0 - 5 + it * FUSED_R + wv;
    if (r < yend + 5) {
      const int gy = row_of(r, ny, walls);
      const int64_t o = (int64_t)gy * pitch + gx;
      pf_phi = phi_in[o];
      pf_c = c_in[o];
    }
  };
  auto load_s2 = [&](int it) {
    const int r = y0 - 5 + it * FUSED_R + wv - 2;
    if (l2 && r >= y0 - 3 && r < yend + 3) {
      const int gy = row_of(r, ny, walls), gym = row_of(r - 1, ny, walls), gyp = row_of(r + 1, ny, walls);
      const int64_t r0 = (int64_t)gy * pitch, rm = (int64_t)gym * pitch, rp = (int64_t)gyp * pitch;
      // behind a plate: the node's own opposite population (halfway bounce-back)
      const bool bb0 = walls && r == 0, bbn = walls && r == ny - 1;
      pf[0] = fin[r0 + gx];
      pf[1] = fin[plane + r0 + gxm];
      pf[2] = bb0 ? fin[4 * plane + r0 + gx] : fin[2 * plane + rm + gx];
      pf[3] = fin[3 * plane + r0 + gxp];
      pf[4] = bbn ? fin[2 * plane + r0 + gx] : fin[4 * plane + rp + gx];
      pf[5] = bb0 ? fin[7 * plane + r0 + gx] : fin[5 * plane + rm + gxm];
      pf[6] = bb0 ? fin[8 * plane + r0 + gx] : fin[6 * plane + rm + gxp];
      pf[7] = bbn ? fin[5 * plane + r0 + gx] : fin[7 * plane + rp + gxp];
      pf[8] = bbn ? fin[6 * plane + r0 + gx] : fin[8 * plane + rp + gxm];
    }
  };
  load_s0(0);
  load_s2(0);

  for (int it = 0; it < nit; ++it) {
    const int q0 = y0 - 5 + it * FUSED_R;
    // ---- s0: store phi^n, c^n of row q0 + wv, then prefetch the next sweep's row
    {
      const int r = q0 + wv;
      if (r < yend + 5) {
        r_phi[r & (RING - 1)][lane] = pf_phi;
        r_c[r & (RING - 1)][lane] = pf_c;
      }
      load_s0(it + 1);
    }
    __syncthreads();
    // ---- s1: mu_phi and X (Eqs. 3, 5)
    {
      const int r = q0 - 1 + wv;
      if (l1 && r >= y0 - 4 && r < yend + 4) {
        const int su = (r + 1) & (RING - 1), sm = r & (RING - 1), sdn = (r - 1) & (RING - 1);
        T gpx, gpy, gcx, gcy;
        grad9r(r_phi[su], r_phi[sm], r_phi[sdn], lane, gpx, gpy);
        grad9r(r_c[su], r_c[sm], r_c[sdn], lane, gcx, gcy);
        const T lp = lap9r(r_phi[su], r_phi[sm], r_phi[sdn], lane);
        const T ph = r_phi[sm][lane];
        const T B = B0 + B1 * r_c[sm][lane];
        const T mu = ((a * ph + b * (ph * ph * ph)) - B * lp) - B1 * (gpx * gcx + gpy * gcy);
        const T X = halfB1 * (gpx * gpx + gpy * gpy);
        r_mu[sm][lane] = mu;
        r_X[sm][lane] = X;
        if (DBG && own_col && r >= y0 && r < yend) {
          const int64_t q = (int64_t)r * nx + (x0 + col);
          dbg[0 * nplane + q] = (double)mu;
          dbg[1 * nplane + q] = (double)X;
        }
      }
    }
    __syncthreads();
    // ---- s2: force, moments, collision
    {
      const int r = q0 - 2 + wv;
      if (l2 && r >= y0 - 3 && r < yend + 3) {
        const int su = (r + 1) & (RING - 1), sm = r & (RING - 1), sdn = (r - 1) & (RING - 1);
        T gmx, gmy, gXx, gXy, gcx, gcy;
        grad9r(r_mu[su], r_mu[sm], r_mu[sdn], lane, gmx, gmy);
        grad9r(r_X[su], r_X[sm], r_X[sdn], lane, gXx, gXy);
        grad9r(r_c[su], r_c[sm], r_c[sdn], lane, gcx, gcy);
        const T ph = r_phi[sm][lane], cv = r_c[sm][lane];
        const T Fx = (-(ph * gmx) - gcx) - cv * gXx;
        const T Fy = (-(ph * gmy) - gcy) - cv * gXy;
        T d[9], dn, nn, ux, uy;
        lb_moments<T, P>(pf, lbk, Fx, Fy, d, dn, nn, ux, uy);
        r_ux[sm][lane] = ux;
        r_uy[sm][lane] = uy;
        if (own_col && r >= y0 && r < yend) {
          P out[9];
          double sv[9];
          lb_collide<T, P>(d, dn, nn, ux, uy, Fx, Fy, lbk, out, sv);
          const int64_t o = (int64_t)r * pitch + gx;
          for (int i = 0; i < 9; ++i) fout[i * plane + o] = out[i];
          if (DBG) {
            const int64_t q = (int64_t)r * nx + (x0 + col);
            dbg[2 * nplane + q] = (double)Fx;
            dbg[3 * nplane + q] = (double)Fy;
            dbg[4 * nplane + q] = (double)nn;
            dbg[5 * nplane + q] = (double)ux;
            dbg[6 * nplane + q] = (double)uy;
            if (export_all(dbg_inst))
              for (int i = 0; i < 9; ++i) dbg[(13 + i) * nplane + q] = sv[i];
          }
        }
      }
      load_s2(it + 1);
    }
    __syncthreads();
    // ---- s3: advection half-step (Eqs. 16-17)
    {
      const int r = q0 - 3 + wv;
      if (l3 && r >= y0 - 2 && r < yend + 2) {
        const int su = (r + 1) & (RING - 1), sm = r & (RING - 1), sdn = (r - 1) & (RING - 1);
        // u^n beyond a plate is not computed: its mirror image with u_y reversed
        const T uc = r_ux[sm][lane], ue = r_ux[sm][lane + 1], uw = r_ux[sm][lane - 1], vc = r_uy[sm][lane];
        const T vn = (walls && r == ny - 1) ? -vc : r_uy[su][lane];
        const T vs = (walls && r == 0) ? -vc : r_uy[sdn][lane];
        const T ph = advect_n(r_phi[sm][lane], r_phi[sm][lane + 1], r_phi[sm][lane - 1], r_phi[su][lane],
                              r_phi[sdn][lane], uc, ue, uw, vc, vn, vs, adv);
        const T ch = advect_n(r_c[sm][lane], r_c[sm][lane + 1], r_c[sm][lane - 1], r_c[su][lane], r_c[sdn][lane], uc,
                              ue, uw, vc, vn, vs, adv);
        r_ph[sm][lane] = ph;
        r_ch[sm][lane] = ch;
        if (DBG && own_col && r >= y0 && r < yend) {
          const int64_t q = (int64_t)r * nx + (x0 + col);
          dbg[7 * nplane + q] = (double)ph;
          dbg[8 * nplane + q] = (double)ch;
        }
      }
    }
    __syncthreads();
    // ---- s4: bracket M of Eq. (18) and X^{n+1/2}
    {
      const int r = q0 - 4 + wv;
      if (l4 && r >= y0 - 1 && r < yend + 1) {
        // half-step fields beyond a plate: the mirror image of the boundary row
        const int sm = r & (RING - 1);
        const int su = (walls && r == ny - 1) ? sm : (r + 1) & (RING - 1);
        const int sdn = (walls && r == 0) ? sm : (r - 1) & (RING - 1);
        T gphx, gphy, gchx, gchy;
        grad9r(r_ph[su], r_ph[sm], r_ph[sdn], lane, gphx, gphy);
        grad9r(r_ch[su], r_ch[sm], r_ch[sdn], lane, gchx, gchy);
        const T lph = lap9r(r_ph[su], r_ph[sm], r_ph[sdn], lane);
        const T pn = r_phi[sm][lane];
        const T Bh = B0 + B1 * r_ch[sm][lane];
        const T M = ((a * r_ph[sm][lane] + b * (pn * pn * pn)) - Bh * lph) - B1 * (gchx * gphx + gchy * gphy);
        const T Xh = halfB1 * (gphx * gphx + gphy * gphy);
        r_M[sm][lane] = M;
        r_Xh[sm][lane] = Xh;
        if (DBG && own_col && r >= y0 && r < yend) {
          const int64_t q = (int64_t)r * nx + (x0 + col);
          dbg[9 * nplane + q] = (double)M;
          dbg[10 * nplane + q] = (double)Xh;
        }
      }
    }
    __syncthreads();
    // ---- s5: phi^{n+1}, c^{n+1} (Eqs. 18, 19) and centre-of-mass contributions
    int kd = -1;
    double cv0 = 0.0, cv1 = 0.0, cv2 = 0.0;
    {
      const int r = q0 - 5 + wv;
      if (own_col && r >= y0 && r < yend) {
        const int sm = r & (RING - 1);
        const int su = (walls && r == ny - 1) ? sm : (r + 1) & (RING - 1);
        const int sdn = (walls && r == 0) ? sm : (r - 1) & (RING - 1);
        const T phn = r_ph[sm][lane] + Gamma * lap9r(r_M[su], r_M[sm], r_M[sdn], lane);
        const T ch = r_ch[sm][lane];
        const T lch = lap9r(r_ch[su], r_ch[sm], r_ch[sdn], lane);
        const T dv = div9r(r_ch[su], r_ch[sm], r_ch[sdn], D, r_Xh[su], r_Xh[sm], r_Xh[sdn], lane);
        const double xd = (double)(x0 + col), yd = (double)r;
        int cnt = 0;
        if (nd > 0) {
          for (int w = 0; w < MASK_WORDS; ++w) {
            unsigned long long m = sh.src_mask[w];
            while (m) {
              const int k = w * 64 + __ffsll(m) - 1;
              m &= m - 1;
              const DropDev d = drops[I.drop_base + k];
              const double px = d.x + (d.R - d.Rs) * d.ex, py = d.y + (d.R - d.Rs) * d.ey;
              const double dx = minimg(xd - px, (double)nx), dy = minimg(yd - py, I.yper);
              if (dx * dx + dy * dy <= d.Rs * d.Rs) ++cnt;
            }
          }
        }
        const double src = A * (double)cnt;
        const T cn = (((ch + D * lch) + dv) - gam * (ch - c0)) + T(src);
        const int64_t o = (int64_t)r * pitch + gx;
        phi_out[o] = phn;
        c_out[o] = cn;
        if (DBG && export_all(dbg_inst)) {
          const int64_t q = (int64_t)r * nx + (x0 + col);
          dbg[11 * nplane + q] = (double)phn;
          dbg[12 * nplane + q] = (double)cn;
        }
        const double v = (double)phn;
        if (nd > 0 && v >= 0.0) {
          // nearest centre among the candidates (a single candidate is the nearest)
          int best = -1;
          if (ncand == 1) {
            best = cand0;
          } else {
            double bd = 0.0;
            for (int w = 0; w < MASK_WORDS; ++w) {
              unsigned long long m = sh.near_mask[w];
              while (m) {
                const int k = w * 64 + __ffsll(m) - 1;
                m &= m - 1;
                const DropDev d = drops[I.drop_base + k];
                const double dx = minimg(xd - d.x, (double)nx), dy = minimg(yd - d.y, I.yper);
                const double d2 = dx * dx + dy * dy;
                if (best < 0 || d2 < bd) {
                  best = k;
                  bd = d2;
                }
              }
            }
          }
          const DropDev d = drops[I.drop_base + best];
          kd = best;
          cv0 = v;
          cv1 = v * minimg(xd - d.x, (double)nx);
          cv2 = v * minimg(yd - d.y, I.yper);
          if (kd == cand0) {  // the slot: this thread's running sums, in row order
            sh.slot[0][tid] += cv0;
            sh.slot[1][tid] += cv1;
            sh.slot[2][tid] += cv2;
            met0 = true;
            kd = -1;
          }
        }
      }
    }
    // other candidates (rare): deterministic per-sweep workgroup sums of their contributions, added to the
    // strip's partials in global memory (with a single candidate there are none, and no barrier is needed)
    if (ncand > 1 && __syncthreads_or(kd >= 0)) {
      if (tid < MASK_WORDS) sh.it_mask[tid] = 0ull;
      __syncthreads();
      if (kd >= 0) atomicOr(&sh.it_mask[kd >> 6], 1ull << (kd & 63));
      __syncthreads();
      for (int w = 0; w < MASK_WORDS; ++w) {
        unsigned long long m = sh.it_mask[w];
        while (m) {
          const int k = w * 64 + __ffsll(m) - 1;
          m &= m - 1;
          double s0 = kd == k ? cv0 : 0.0, s1 = kd == k ? cv1 : 0.0, s2 = kd == k ? cv2 : 0.0;
          block_reduce3(s0, s1, s2, sh.red);
          if (tid == 0) {
            const unsigned long long bit = 1ull << (k & 63);
            double* const p = part_t + (int64_t)k * 3;
            if (sh.seg_mask[k >> 6] & bit) {
              p[0] += s0;
              p[1] += s1;
              p[2] += s2;
            } else {
              sh.seg_mask[k >> 6] |= bit;
              p[0] = s0;
              p[1] = s1;
              p[2] = s2;
            }
          }
        }
      }
    }
  }
  if (nd == 0) return;
  // the slot's workgroup sum (fixed order), and the presence mask
  if (__syncthreads_or(met0)) {
    double s0 = sh.slot[0][tid], s1 = sh.slot[1][tid], s2 = sh.slot[2][tid];
    block_reduce3(s0, s1, s2, sh.red);
    if (tid == 0) {
      double* const p = part_t + (int64_t)cand0 * 3;
      p[0] = s0;
      p[1] = s1;
      p[2] = s2;
      sh.seg_mask[cand0 >> 6] |= 1ull << (cand0 & 63);
    }
  }
  __syncthreads();
  if (tid < MASK_WORDS) mask[(int64_t)sd.t * MASK_WORDS + tid] = sh.seg_mask[tid];
}

// ------------------------------------------------------------------------------------------------
// Wavefront-per-strip timestep.  The same six skewed stages as k_step, but each 64-lane wavefront
// (a workgroup of its own) owns one strip segment and sweeps it one row per iteration with no
// workgroup barrier: the rows that a stage's y-stencil needs stay in registers (a short window per
// field, rotated every iteration), and the x-neighbours come from whole-wave DPP lane shifts.  Lane l
// handles column x0 + l - 5 (periodic); the 5 halo lanes per side absorb the invalid edge lanes of
// the shifts (each stencil stage spoils one more lane at each end, five stages in all).

// Whole-wave DPP lane shifts: E receives the value of lane l + 1 (the east neighbour column), W that of
// lane l - 1 (west).  Written as one asm group per neighbourhood so that the shifted registers need no
// initialisation (the lane without a source keeps an unspecified value; it lies in the halo) and a single
// s_nop covers the read-after-VALU-write hazard of DPP.
__device__ __forceinline__ void shift_ew(float v, float& e, float& w) {
  int ei, wi;
  asm("s_nop 1\n\t"
      "v_mov_b32_dpp %0, %2 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %1, %2 wave_shr:1 row_mask:0xf bank_mask:0xf"
      : "=&v"(ei), "=&v"(wi)
      : "v"(__float_as_int(v)));
  e = __int_as_float(ei);
  w = __int_as_float(wi);
}
__device__ __forceinline__ void shift_ew(double v, double& e, double& w) {
  int elo, ehi, wlo, whi;
  asm("s_nop 1\n\t"
      "v_mov_b32_dpp %0, %4 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %1, %5 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %2, %4 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %3, %5 wave_shr:1 row_mask:0xf bank_mask:0xf"
      : "=&v"(elo), "=&v"(ehi), "=&v"(wlo), "=&v"(whi)
      : "v"(__double2loint(v)), "v"(__double2hiint(v)));
  e = __hiloint2double(ehi, elo);
  w = __hiloint2double(whi, wlo);
}

// Element at a per-lane byte offset from a wave-uniform row pointer (selects the scalar-base form of the
// global load/store instructions).
template <typename T>
__device__ __forceinline__ T ld_col(const T* row, unsigned byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(row) + byte_off);
}
template <typename T>
__device__ __forceinline__ void st_col(T* row, unsigned byte_off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(row) + byte_off) = v;
}

// 64-bit value held by lane `l` (uniform) of a wavefront.
__device__ __forceinline__ unsigned long long read_lane64(unsigned long long v, int l) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(v & 0xffffffffull), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(v >> 32), l);
  return ((unsigned long long)hi << 32) | lo;
}

// The nine values of a 3 x 3 neighbourhood of one lane: rows up = r + 1 (north), mid = r, dn = r - 1.
template <typename T>
struct Nbr {
  T c, e, w, n, s, ne, nw, se, sw;
};

__device__ __forceinline__ Nbr<float> nbr(float up, float mid, float dn) {
  Nbr<float> g;
  g.c = mid;
  g.n = up;
  g.s = dn;
  int r[6];
  asm("s_nop 1\n\t"
      "v_mov_b32_dpp %0, %6 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %1, %6 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %2, %7 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %3, %7 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %4, %8 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %5, %8 wave_shr:1 row_mask:0xf bank_mask:0xf"
      : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5])
      : "v"(__float_as_int(mid)), "v"(__float_as_int(up)), "v"(__float_as_int(dn)));
  g.e = __int_as_float(r[0]);
  g.w = __int_as_float(r[1]);
  g.ne = __int_as_float(r[2]);
  g.nw = __int_as_float(r[3]);
  g.se = __int_as_float(r[4]);
  g.sw = __int_as_float(r[5]);
  return g;
}

__device__ __forceinline__ Nbr<double> nbr(double up, double mid, double dn) {
  Nbr<double> g;
  g.c = mid;
  g.n = up;
  g.s = dn;
  int r[12];
  asm("s_nop 1\n\t"
      "v_mov_b32_dpp %0, %12 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %1, %13 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %2, %12 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %3, %13 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %4, %14 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %5, %15 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %6, %14 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %7, %15 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %8, %16 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %9, %17 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %10, %16 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %11, %17 wave_shr:1 row_mask:0xf bank_mask:0xf"
      : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]), "=&v"(r[6]), "=&v"(r[7]),
        "=&v"(r[8]), "=&v"(r[9]), "=&v"(r[10]), "=&v"(r[11])
      : "v"(__double2loint(mid)), "v"(__double2hiint(mid)), "v"(__double2loint(up)), "v"(__double2hiint(up)),
        "v"(__double2loint(dn)), "v"(__double2hiint(dn)));
  g.e = __hiloint2double(r[1], r[0]);
  g.w = __hiloint2double(r[3], r[2]);
  g.ne = __hiloint2double(r[5], r[4]);
  g.nw = __hiloint2double(r[7], r[6]);
  g.se = __hiloint2double(r[9], r[8]);
  g.sw = __hiloint2double(r[11], r[10]);
  return g;
}

template <typename T>
__device__ __forceinline__ void grad9n(const Nbr<T>& g, T& gx, T& gy) {
  gx = (T(4) * (g.e - g.w) + ((g.ne - g.nw) + (g.se - g.sw))) * cst<T>(1.0 / 12.0);
  gy = (T(4) * (g.n - g.s) + ((g.ne - g.se) + (g.nw - g.sw))) * cst<T>(1.0 / 12.0);
}

template <typename T>
__device__ __forceinline__ T lap9n(const Nbr<T>& g) {
  return (T(4) * ((g.e + g.w) + (g.n + g.s)) + ((g.ne + g.nw) + (g.se + g.sw)) - T(20) * g.c) * cst<T>(1.0 / 6.0);
}

template <typename T>
__device__ __forceinline__ T div9n(const Nbr<T>& c, const Nbr<T>& X, T D) {
  const T k0 = D * c.c, X0 = X.c;
  const T t1 = (k0 + D * c.e) * (X.e - X0);
  const T t2 = (k0 + D * c.n) * (X.n - X0);
  const T t3 = (k0 + D * c.w) * (X.w - X0);
  const T t4 = (k0 + D * c.s) * (X.s - X0);
  const T t5 = (k0 + D * c.ne) * (X.ne - X0);
  const T t6 = (k0 + D * c.nw) * (X.nw - X0);
  const T t7 = (k0 + D * c.sw) * (X.sw - X0);
  const T t8 = (k0 + D * c.se) * (X.se - X0);
  return (T(4) * ((t1 + t3) + (t2 + t4)) + ((t5 + t6) + (t7 + t8))) * cst<T>(1.0 / 12.0);
}


// The 9-point gradient and Laplacian of a 3 x 3 neighbourhood (rows up, mid, dn) as grad9n and lap9n compute
// them, the same operations in the same order, from row terms: D = e - w and S = e + w of each row, the
// vertical difference V = n - s and its neighbours' sum Y = V(east) + V(west), which equals
// (ne - se) + (nw - sw) exactly (a lane shift commutes with a lane-wise difference).  In FP32 the shift
// rides on the subtraction or addition itself (a DPP operand), so a row costs three instructions instead of
// two moves and two operations; FP64 operations take no DPP operand and use the neighbourhood.
// S of the rows u, m, d (the Laplacian alone)
__device__ __forceinline__ void rows_s(float u, float m, float d, float (&S)[3]) {
  int t[3], r[3];
  asm("s_nop 1\n\t"
      "v_mov_b32_dpp %0, %6 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %1, %7 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_mov_b32_dpp %2, %8 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_add_f32_dpp %3, %6, %0 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_add_f32_dpp %4, %7, %1 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_add_f32_dpp %5, %8, %2 wave_shl:1 row_mask:0xf bank_mask:0xf"
      : "=&v"(t[0]), "=&v"(t[1]), "=&v"(t[2]), "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2])
      : "v"(__float_as_int(u)), "v"(__float_as_int(m)), "v"(__float_as_int(d)));
  for (int i = 0; i < 3; ++i) S[i] = __int_as_float(r[i]);
}
// D, S (with DS) of the rows u, m, d, and V = u - d with Y = V(east) + V(west), in one group: V is
// written first, so the row operations in between cover the DPP read-after-write of V.
template <bool DS>
__device__ __forceinline__ void rows_dvy(float u, float m, float d, float (&D)[3], float (&S)[3], float& V,
                                         float& Y) {
  int t[4], r[6], v, y;
  if constexpr (DS) {
    asm("s_nop 1\n\t"
        "v_sub_f32 %10, %12, %14\n\t"
        "v_mov_b32_dpp %0, %12 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_mov_b32_dpp %1, %13 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_mov_b32_dpp %2, %14 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_sub_f32_dpp %4, %12, %0 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %5, %12, %0 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_sub_f32_dpp %6, %13, %1 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %7, %13, %1 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_sub_f32_dpp %8, %14, %2 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %9, %14, %2 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_mov_b32_dpp %3, %10 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %11, %10, %3 wave_shl:1 row_mask:0xf bank_mask:0xf"
        : "=&v"(t[0]), "=&v"(t[1]), "=&v"(t[2]), "=&v"(t[3]), "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]),
          "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]), "=&v"(v), "=&v"(y)
        : "v"(__float_as_int(u)), "v"(__float_as_int(m)), "v"(__float_as_int(d)));
    for (int i = 0; i < 3; ++i) {
      D[i] = __int_as_float(r[2 * i]);
      S[i] = __int_as_float(r[2 * i + 1]);
    }
  } else {
    asm("s_nop 1\n\t"
        "v_sub_f32 %7, %9, %11\n\t"
        "v_mov_b32_dpp %0, %9 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_mov_b32_dpp %1, %10 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_mov_b32_dpp %2, %11 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_sub_f32_dpp %4, %9, %0 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_sub_f32_dpp %5, %10, %1 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_sub_f32_dpp %6, %11, %2 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_mov_b32_dpp %3, %7 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %8, %7, %3 wave_shl:1 row_mask:0xf bank_mask:0xf"
        : "=&v"(t[0]), "=&v"(t[1]), "=&v"(t[2]), "=&v"(t[3]), "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(v),
          "=&v"(y)
        : "v"(__float_as_int(u)), "v"(__float_as_int(m)), "v"(__float_as_int(d)));
    for (int i = 0; i < 3; ++i) D[i] = __int_as_float(r[i]);
  }
  V = __int_as_float(v);
  Y = __int_as_float(y);
}
// The x-differences of the printed advection half-step (Eqs. 16-17) for u, phi and c of one row: ue - uw, and
// for g = phi, c the backward gc - gw and forward ge - gc differences (the upwind side picks one), with the
// shifts on the subtractions.
__device__ __forceinline__ void adv_dx(float u, float p, float c, float& du, float& pb, float& pf, float& cb,
                                       float& cf) {
  int t, r[5];
  asm("s_nop 1\n\t"
      "v_mov_b32_dpp %0, %6 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_sub_f32_dpp %1, %6, %0 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_subrev_f32_dpp %2, %7, %7 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_sub_f32_dpp %3, %7, %7 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_subrev_f32_dpp %4, %8, %8 wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_sub_f32_dpp %5, %8, %8 wave_shl:1 row_mask:0xf bank_mask:0xf"
      : "=&v"(t), "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4])
      : "v"(__float_as_int(u)), "v"(__float_as_int(p)), "v"(__float_as_int(c)));
  du = __int_as_float(r[0]);
  pb = __int_as_float(r[1]);
  pf = __int_as_float(r[2]);
  cb = __int_as_float(r[3]);
  cf = __int_as_float(r[4]);
}
// gradient (as grad9n) and, with LAP, Laplacian (as lap9n) of the neighbourhood of rows up, mid, dn
template <bool LAP, typename T>
__device__ __forceinline__ void sten(T up, T mid, T dn, T& gx, T& gy, T& lap) {
  if constexpr (sizeof(T) == 8) {
    const Nbr<T> g = nbr(up, mid, dn);
    grad9n(g, gx, gy);
    if constexpr (LAP) lap = lap9n(g);
  } else {
    float D[3], S[3], V, Y;
    rows_dvy<LAP>(up, mid, dn, D, S, V, Y);
    gx = (4.0f * D[1] + (D[0] + D[2])) * cst<float>(1.0 / 12.0);
    gy = (4.0f * V + Y) * cst<float>(1.0 / 12.0);
    if constexpr (LAP) lap = (4.0f * (S[1] + (up + dn)) + (S[0] + S[2]) - 20.0f * mid) * cst<float>(1.0 / 6.0);
  }
}
// the Laplacian alone (as lap9n)
template <typename T>
__device__ __forceinline__ T sten_lap(T up, T mid, T dn) {
  if constexpr (sizeof(T) == 8) {
    return lap9n(nbr(up, mid, dn));
  } else {
    float S[3];
    rows_s(up, mid, dn, S);
    return (4.0f * (S[1] + (up + dn)) + (S[0] + S[2]) - 20.0f * mid) * cst<float>(1.0 / 6.0);
  }
}

// DBG as for k_step.  PLAIN: every lattice of the launch is periodic in y and advects by the printed Eqs. (16)-(17), so the
// plate mirrors and the flux form compile away.  Occupancy targets: FP64 keeps its windows and two prefetch
// sets in registers at two waves per SIMD; FP16 storage takes three; FP32 (one prefetch set, scalar-base
// addresses) fits four, its export instance three.
template <typename T, typename P, bool DBG, bool PLAIN>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 2 : sizeof(P) == 4 && !DBG ? 4 : 3))) void k_wave(int parity, const TileDev* __restrict__ segs,
                                             const InstDev* __restrict__ insts, T* __restrict__ buf,
                                             const DropDev* __restrict__ drops, double* __restrict__ part,
                                             uint64_t* __restrict__ mask, const int64_t* __restrict__ step,
                                             double* __restrict__ dbg, int dbg_inst) {
  // centre-of-mass sums of the segment's first CM_SLOTS nearest-centre candidates, per lane (a lane adds its
  // own nodes row after row; one butterfly per slot at the end of the segment)
  __shared__ double acc[CM_SLOTS][3][64];
  // droplet candidates of this segment (read-only after set-up): near the box, and production disks reaching it
  __shared__ unsigned long long s_near[MASK_WORDS], s_src[MASK_WORDS];
  // slot of each droplet (CM_SLOTS: none) and droplet of each slot
  __shared__ unsigned char s_slot[MAXDROP];
  __shared__ int s_cand[CM_SLOTS];
  __shared__ double s_cxy[CM_SLOTS][2];  // centre of each slot's droplet

  const TileDev sd = segs[blockIdx.x];
  if (sd.inst < 0) return;
  if (DBG && sd.inst != export_inst(dbg_inst)) return;
  const InstDev& I = insts[sd.inst];
  const int lane = threadIdx.x;
  const int nx = I.nx, ny = I.ny, pitch = I.pitch, nd = I.ndrop;
  const int x0 = sd.x0, y0 = sd.y0;
  const int yend = min(y0 + I.seg_rows, ny);
  const int xend = min(x0 + I.strip_w, nx);
  const int col = lane - 5;
  const int gx = wrap_idx(x0 + col, nx);
  const int gxm = gx == 0 ? nx - 1 : gx - 1, gxp = gx == nx - 1 ? 0 : gx + 1;
  const bool own_col = col >= 0 && col < I.strip_w && x0 + col < nx;
  const int64_t plane = I.pstride;
  const T* __restrict__ phi_in = buf + I.off_phi[parity];
  const T* __restrict__ c_in = buf + I.off_c[parity];
  const P* __restrict__ fin = reinterpret_cast<const P*>(buf + I.off_f[parity]);
  P* __restrict__ fout = reinterpret_cast<P*>(buf + I.off_f[parity ^ 1]);
  const T wr0 = T(I.wn[0]), wr1 = T(I.wn[1]), wr5 = T(I.wn[2]);
  T* __restrict__ phi_out = buf + I.off_phi[parity ^ 1];
  T* __restrict__ c_out = buf + I.off_c[parity ^ 1];
  const int64_t nplane = (int64_t)nx * ny;

  // --- droplet culling for the owned box [x0, xend) x [y0, yend); lane l examines droplets l + 64 w.
  // The candidate masks go to LDS; the mask of droplets met (seg_v) is kept lane-distributed (lane w holds
  // word w) to spare scalar registers.
  unsigned long long seg_v = 0ull;
  if (lane < MASK_WORDS) {
    s_near[lane] = 0ull;
    s_src[lane] = 0ull;
  }
  bool any_src = false;
  if (nd > 0) {
    const double Lx = nx, Ly = I.yper;
    const double xm = 0.5 * (x0 + xend - 1), ym = 0.5 * (y0 + yend - 1);
    const double hx = 0.5 * (xend - 1 - x0), hy = 0.5 * (yend - 1 - y0);
    double mind2[MASK_WORDS];
    bool srcf[MASK_WORDS];
    double thr = 1e300;
    for (int w = 0; w < MASK_WORDS; ++w) {
      const int k = w * 64 + lane;
      mind2[w] = 1e300;
      srcf[w] = false;
      if (k < nd) {
        const DropDev d = drops[I.drop_base + k];
        const double ddx = fabs(minimg(xm - d.x, Lx)), ddy = fabs(minimg(ym - d.y, Ly));
        const double ux = ddx + hx, uy = ddy + hy;
        thr = fmin(thr, ux * ux + uy * uy);
        const double lx = fmax(0.0, ddx - hx), ly = fmax(0.0, ddy - hy);
        mind2[w] = lx * lx + ly * ly;
        if (d.active) {
          const double px = d.x + (d.R - d.Rs) * d.ex, py = d.y + (d.R - d.Rs) * d.ey;
          const double sdx = fmax(0.0, fabs(minimg(xm - px, Lx)) - hx);
          const double sdy = fmax(0.0, fabs(minimg(ym - py, Ly)) - hy);
          const double rr = d.Rs + 1e-6;
          srcf[w] = sdx * sdx + sdy * sdy <= rr * rr;
        }
      }
    }
    for (int o = 32; o > 0; o >>= 1) thr = fmin(thr, __shfl_xor(thr, o, 64));
    const double lim = thr * (1.0 + 1e-12) + 1e-6;
    for (int w = 0; w < MASK_WORDS; ++w) {
      const unsigned long long nb = __ballot(w * 64 + lane < nd && mind2[w] <= lim);
      const unsigned long long sb = __ballot(srcf[w]);
      if (lane == w) {
        s_near[w] = nb;
        s_src[w] = sb;
      }
      any_src = any_src || sb != 0ull;
    }
  }
  for (int s = 0; s < CM_SLOTS; ++s) acc[s][0][lane] = acc[s][1][lane] = acc[s][2][lane] = 0.0;
  int ncand = 0;  // wave-uniform: number of nearest-centre candidates
  if (nd > 0) {
    __syncthreads();  // s_near complete
    for (int w = 0; w < MASK_WORDS; ++w) {
      const unsigned long long m = s_near[w];
      const int k = w * 64 + lane;
      const int r = ncand + __popcll(m & ((1ull << lane) - 1ull));  // candidates below droplet k
      const bool cand = (m >> lane) & 1ull;
      s_slot[k] = (unsigned char)(cand && r < CM_SLOTS ? r : CM_SLOTS);
      if (cand && r < CM_SLOTS) {
        const DropDev d = drops[I.drop_base + k];
        s_cand[r] = k;
        s_cxy[r][0] = d.x;
        s_cxy[r][1] = d.y;
      }
      ncand += __popcll(m);
    }
    ncand = __builtin_amdgcn_readfirstlane(ncand);
  }
  unsigned slots_met = 0u;  // wave-uniform: slot s received a node
  const int t_local = sd.t - I.tile_base[TILING_FUSED];
  double* const part_t = part + I.part_base[TILING_FUSED] + (int64_t)t_local * nd * 3;
  __syncthreads();  // the candidate masks in LDS are complete
  const double tn = (double)(*step);
  const double A = I.A0 * (tn < I.t_star ? tn : I.t_star);

  const T a = T(I.a), b = T(I.b), B0 = T(I.B0), B1 = T(I.B1), halfB1 = T(I.halfB1);
  const T omega = T(I.omega), coef = T(I.coef);
  const T w0 = cst<T>(4.0 / 9.0), w1 = cst<T>(1.0 / 9.0), w5 = cst<T>(1.0 / 36.0);
  const T cw0 = coef * w0, cw1 = coef * w1, cw5 = coef * w5;
  const LbConst<T> lbk{w0, w1, w5, cw0, cw1, cw5, omega, wr0, wr1, wr5, T(I.n0)};
  const T Gamma = T(I.Gamma), D = T(I.D), gam = T(I.gamma), c0 = T(I.c0);
  const int adv = PLAIN ? 0 : I.advection;

  // Register windows.  In the iteration whose stage-0 row is q, stage s works on row q - s; the
  // digit in a window name is the row offset below q (P2 = phi^n of row q - 2, ...).
  T P0 = T(0), P1 = T(0), P2 = T(0), P3 = T(0), P4 = T(0);     // phi^n
  T C0 = T(0), C1 = T(0), C2 = T(0), C3 = T(0), C4 = T(0);     // c^n
  T MU1 = T(0), MU2 = T(0), MU3 = T(0), X1 = T(0), X2 = T(0), X3 = T(0);  // mu_phi, X
  T GCX1 = T(0), GCX2 = T(0), GCY1 = T(0), GCY2 = T(0);  // grad c^n (9-point), from stage 1 for stage 2
  T UX2 = T(0), UX3 = T(0), UX4 = T(0), UY2 = T(0), UY3 = T(0), UY4 = T(0);  // u^n
  T PH3 = T(0), PH4 = T(0), PH5 = T(0), CH3 = T(0), CH4 = T(0), CH5 = T(0), CH6 = T(0);  // phi, c at n+1/2
  T M4 = T(0), M5 = T(0), M6 = T(0), XH4 = T(0), XH5 = T(0), XH6 = T(0);  // M, X^{n+1/2}

  // Prefetch sets: phi, c of a coming stage-0 row and the pulled populations of a coming stage-2 row,
  // PFD rows ahead.  With PFD = 2 the sweep is unrolled by two and the sets alternate, so that no
  // register holding an outstanding load is ever copied.  Two sets in FP64 and with FP16 storage; FP32 keeps
  // one (two, at four waves per SIMD, were 1.4 % slower on the 2048^2 emulsion, 1-3 % faster on the batch of
  // small lattices and at 4096^2).
  constexpr int PFD = sizeof(T) == 8 || sizeof(P) == 2 ? 2 : 1;
  struct Pref {
    T phi, c;
    P f[9];
  };
  Pref pfs[PFD];
  // Addresses: a wave-uniform row pointer (scalar registers) plus a per-lane 32-bit column byte offset.
  unsigned bx = (unsigned)gx * sizeof(T);
  unsigned fx = (unsigned)gx * sizeof(P), fxm = (unsigned)gxm * sizeof(P), fxp = (unsigned)gxp * sizeof(P);
  const int walls = PLAIN ? 0 : I.walls;
  // the loads of stage-0 row r (stored row gy) and of the pulls into stage-2 row r (stored rows gym, gy, gyp
  // for r - 1, r, r + 1)
  auto load_s0_rows = [&](Pref& p, int gy) {
    const int64_t ro = (int64_t)gy * pitch;
    p.phi = ld_col(phi_in + ro, bx);
    p.c = ld_col(c_in + ro, bx);
  };
  auto load_s2_rows = [&](Pref& p, int r, int gym, int gy, int gyp) {
    const int64_t r0 = (int64_t)gy * pitch, rm = (int64_t)gym * pitch, rp = (int64_t)gyp * pitch;
    // behind a plate: the node's own opposite population (halfway bounce-back)
    const bool bb0 = walls && r == 0, bbn = walls && r == ny - 1;
    p.f[0] = ld_col(fin + r0, fx);
    p.f[1] = ld_col(fin + plane + r0, fxm);
    p.f[2] = bb0 ? ld_col(fin + 4 * plane + r0, fx) : ld_col(fin + 2 * plane + rm, fx);
    p.f[3] = ld_col(fin + 3 * plane + r0, fxp);
    p.f[4] = bbn ? ld_col(fin + 2 * plane + r0, fx) : ld_col(fin + 4 * plane + rp, fx);
    p.f[5] = bb0 ? ld_col(fin + 7 * plane + r0, fx) : ld_col(fin + 5 * plane + rm, fxm);
    p.f[6] = bb0 ? ld_col(fin + 8 * plane + r0, fx) : ld_col(fin + 6 * plane + rm, fxp);
    p.f[7] = bbn ? ld_col(fin + 5 * plane + r0, fx) : ld_col(fin + 7 * plane + rp, fxp);
    p.f[8] = bbn ? ld_col(fin + 6 * plane + r0, fx) : ld_col(fin + 8 * plane + rp, fxm);
  };
  auto load_s0 = [&](Pref& p, int r) { load_s0_rows(p, row_of(r, ny, walls)); };
  auto load_s2 = [&](Pref& p, int r) {
    load_s2_rows(p, r, row_of(r - 1, ny, walls), row_of(r, ny, walls), row_of(r + 1, ny, walls));
  };
  // Set j serves the iterations it = j (mod PFD): stage-0 row y0 - 5 + it, stage-2 row y0 - 7 + it, whose
  // first valid row y0 - 3 comes at it = 4.
  for (int j = 0; j < PFD; ++j) {
    load_s0(pfs[j], y0 - 5 + j);
    load_s2(pfs[j], y0 - 3 + ((j - 4) % PFD + PFD) % PFD);
  }

  const int nit = (yend - y0) + 10;
  // PLAIN lattices are periodic in y: the stored rows of the coming loads advance by one per iteration and
  // are tracked from one iteration to the next (stage-0 row q + PFD; row r + PFD - 1 of the stage-2 pulls).
  int nr0 = wrap_idx(y0 - 5 + PFD, ny), nr2 = wrap_idx(y0 - 8 + PFD, ny);
  auto next_row = [&](int g) { return g + 1 == ny ? 0 : g + 1; };
  // one sweep iteration; `pf` holds the stage-0 row q and the stage-2 row q - 2, and is refilled for
  // the rows PFD further on
  auto sweep = [&](int it, Pref& pf) {
    const int q = y0 - 5 + it;
    // FP32: the column offsets pass an empty asm each iteration, so that the compiler cannot hoist a 64-bit
    // per-lane address (row-independent base + offset) out of the loop and keeps the scalar-base form; this
    // frees about 30 VGPRs, enough for four wavefronts per SIMD.  (FP64 and FP16 storage ran slower with it.)
    if constexpr (sizeof(T) == 4 && sizeof(P) == 4) asm volatile("" : "+v"(bx), "+v"(fx), "+v"(fxm), "+v"(fxp));
    int g0 = 0, g2m = 0, g2 = 0, g2p = 0;
    if constexpr (PLAIN) {
      g0 = nr0;
      nr0 = next_row(nr0);
      g2m = nr2;
      g2 = next_row(g2m);
      g2p = next_row(g2);
      nr2 = g2;
    }
    // ---- s0: phi^n, c^n of row q; prefetch row q + PFD
    P0 = pf.phi;
    C0 = pf.c;
    if (q + PFD < yend + 5) {
      if constexpr (PLAIN)
        load_s0_rows(pf, g0);
      else
        load_s0(pf, q + PFD);
    }
    // ---- s1: mu_phi and X (Eqs. 3, 5) at row q - 1
    if (q - 1 >= y0 - 4 && q - 1 < yend + 4) {
      T gpx, gpy, gcx, gcy, lp, nolap;
      sten<true>(P0, P1, P2, gpx, gpy, lp);
      sten<false>(C0, C1, C2, gcx, gcy, nolap);
      GCX1 = gcx;
      GCY1 = gcy;
      const T ph = P1;
      const T B = B0 + B1 * C1;
      MU1 = ((a * ph + b * (ph * ph * ph)) - B * lp) - B1 * (gpx * gcx + gpy * gcy);
      X1 = halfB1 * (gpx * gpx + gpy * gpy);
      if (DBG && own_col && q - 1 >= y0 && q - 1 < yend) {
        const int64_t qq = (int64_t)(q - 1) * nx + (x0 + col);
        dbg[0 * nplane + qq] = (double)MU1;
        dbg[1 * nplane + qq] = (double)X1;
      }
    }
    // ---- s2: force, moments, collision at row q - 2
    if (q - 2 >= y0 - 3 && q - 2 < yend + 3) {
      const int r = q - 2;
      T gmx, gmy, gXx, gXy, nolap;
      sten<false>(MU1, MU2, MU3, gmx, gmy, nolap);
      sten<false>(X1, X2, X3, gXx, gXy, nolap);
      const T gcx = GCX2, gcy = GCY2;
      const T ph = P2, cv = C2;
      const T Fx = (-(ph * gmx) - gcx) - cv * gXx;
      const T Fy = (-(ph * gmy) - gcy) - cv * gXy;
      T d[9], dn, nn, ux, uy;
      lb_moments<T, P>(pf.f, lbk, Fx, Fy, d, dn, nn, ux, uy);
      UX2 = ux;
      UY2 = uy;
      if (own_col && r >= y0 && r < yend) {
        P out[9];
        double sv[9];
        lb_collide<T, P>(d, dn, nn, ux, uy, Fx, Fy, lbk, out, sv);
        P* const o = fout + (int64_t)r * pitch;
        for (int i = 0; i < 9; ++i) st_col(o + i * plane, fx, out[i]);
        if (DBG) {
          const int64_t qq = (int64_t)r * nx + (x0 + col);
          dbg[2 * nplane + qq] = (double)Fx;
          dbg[3 * nplane + qq] = (double)Fy;
          dbg[4 * nplane + qq] = (double)nn;
          dbg[5 * nplane + qq] = (double)ux;
          dbg[6 * nplane + qq] = (double)uy;
          if (export_all(dbg_inst))
            for (int i = 0; i < 9; ++i) dbg[(13 + i) * nplane + qq] = sv[i];
        }
      }
      if (r + PFD < yend + 3) {
        if constexpr (PLAIN)
          load_s2_rows(pf, r + PFD, g2m, g2, g2p);
        else
          load_s2(pf, r + PFD);
      }
    }
    // ---- s3: advection half-step (Eqs. 16-17) at row q - 3
    if (q - 3 >= y0 - 2 && q - 3 < yend + 2) {
      if constexpr (PLAIN && sizeof(T) == 4) {
        // advect_n's printed form with the x-differences from adv_dx (same operations, same order)
        float du, pb, pfw, cb, cfw;
        adv_dx(UX3, P3, C3, du, pb, pfw, cb, cfw);
        const T uc = UX3, vc = UY3, vn = UY2, vs = UY4;
        const T divu = T(0.5) * du + T(0.5) * (vn - vs);
        const T dpx = uc > T(0) ? pb : pfw, dcx = uc > T(0) ? cb : cfw;
        const T dpy = vc > T(0) ? P3 - P4 : P2 - P3, dcy = vc > T(0) ? C3 - C4 : C2 - C3;
        PH3 = P3 - ((P3 * divu + uc * dpx) + vc * dpy);
        CH3 = C3 - ((C3 * divu + uc * dcx) + vc * dcy);
      } else {
        T ue, uw, pe, pw, ce, cw;
        shift_ew(UX3, ue, uw);
        shift_ew(P3, pe, pw);
        shift_ew(C3, ce, cw);
        // u^n beyond a plate is not computed: its mirror image with u_y reversed
        const T vn = (walls && q - 3 == ny - 1) ? -UY3 : UY2, vs = (walls && q - 3 == 0) ? -UY3 : UY4;
        PH3 = advect_n(P3, pe, pw, P2, P4, UX3, ue, uw, UY3, vn, vs, adv);
        CH3 = advect_n(C3, ce, cw, C2, C4, UX3, ue, uw, UY3, vn, vs, adv);
      }
      if (DBG && own_col && q - 3 >= y0 && q - 3 < yend) {
        const int64_t qq = (int64_t)(q - 3) * nx + (x0 + col);
        dbg[7 * nplane + qq] = (double)PH3;
        dbg[8 * nplane + qq] = (double)CH3;
      }
    }
    // ---- s4: bracket M of Eq. (18) and X^{n+1/2} at row q - 4
    if (q - 4 >= y0 - 1 && q - 4 < yend + 1) {
      // half-step fields beyond a plate: the mirror image of the boundary row
      const bool top = walls && q - 4 == ny - 1, bot = walls && q - 4 == 0;
      T gphx, gphy, gchx, gchy, lph, nolap;
      sten<true>(top ? PH4 : PH3, PH4, bot ? PH4 : PH5, gphx, gphy, lph);
      sten<false>(top ? CH4 : CH3, CH4, bot ? CH4 : CH5, gchx, gchy, nolap);
      const T pn = P4;
      const T Bh = B0 + B1 * CH4;
      M4 = ((a * PH4 + b * (pn * pn * pn)) - Bh * lph) - B1 * (gchx * gphx + gchy * gphy);
      XH4 = halfB1 * (gphx * gphx + gphy * gphy);
      if (DBG && own_col && q - 4 >= y0 && q - 4 < yend) {
        const int64_t qq = (int64_t)(q - 4) * nx + (x0 + col);
        dbg[9 * nplane + qq] = (double)M4;
        dbg[10 * nplane + qq] = (double)XH4;
      }
    }
    // ---- s5: phi^{n+1}, c^{n+1} (Eqs. 18, 19) at row q - 5 and centre-of-mass contributions
    if (q - 5 >= y0) {
      const int r = q - 5;
      const bool top = walls && r == ny - 1, bot = walls && r == 0;
      const Nbr<T> gch = nbr(top ? CH5 : CH4, CH5, bot ? CH5 : CH6), gXh = nbr(top ? XH5 : XH4, XH5, bot ? XH5 : XH6);
      const T phn = PH5 + Gamma * sten_lap(top ? M5 : M4, M5, bot ? M5 : M6);
      const T ch = CH5;
      const T lch = lap9n(gch);
      const T dv = div9n(gch, gXh, D);
      const double xd = (double)(x0 + col), yd = (double)r;
      int cnt = 0;
      for (int w = 0; any_src && w < MASK_WORDS; ++w) {
        unsigned long long m = s_src[w];
        while (m) {
          const int k = w * 64 + __ffsll(m) - 1;
          m &= m - 1;
          const DropDev d = drops[I.drop_base + k];
          const double px = d.x + (d.R - d.Rs) * d.ex, py = d.y + (d.R - d.Rs) * d.ey;
          const double dx = minimg(xd - px, (double)nx), dy = minimg(yd - py, I.yper);
          if (dx * dx + dy * dy <= d.Rs * d.Rs) ++cnt;
        }
      }
      const double src = A * (double)cnt;
      const T cn = (((ch + D * lch) + dv) - gam * (ch - c0)) + T(src);
      int kd = -1;
      double cv0 = 0.0, cv1 = 0.0, cv2 = 0.0;
      if (own_col) {
        st_col(phi_out + (int64_t)r * pitch, bx, phn);
        st_col(c_out + (int64_t)r * pitch, bx, cn);
        if (DBG && export_all(dbg_inst)) {
          const int64_t qq = (int64_t)r * nx + (x0 + col);
          dbg[11 * nplane + qq] = (double)phn;
          dbg[12 * nplane + qq] = (double)cn;
        }
        const double v = (double)phn;
        if (nd > 0 && v >= 0.0) {
          // nearest centre among the candidates (a single candidate is the nearest)
          int best = -1;
          if (ncand == 1) {
            best = s_cand[0];
          } else {
            double bd = 0.0;
            for (int w = 0; w < MASK_WORDS; ++w) {
              unsigned long long m = s_near[w];
              while (m) {
                const int k = w * 64 + __ffsll(m) - 1;
                m &= m - 1;
                const DropDev d = drops[I.drop_base + k];
                const double dx = minimg(xd - d.x, (double)nx), dy = minimg(yd - d.y, I.yper);
                const double d2 = dx * dx + dy * dy;
                if (best < 0 || d2 < bd) {
                  best = k;
                  bd = d2;
                }
              }
            }
          }
          const int sl = s_slot[best];
          double cx, cy;
          if (sl < CM_SLOTS) {
            cx = s_cxy[sl][0];
            cy = s_cxy[sl][1];
          } else {
            const DropDev d = drops[I.drop_base + best];
            cx = d.x;
            cy = d.y;
          }
          kd = best;
          cv0 = v;
          cv1 = v * minimg(xd - cx, (double)nx);
          cv2 = v * minimg(yd - cy, I.yper);
        }
      }
      // centre-of-mass contributions: candidate number r of the segment (in droplet order) has slot r; a lane
      // adds its node to its slot.  Candidates beyond the slots (rare) take the row's wave sum (fixed
      // butterfly order) straight into the strip's partials.
      if (nd > 0 && __ballot(kd >= 0) != 0ull) {
        const int slot = kd >= 0 ? (int)s_slot[kd] : CM_SLOTS;
        if (slot < CM_SLOTS) {
          acc[slot][0][lane] += cv0;
          acc[slot][1][lane] += cv1;
          acc[slot][2][lane] += cv2;
        }
        for (int s = 0; s < CM_SLOTS; ++s)
          if (__ballot(slot == s) != 0ull) slots_met |= 1u << s;
        unsigned long long pend = __ballot(slot == CM_SLOTS && kd >= 0);
        while (pend) {
          const int k = __builtin_amdgcn_readlane(kd, __ffsll(pend) - 1);
          const bool sel = kd == k;
          double s0 = sel ? cv0 : 0.0, s1 = sel ? cv1 : 0.0, s2 = sel ? cv2 : 0.0;
          for (int o = 32; o > 0; o >>= 1) {
            s0 += __shfl_xor(s0, o, 64);
            s1 += __shfl_xor(s1, o, 64);
            s2 += __shfl_xor(s2, o, 64);
          }
          const unsigned long long bit = 1ull << (k & 63);
          const bool seen = (read_lane64(seg_v, k >> 6) & bit) != 0ull;
          if (lane == (k >> 6)) seg_v |= bit;
          if (lane == 0) {
            double* const p = part_t + (int64_t)k * 3;
            if (seen) {
              p[0] += s0;
              p[1] += s1;
              p[2] += s2;
            } else {
              p[0] = s0;
              p[1] = s1;
              p[2] = s2;
            }
          }
          pend &= ~__ballot(sel);
        }
      }
    }
    // ---- rotate the windows by one row
    P4 = P3; P3 = P2; P2 = P1; P1 = P0;
    C4 = C3; C3 = C2; C2 = C1; C1 = C0;
    MU3 = MU2; MU2 = MU1; X3 = X2; X2 = X1; GCX2 = GCX1; GCY2 = GCY1;
    UX4 = UX3; UX3 = UX2; UY4 = UY3; UY3 = UY2;
    PH5 = PH4; PH4 = PH3; CH6 = CH5; CH5 = CH4; CH4 = CH3;
    M6 = M5; M5 = M4; XH6 = XH5; XH5 = XH4;
  };
  for (int it = 0; it < nit; it += PFD) {
#pragma unroll
    for (int j = 0; j < PFD; ++j)
      if (it + j < nit) sweep(it + j, pfs[j]);
  }
  if (nd == 0) return;
  // the slots' wave sums (fixed butterfly order), for the candidates that received nodes
  for (int s = 0; s < CM_SLOTS; ++s) {
    if (!(slots_met & (1u << s))) continue;
    const int k = s_cand[s];
    double s0 = acc[s][0][lane], s1 = acc[s][1][lane], s2 = acc[s][2][lane];
    for (int o = 32; o > 0; o >>= 1) {
      s0 += __shfl_xor(s0, o, 64);
      s1 += __shfl_xor(s1, o, 64);
      s2 += __shfl_xor(s2, o, 64);
    }
    if (lane == (k >> 6)) seg_v |= 1ull << (k & 63);
    if (lane == 0) {
      double* const p = part_t + (int64_t)k * 3;
      p[0] = s0;
      p[1] = s1;
      p[2] = s2;
    }
  }
  if (lane < MASK_WORDS) mask[(int64_t)sd.t * MASK_WORDS + lane] = seg_v;
}

}  // namespace

// ------------------------------------------------------------------------------------------------
template <typename T, typename P>
hipError_t launch_lb(hipStream_t s, int mode, int parity, int ntiles_launch, const TileDev* tiles,
                     const InstDev* inst, T* buf, double* dbg, int dbg_inst) {
  if (ntiles_launch <= 0) return hipSuccess;
  dim3 grid(ntiles_launch), block(NTHREADS);
  if (mode == 0)
    hipLaunchKernelGGL((k_lb<T, P, 0>), grid, block, 0, s, parity, tiles, inst, buf, dbg, dbg_inst);
  else if (mode == 1)
    hipLaunchKernelGGL((k_lb<T, P, 1>), grid, block, 0, s, parity, tiles, inst, buf, dbg, dbg_inst);
  else
    hipLaunchKernelGGL((k_lb<T, P, 2>), grid, block, 0, s, parity, tiles, inst, buf, dbg, dbg_inst);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fd(hipStream_t s, int mode, int parity, int ntiles_launch, const TileDev* tiles,
                     const InstDev* inst, T* buf, const DropDev* drops, double* part, uint64_t* mask,
                     const int64_t* step, double* dbg, int dbg_inst) {
  if (ntiles_launch <= 0) return hipSuccess;
  dim3 grid(ntiles_launch), block(NTHREADS);
  if (mode == 0)
    hipLaunchKernelGGL((k_fd<T, 0>), grid, block, 0, s, parity, tiles, inst, buf, drops, part, mask, step,
                       dbg, dbg_inst);
  else
    hipLaunchKernelGGL((k_fd<T, 1>), grid, block, 0, s, parity, tiles, inst, buf, drops, part, mask, step,
                       dbg, dbg_inst);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cm_partials(hipStream_t s, int parity, int ntiles_launch, const TileDev* tiles,
                              const InstDev* inst, T* buf, const DropDev* drops, double* part,
                              uint64_t* mask) {
  if (ntiles_launch <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_cm_partials<T>), dim3(ntiles_launch), dim3(NTHREADS), 0, s, parity, tiles, inst,
                     buf, drops, part, mask);
  return hipGetLastError();
}

template <typename T, typename P>
hipError_t launch_obs(hipStream_t s, int parity, int ntiles_launch, const TileDev* tiles,
                      const InstDev* inst, T* buf, const DropDev* drops, double* obs_part, int obs_stride) {
  if (ntiles_launch <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_obs<T, P>), dim3(ntiles_launch), dim3(NTHREADS), 0, s, parity, tiles, inst, buf, drops,
                     obs_part, obs_stride);
  return hipGetLastError();
}

template <typename T, typename P>
hipError_t launch_step(hipStream_t s, int parity, int nseg_launch, const TileDev* segs, const InstDev* inst, T* buf,
                       const DropDev* drops, double* part, uint64_t* mask, const int64_t* step, double* dbg,
                       int dbg_inst) {
  if (nseg_launch <= 0) return hipSuccess;
  if (dbg)
    hipLaunchKernelGGL((k_step<T, P, true>), dim3(nseg_launch), dim3(NTHREADS), 0, s, parity, segs, inst, buf,
                       drops, part, mask, step, dbg, dbg_inst);
  else
    hipLaunchKernelGGL((k_step<T, P, false>), dim3(nseg_launch), dim3(NTHREADS), 0, s, parity, segs, inst, buf,
                       drops, part, mask, step, dbg, dbg_inst);
  return hipGetLastError();
}

template <typename T, typename P>
hipError_t launch_wave(hipStream_t s, int parity, int nseg_launch, const TileDev* segs, const InstDev* inst, T* buf,
                       const DropDev* drops, double* part, uint64_t* mask, const int64_t* step, double* dbg,
                       int dbg_inst, bool plain) {
  if (nseg_launch <= 0) return hipSuccess;
  const dim3 g(nseg_launch), b(64);
  if (dbg && plain)
    hipLaunchKernelGGL((k_wave<T, P, true, true>), g, b, 0, s, parity, segs, inst, buf, drops, part, mask, step, dbg,
                       dbg_inst);
  else if (dbg)
    hipLaunchKernelGGL((k_wave<T, P, true, false>), g, b, 0, s, parity, segs, inst, buf, drops, part, mask, step, dbg,
                       dbg_inst);
  else if (plain)
    hipLaunchKernelGGL((k_wave<T, P, false, true>), g, b, 0, s, parity, segs, inst, buf, drops, part, mask, step,
                       dbg, dbg_inst);
  else
    hipLaunchKernelGGL((k_wave<T, P, false, false>), g, b, 0, s, parity, segs, inst, buf, drops, part, mask, step,
                       dbg, dbg_inst);
  return hipGetLastError();
}

// Launchers of the kernels that touch only the FP fields (instantiated once per arithmetic type T) and of
// those that also touch the populations (once per pair T, P of arithmetic and population storage type).
#define LBM_INSTANTIATE_FIELDS(T)                                                                         \
  template hipError_t launch_fd<T>(hipStream_t, int, int, int, const TileDev*, const InstDev*, T*,        \
                                   const DropDev*, double*, uint64_t*, const int64_t*, double*, int);     \
  template hipError_t launch_cm_partials<T>(hipStream_t, int, int, const TileDev*, const InstDev*, T*,    \
                                            const DropDev*, double*, uint64_t*);
#define LBM_INSTANTIATE_POPS(T, P)                                                                        \
  template hipError_t launch_lb<T, P>(hipStream_t, int, int, int, const TileDev*, const InstDev*, T*,     \
                                      double*, int);                                                      \
  template hipError_t launch_obs<T, P>(hipStream_t, int, int, const TileDev*, const InstDev*, T*,         \
                                       const DropDev*, double*, int);                                     \
  template hipError_t launch_step<T, P>(hipStream_t, int, int, const TileDev*, const InstDev*, T*,        \
                                        const DropDev*, double*, uint64_t*, const int64_t*, double*, int); \
  template hipError_t launch_wave<T, P>(hipStream_t, int, int, const TileDev*, const InstDev*, T*,        \
                                        const DropDev*, double*, uint64_t*, const int64_t*, double*, int, bool);

}  // namespace lbm
