// Reverse-mode (adjoint) kernels of one timestep of the hybrid scheme (Sec. 2, Eqs. 3, 5, 10-19) on a lattice
// periodic in x, and in y or between two plates: given the adjoint (f_bar, phi_bar, c_bar) of the state at n + 1
// and the forward intermediates of step n, they produce the adjoint of the state at n and the step's
// contribution to the derivative with respect to the production rate A0.
//
// The discrete forward step is differentiated as written (the exact transpose of each operation).  On a
// periodic lattice the 9-point gradient is antisymmetric and the 9-point Laplacian symmetric, so their
// transposes are -grad9 and lap9; with walls the mirror ghost rows enter as described at Nbh and G9y_T.
// Held fixed (non-differentiable): the membership of each node in the production disks, the upwind side chosen
// by the sign of u in Eqs. (16)-(17), and the droplet masks.
//
// Five launches per step, each one stencil layer deep over dense [ny][nx] planes:
//   K1  gradient planes of the forward fields; adjoint of Eq. (19) (c update, link divergence, production
//       rate) and of the phi update of Eq. (18) down to the bracket M
//   K2  adjoint of M (Eq. 18) and of X^{n+1/2} down to phi^{n+1/2}, c^{n+1/2}
//   K3  adjoint of the advection half-step (Eqs. 16-17), then of streaming and collision (Eqs. 10-13)
//       and of the velocity with half the force (Eq. 11) down to f^n, F
//   K4  adjoint of the force (Eq. 14) down to mu_phi, X, phi^n, c^n
//   K5  adjoint of mu_phi and X (Eqs. 3, 5) down to phi^n, c^n
#pragma once
#include "lbm_adjoint.h"
#include "lbm_kernels_impl.h"

namespace lbm {
namespace {

constexpr int ADJ_THREADS = 256;  // adj_blocks() in lbm_adjoint.h assumes this size

// 3 x 3 neighbourhood of node (x, y) of a dense plane: periodic in x, and in y without walls.  With walls a
// row beyond a plate is the mirror image of the boundary row (the forward's ghost rows), and odd(dy) is -1 for
// such a row: a field that is odd under the mirror (u_y in the forward; the adjoint operand of a transposed
// y-gradient, see below) changes sign there.
struct Nbh {
  int x, y, nx;
  int xs[3], ys[3];
  int sg[3];
  __device__ int d(int dx, int dy) const { return ys[dy + 1] * nx + xs[dx + 1]; }
  __device__ int p(int dx, int dy, int pitch) const { return ys[dy + 1] * pitch + xs[dx + 1]; }
  __device__ int odd(int dy) const { return sg[dy + 1]; }
};

__device__ __forceinline__ Nbh make_nbh(int idx, int nx, int ny, int walls) {
  Nbh k;
  k.nx = nx;
  k.y = idx / nx;
  k.x = idx - k.y * nx;
  k.xs[0] = k.x == 0 ? nx - 1 : k.x - 1;
  k.xs[1] = k.x;
  k.xs[2] = k.x == nx - 1 ? 0 : k.x + 1;
  const bool bot = k.y == 0, top = k.y == ny - 1;
  k.ys[0] = bot ? (walls ? 0 : ny - 1) : k.y - 1;
  k.ys[1] = k.y;
  k.ys[2] = top ? (walls ? ny - 1 : 0) : k.y + 1;
  k.sg[0] = walls && bot ? -1 : 1;
  k.sg[1] = 1;
  k.sg[2] = walls && top ? -1 : 1;
  return k;
}

// Transposes of the 9-point operators with the mirror ghost rows of the walls.  On a periodic lattice
// G9x^T = -G9x, G9y^T = -G9y and L9^T = L9.  With walls, the outputs at a boundary row also read the ghost row,
// which is the boundary row itself, and there are no outputs beyond the plate.  Gathering at node j, both
// effects together amount to evaluating the same periodic formula with the adjoint operand continued across
// the plate by its mirror image: even for L9 and G9x (symmetric in y), odd for G9y (antisymmetric in y).
template <typename T, class V>
__device__ __forceinline__ T G9y_T(const Nbh& k, V v) {
  auto w = [&](int dx, int dy) { return T(k.odd(dy)) * v(dx, dy); };
  return G9y<T>(w);
}

// 9-point stencils of a value function v(dx, dy), grouped as in the forward kernels.
template <typename T, class V>
__device__ __forceinline__ T G9x(V v) {
  return (T(4) * (v(1, 0) - v(-1, 0)) + ((v(1, 1) - v(-1, 1)) + (v(1, -1) - v(-1, -1)))) * cst<T>(1.0 / 12.0);
}
template <typename T, class V>
__device__ __forceinline__ T G9y(V v) {
  return (T(4) * (v(0, 1) - v(0, -1)) + ((v(1, 1) - v(1, -1)) + (v(-1, 1) - v(-1, -1)))) * cst<T>(1.0 / 12.0);
}
template <typename T, class V>
__device__ __forceinline__ T L9(V v) {
  return (T(4) * ((v(1, 0) + v(-1, 0)) + (v(0, 1) + v(0, -1))) + ((v(1, 1) + v(-1, 1)) + (v(1, -1) + v(-1, -1))) -
          T(20) * v(0, 0)) *
         cst<T>(1.0 / 6.0);
}

// Number of active production disks containing node (x, y) (the forward's source count at step n).
__device__ int source_count_at(double x, double y, const DropDev* drops, int ndrop, const AdjModel& m) {
  int cnt = 0;
  for (int k = 0; k < ndrop; ++k) {
    const DropDev d = drops[k];
    if (!d.active) continue;
    const double px = d.x + (d.R - d.Rs) * d.ex, py = d.y + (d.R - d.Rs) * d.ey;
    const double dx = minimg(x - px, (double)m.nx), dy = minimg(y - py, m.yper);
    if (dx * dx + dy * dy <= d.Rs * d.Rs) ++cnt;
  }
  return cnt;
}

template <typename T>
__global__ __launch_bounds__(ADJ_THREADS) void k_adj1(AdjModel m, AdjFwd f, AdjPlanes<T> p, const DropDev* drops,
                                                      int ndrop, double* part) {
  __shared__ double red[ADJ_THREADS / 64];
  const int N = m.nx * m.ny;
  const int idx = blockIdx.x * ADJ_THREADS + threadIdx.x;
  double src = 0.0;
  if (idx < N) {
    const Nbh k = make_nbh(idx, m.nx, m.ny, m.walls);
    const int pitch = p.pitch;
    auto phi = [&](int dx, int dy) { return p.phi[k.p(dx, dy, pitch)]; };
    auto cc = [&](int dx, int dy) { return p.c[k.p(dx, dy, pitch)]; };
    auto ph = [&](int dx, int dy) { return T(f.ph[k.d(dx, dy)]); };
    auto ch = [&](int dx, int dy) { return T(f.ch[k.d(dx, dy)]); };
    auto mu = [&](int dx, int dy) { return T(f.mu[k.d(dx, dy)]); };
    auto X = [&](int dx, int dy) { return T(f.X[k.d(dx, dy)]); };
    // gradient planes of the forward fields (used by the later launches at neighbouring nodes)
    p.gpx[idx] = G9x<T>(phi);
    p.gpy[idx] = G9y<T>(phi);
    p.gcx[idx] = G9x<T>(cc);
    p.gcy[idx] = G9y<T>(cc);
    p.lp[idx] = L9<T>(phi);
    p.gphx[idx] = G9x<T>(ph);
    p.gphy[idx] = G9y<T>(ph);
    p.gchx[idx] = G9x<T>(ch);
    p.gchy[idx] = G9y<T>(ch);
    p.lph[idx] = L9<T>(ph);
    p.gmx[idx] = G9x<T>(mu);
    p.gmy[idx] = G9y<T>(mu);
    p.gXx[idx] = G9x<T>(X);
    p.gXy[idx] = G9y<T>(X);

    const T D = T(m.D), a = T(m.a);
    auto pb1 = [&](int dx, int dy) { return p.pb1[k.d(dx, dy)]; };
    auto cb1 = [&](int dx, int dy) { return p.cb1[k.d(dx, dy)]; };
    auto Xh = [&](int dx, int dy) { return T(f.Xh[k.d(dx, dy)]); };
    auto kD = [&](int dx, int dy) { return D * T(f.ch[k.d(dx, dy)]); };
    // phi^{n+1} = phi^{n+1/2} + Gamma lap9(M)  ->  M_bar = Gamma lap9(phi_bar')
    const T Mb = T(m.Gamma) * L9<T>(pb1);
    p.Mb[idx] = Mb;
    p.phb[idx] = pb1(0, 0) + a * Mb;  // the rest of phi_bar^{n+1/2} needs M_bar at the neighbours
    // c^{n+1} = c^{n+1/2} + D lap9(c^{n+1/2}) + Div(D c^{n+1/2}, X^{n+1/2}) - gamma (c^{n+1/2} - c0) + A(n) count
    // Div(k, X)(q) = sum_i W_i (k(q) + k(q + e_i)) (X(q + e_i) - X(q)) / 12, W = 4 on axis links, 1 on diagonals:
    // node r enters as q (all links) and as q + e_i of its neighbour q = r - e_i.
    const int EXs[8] = {1, 0, -1, 0, 1, -1, -1, 1}, EYs[8] = {0, 1, 0, -1, 1, 1, -1, -1};
    T kb_ax = T(0), kb_dg = T(0), Xb_ax = T(0), Xb_dg = T(0);
    const T cb0 = cb1(0, 0), Xh0 = Xh(0, 0), k0 = kD(0, 0);
    for (int i = 0; i < 8; ++i) {
      const int ex = EXs[i], ey = EYs[i];
      const T cbm = cb1(-ex, -ey);
      const T tk = cb0 * (Xh(ex, ey) - Xh0) + cbm * (Xh0 - Xh(-ex, -ey));
      const T tX = cbm * (kD(-ex, -ey) + k0) - cb0 * (k0 + kD(ex, ey));
      if (i < 4) {
        kb_ax += tk;
        Xb_ax += tX;
      } else {
        kb_dg += tk;
        Xb_dg += tX;
      }
    }
    const T kb = (T(4) * kb_ax + kb_dg) * cst<T>(1.0 / 12.0);
    p.Xhb[idx] = (T(4) * Xb_ax + Xb_dg) * cst<T>(1.0 / 12.0);
    p.chb[idx] = (T(1) - T(m.gamma)) * cb0 + D * L9<T>(cb1) + D * kb;
    // d c^{n+1}(r) / d A0 = min(n, t*) count_n(r)
    if (m.ramp != 0.0 && ndrop > 0) {
      const int cnt = source_count_at((double)k.x, (double)k.y, drops, ndrop, m);
      src = (double)cb0 * m.ramp * (double)cnt;
    }
  }
  // deterministic per-block partial sum of the A0 contribution, added to the block's running total (steps
  // are taken one after another, so each block's total accumulates in a fixed order)
  for (int o = 32; o > 0; o >>= 1) src += __shfl_xor(src, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = src;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < ADJ_THREADS / 64; ++w) s += red[w];
    part[blockIdx.x] += s;
  }
}

template <typename T>
__global__ __launch_bounds__(ADJ_THREADS) void k_adj2(AdjModel m, AdjFwd f, AdjPlanes<T> p) {
  const int N = m.nx * m.ny;
  const int idx = blockIdx.x * ADJ_THREADS + threadIdx.x;
  if (idx >= N) return;
  const Nbh k = make_nbh(idx, m.nx, m.ny, m.walls);
  const T B0 = T(m.B0), B1 = T(m.B1), b = T(m.b);
  auto BM = [&](int dx, int dy) { const int q = k.d(dx, dy); return (B0 + B1 * T(f.ch[q])) * p.Mb[q]; };
  auto gchxM = [&](int dx, int dy) { const int q = k.d(dx, dy); return p.gchx[q] * p.Mb[q]; };
  auto gchyM = [&](int dx, int dy) { const int q = k.d(dx, dy); return p.gchy[q] * p.Mb[q]; };
  auto gphxX = [&](int dx, int dy) { const int q = k.d(dx, dy); return p.gphx[q] * p.Xhb[q]; };
  auto gphyX = [&](int dx, int dy) { const int q = k.d(dx, dy); return p.gphy[q] * p.Xhb[q]; };
  auto gphxM = [&](int dx, int dy) { const int q = k.d(dx, dy); return p.gphx[q] * p.Mb[q]; };
  auto gphyM = [&](int dx, int dy) { const int q = k.d(dx, dy); return p.gphy[q] * p.Mb[q]; };
  // M = a phi^{1/2} + b (phi^n)^3 - B(c^{1/2}) lap9(phi^{1/2}) - B1 grad9 c^{1/2} . grad9 phi^{1/2};
  // X^{1/2} = (B1/2) |grad9 phi^{1/2}|^2
  p.phb[idx] = ((p.phb[idx] - L9<T>(BM)) + B1 * (G9x<T>(gchxM) + G9y_T<T>(k, gchyM))) -
               B1 * (G9x<T>(gphxX) + G9y_T<T>(k, gphyX));
  p.chb[idx] = (p.chb[idx] - B1 * p.lph[idx] * p.Mb[idx]) + B1 * (G9x<T>(gphxM) + G9y_T<T>(k, gphyM));
  const T ph0 = p.phi[k.p(0, 0, p.pitch)];
  p.pb[idx] = T(3) * b * (ph0 * ph0) * p.Mb[idx];
}

template <typename T>
__global__ __launch_bounds__(ADJ_THREADS) void k_adj3(AdjModel m, AdjFwd f, AdjPlanes<T> p) {
  const int N = m.nx * m.ny;
  const int idx = blockIdx.x * ADJ_THREADS + threadIdx.x;
  if (idx >= N) return;
  const Nbh k = make_nbh(idx, m.nx, m.ny, m.walls);
  const int pitch = p.pitch;
  auto ux = [&](int dx, int dy) { return T(f.ux[k.d(dx, dy)]); };
  // beyond a plate the forward's advection stencil sees u_y reversed
  auto uy = [&](int dx, int dy) { return T(k.odd(dy)) * T(f.uy[k.d(dx, dy)]); };
  // With walls the gathered formula below holds as written once ob, g and u_x are continued across a plate by
  // their mirror images and u_y by its negative mirror image (the outputs at a boundary row read the ghost row,
  // and no outputs lie beyond the plate).
  // Advection of Eqs. (16)-(17), o(r) = g - [g divu + ux dgx + uy dgy], divu = (ux(E) - ux(W))/2 +
  // (uy(N) - uy(S))/2, dgx = g - g(W) if ux > 0 else g(E) - g (same in y); gathered at node q.
  T uxb = T(0), uyb = T(0);
  T gb[2];
  for (int which = 0; which < 2; ++which) {
    const T* g = which == 0 ? p.phi : p.c;
    const T* ob = which == 0 ? p.phb : p.chb;
    auto G = [&](int dx, int dy) { return g[k.p(dx, dy, pitch)]; };
    auto O = [&](int dx, int dy) { return ob[k.d(dx, dy)]; };
    const T u0 = ux(0, 0), v0 = uy(0, 0), g0 = G(0, 0), o0 = O(0, 0);
    const T divu = T(0.5) * (ux(1, 0) - ux(-1, 0)) + T(0.5) * (uy(0, 1) - uy(0, -1));
    const T sx = u0 > T(0) ? T(1) : T(-1), sy = v0 > T(0) ? T(1) : T(-1);
    const T dgx = u0 > T(0) ? g0 - G(-1, 0) : G(1, 0) - g0;
    const T dgy = v0 > T(0) ? g0 - G(0, -1) : G(0, 1) - g0;
    T acc = o0 * (((T(1) - divu) - u0 * sx) - v0 * sy);
    {
      const T ue = ux(1, 0), uw = ux(-1, 0), vn = uy(0, 1), vs = uy(0, -1);
      acc += O(1, 0) * (ue > T(0) ? ue : T(0));
      acc += O(-1, 0) * (uw > T(0) ? T(0) : -uw);
      acc += O(0, 1) * (vn > T(0) ? vn : T(0));
      acc += O(0, -1) * (vs > T(0) ? T(0) : -vs);
    }
    gb[which] = acc;
    uxb += (-(o0 * dgx) - T(0.5) * (O(-1, 0) * G(-1, 0))) + T(0.5) * (O(1, 0) * G(1, 0));
    uyb += (-(o0 * dgy) - T(0.5) * (O(0, -1) * G(0, -1))) + T(0.5) * (O(0, 1) * G(0, 1));
  }
  p.pb[idx] += gb[0];
  T cbv = gb[1];

  // Streaming (Eq. 10): f^{n+1}_i(r + e_i) = f*_i(r)  ->  f*_bar_i(r) = f_bar'_i(r + e_i).  With walls, a
  // population streamed into a plate returns to r reversed: f^{n+1}_opp(i)(r) = f*_i(r)  ->  f*_bar_i(r) =
  // f_bar'_opp(i)(r).
  const int EX9[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1}, EY9[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const int OPP9[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  const T W9[9] = {cst<T>(4.0 / 9.0),  cst<T>(1.0 / 9.0),  cst<T>(1.0 / 9.0),  cst<T>(1.0 / 9.0), cst<T>(1.0 / 9.0),
                   cst<T>(1.0 / 36.0), cst<T>(1.0 / 36.0), cst<T>(1.0 / 36.0), cst<T>(1.0 / 36.0)};
  const T nn = T(f.n[idx]), u = ux(0, 0), v = uy(0, 0), Fx = T(f.Fx[idx]), Fy = T(f.Fy[idx]);
  const T omega = T(m.omega), coef = T(m.coef);
  const T usq = u * u + v * v;
  T nb = T(0), ub = uxb, vb = uyb, Fxb = T(0), Fyb = T(0), fsb[9];
  for (int i = 0; i < 9; ++i) {
    const T ex = T(EX9[i]), ey = T(EY9[i]);
    const int ty = k.y + EY9[i];
    fsb[i] = m.walls && (ty < 0 || ty >= m.ny) ? p.fb1[(size_t)OPP9[i] * N + idx]
                                               : p.fb1[(size_t)i * N + k.d(EX9[i], EY9[i])];
    const T eu = ex * u + ey * v, eF = ex * Fx + ey * Fy;
    // f* = (1 - omega) f + omega feq(n, u) + Fi(u, F) (Eqs. 10, 12, 13)
    const T feq = W9[i] * nn * (((T(1) + T(3) * eu) + T(4.5) * eu * eu) - T(1.5) * usq);
    nb += fsb[i] * omega * feq / nn;
    const T wn = W9[i] * nn;
    ub += fsb[i] * (omega * wn * ((T(3) * ex + T(9) * eu * ex) - T(3) * u) +
                    coef * W9[i] * (T(9) * ex * eF - T(3) * Fx));
    vb += fsb[i] * (omega * wn * ((T(3) * ey + T(9) * eu * ey) - T(3) * v) +
                    coef * W9[i] * (T(9) * ey * eF - T(3) * Fy));
    Fxb += fsb[i] * coef * W9[i] * (T(3) * (ex - u) + T(9) * eu * ex);
    Fyb += fsb[i] * coef * W9[i] * (T(3) * (ey - v) + T(9) * eu * ey);
  }
  // u = (m + F/2) / n (Eq. 11), n = sum f, m = sum f e
  const T mxb = ub / nn, myb = vb / nn;
  Fxb += T(0.5) * mxb;
  Fyb += T(0.5) * myb;
  nb -= (ub * u + vb * v) / nn;
  for (int i = 0; i < 9; ++i)
    p.fb[(size_t)i * N + idx] = ((T(1) - omega) * fsb[i] + nb) + (T(EX9[i]) * mxb + T(EY9[i]) * myb);
  p.Fxb[idx] = Fxb;
  p.Fyb[idx] = Fyb;
  p.cb[idx] = cbv;
}

template <typename T>
__global__ __launch_bounds__(ADJ_THREADS) void k_adj4(AdjModel m, AdjPlanes<T> p) {
  const int N = m.nx * m.ny;
  const int idx = blockIdx.x * ADJ_THREADS + threadIdx.x;
  if (idx >= N) return;
  const Nbh k = make_nbh(idx, m.nx, m.ny, m.walls);
  const int pitch = p.pitch;
  // F = -phi grad9 mu - grad9 c - c grad9 X (Eq. 14)
  auto Fxb = [&](int dx, int dy) { return p.Fxb[k.d(dx, dy)]; };
  auto Fyb = [&](int dx, int dy) { return p.Fyb[k.d(dx, dy)]; };
  auto phFx = [&](int dx, int dy) { return p.phi[k.p(dx, dy, pitch)] * p.Fxb[k.d(dx, dy)]; };
  auto phFy = [&](int dx, int dy) { return p.phi[k.p(dx, dy, pitch)] * p.Fyb[k.d(dx, dy)]; };
  auto cFx = [&](int dx, int dy) { return p.c[k.p(dx, dy, pitch)] * p.Fxb[k.d(dx, dy)]; };
  auto cFy = [&](int dx, int dy) { return p.c[k.p(dx, dy, pitch)] * p.Fyb[k.d(dx, dy)]; };
  const T fx = p.Fxb[idx], fy = p.Fyb[idx];
  p.pb[idx] -= fx * p.gmx[idx] + fy * p.gmy[idx];
  p.cb[idx] += (G9x<T>(Fxb) + G9y_T<T>(k, Fyb)) - (fx * p.gXx[idx] + fy * p.gXy[idx]);
  p.mub[idx] = G9x<T>(phFx) + G9y_T<T>(k, phFy);
  p.Xb[idx] = G9x<T>(cFx) + G9y_T<T>(k, cFy);
}

template <typename T>
__global__ __launch_bounds__(ADJ_THREADS) void k_adj5(AdjModel m, AdjPlanes<T> p) {
  const int N = m.nx * m.ny;
  const int idx = blockIdx.x * ADJ_THREADS + threadIdx.x;
  if (idx >= N) return;
  const Nbh k = make_nbh(idx, m.nx, m.ny, m.walls);
  const int pitch = p.pitch;
  const T a = T(m.a), b = T(m.b), B0 = T(m.B0), B1 = T(m.B1);
  // mu = a phi + b phi^3 - B(c) lap9 phi - B1 grad9 phi . grad9 c;  X = (B1/2) |grad9 phi|^2 (Eqs. 3, 5)
  auto BMu = [&](int dx, int dy) { return (B0 + B1 * p.c[k.p(dx, dy, pitch)]) * p.mub[k.d(dx, dy)]; };
  auto gcxMu = [&](int dx, int dy) { const int q = k.d(dx, dy); return p.gcx[q] * p.mub[q]; };
  auto gcyMu = [&](int dx, int dy) { const int q = k.d(dx, dy); return p.gcy[q] * p.mub[q]; };
  auto gpxMu = [&](int dx, int dy) { const int q = k.d(dx, dy); return p.gpx[q] * p.mub[q]; };
  auto gpyMu = [&](int dx, int dy) { const int q = k.d(dx, dy); return p.gpy[q] * p.mub[q]; };
  auto gpxX = [&](int dx, int dy) { const int q = k.d(dx, dy); return p.gpx[q] * p.Xb[q]; };
  auto gpyX = [&](int dx, int dy) { const int q = k.d(dx, dy); return p.gpy[q] * p.Xb[q]; };
  const T ph = p.phi[k.p(0, 0, pitch)], mb = p.mub[idx];
  p.pb[idx] += (((a + T(3) * b * (ph * ph)) * mb - L9<T>(BMu)) + B1 * (G9x<T>(gcxMu) + G9y_T<T>(k, gcyMu))) -
               B1 * (G9x<T>(gpxX) + G9y_T<T>(k, gpyX));
  p.cb[idx] += B1 * (G9x<T>(gpxMu) + G9y_T<T>(k, gpyMu)) - B1 * p.lp[idx] * mb;
}

template <typename T>
__global__ __launch_bounds__(ADJ_THREADS) void k_adj_seed(int pass, AdjModel m, const T* phi, int pitch,
                                                          const DropDev* drops, int ndrop, int drop, double delta,
                                                          double sw, T* fb, T* pb, T* cb, double* part) {
  __shared__ double red[ADJ_THREADS / 64];
  const int N = m.nx * m.ny;
  const int idx = blockIdx.x * ADJ_THREADS + threadIdx.x;
  double s = 0.0;
  if (idx < N) {
    const int y = idx / m.nx, x = idx - y * m.nx;
    const double v = (double)phi[(int64_t)y * pitch + x];
    int best = -1;
    double bd = 0.0, bdx = 0.0;
    if (v >= 0.0) {
      for (int q = 0; q < ndrop; ++q) {
        const double dx = minimg((double)x - drops[q].x, (double)m.nx), dy = minimg((double)y - drops[q].y, m.yper);
        const double d2 = dx * dx + dy * dy;
        if (best < 0 || d2 < bd) {
          best = q;
          bd = d2;
          bdx = dx;
        }
      }
    }
    const bool in = best == drop;
    if (pass == 0) {
      s = in ? v : 0.0;
    } else {
      // x_CM^N = x_CM^{N-1} + sum phi dx / sum phi over the droplet's nodes: d/d phi = (dx - delta) / sw
      pb[idx] = in ? T((bdx - delta) / sw) : T(0);
      cb[idx] = T(0);
      for (int i = 0; i < 9; ++i) fb[(size_t)i * N + idx] = T(0);
    }
  }
  if (pass == 0) {
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < ADJ_THREADS / 64; ++w) t += red[w];
      part[blockIdx.x] = t;
    }
  }
}

}  // namespace

template <typename T>
hipError_t launch_adjoint_step(hipStream_t s, const AdjModel& m, const AdjFwd& f, const AdjPlanes<T>& p,
                               const DropDev* drops_n, int ndrop, double* part) {
  const int nb = adj_blocks((int64_t)m.nx * m.ny);
  hipLaunchKernelGGL((k_adj1<T>), dim3(nb), dim3(ADJ_THREADS), 0, s, m, f, p, drops_n, ndrop, part);
  hipLaunchKernelGGL((k_adj2<T>), dim3(nb), dim3(ADJ_THREADS), 0, s, m, f, p);
  hipLaunchKernelGGL((k_adj3<T>), dim3(nb), dim3(ADJ_THREADS), 0, s, m, f, p);
  hipLaunchKernelGGL((k_adj4<T>), dim3(nb), dim3(ADJ_THREADS), 0, s, m, p);
  hipLaunchKernelGGL((k_adj5<T>), dim3(nb), dim3(ADJ_THREADS), 0, s, m, p);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_seed(hipStream_t s, int pass, const AdjModel& m, const T* phi, int pitch,
                               const DropDev* drops_prev, int ndrop, int drop, double delta, double sw, T* fb,
                               T* pb, T* cb, double* part) {
  const int nb = adj_blocks((int64_t)m.nx * m.ny);
  hipLaunchKernelGGL((k_adj_seed<T>), dim3(nb), dim3(ADJ_THREADS), 0, s, pass, m, phi, pitch, drops_prev, ndrop, drop,
                     delta, sw, fb, pb, cb, part);
  return hipGetLastError();
}

#define LBM_INSTANTIATE_ADJOINT(T)                                                                           \
  template hipError_t launch_adjoint_step<T>(hipStream_t, const AdjModel&, const AdjFwd&, const AdjPlanes<T>&, \
                                             const DropDev*, int, double*);                                 \
  template hipError_t launch_adjoint_seed<T>(hipStream_t, int, const AdjModel&, const T*, int, const DropDev*, \
                                             int, int, double, double, T*, T*, T*, double*);

}  // namespace lbm
