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
// Three launches per step, each one stencil layer deep over dense [ny][nx] planes except where two steps share a
// launch (on the tile with a ring, see k_adj12 and k_adj45):
//   K12 (K1, K2)  adjoint of Eq. (19) (c update, link divergence, production rate) and of the phi update of
//                 Eq. (18) down to the bracket M, then of M (Eq. 18) and of X^{n+1/2} down to phi^{n+1/2}, c^{n+1/2}
//   K3            adjoint of the advection half-step (Eqs. 16-17), then of streaming and collision (Eqs. 10-13)
//                 and of the velocity with half the force (Eq. 11) down to f^n, F
//   K45 (K4, K5)  adjoint of the force (Eq. 14) down to mu_phi, X, phi^n, c^n, then of mu_phi and X (Eqs. 3, 5)
//                 down to phi^n, c^n
#pragma once
#include "lbm_adjoint.h"
#include "lbm_kernels_impl.h"

namespace lbm {
namespace {

// A block of the adjoint kernels covers a tile of ADJ_TILE_X x ADJ_TILE_Y nodes, one wavefront per tile row.
// The planes that a kernel reads across the 3 x 3 neighbourhood are first copied to LDS, the tile with a
// one-node halo (ADJ_HN values per plane, at most two per thread), so that each value is loaded from memory
// once per block instead of once per neighbour.
constexpr int ADJ_THREADS = ADJ_TILE_X * ADJ_TILE_Y;
constexpr int ADJ_HX = ADJ_TILE_X + 2, ADJ_HN = ADJ_HX * (ADJ_TILE_Y + 2);
static_assert(ADJ_TILE_X == 64, "one wavefront per tile row");
static_assert(ADJ_HN <= 2 * ADJ_THREADS, "two staged values per thread");

// Workgroups are dealt to the eight XCDs in turn (workgroup b runs on XCD b mod 8), and each XCD has an L2 of
// its own.  Relabelled so that each XCD takes one contiguous run of the lattice's tiles, a tile's rows above
// and below are mostly read by blocks of the same XCD, from its L2.  A bijection of [0, gridDim.x).
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  const int q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

// This thread's node (x, y) and frame index l, and the plane offsets of the (one or two) values it stages.
// Frame row j + 1, column i + 1 holds node (x0 + i, y0 + j) of the tile at (x0, y0); the halo holds the
// periodic neighbours in x, and in y the periodic neighbours or, with walls, the boundary rows that mirror the
// rows beyond the plates (frame rows past the last lattice row that only nodes outside the lattice read are
// clamped to it).
struct Tile {
  int x, y, l;
  bool valid, two;
  int so[2], sp[2];  // dense ([ny][nx]) and pitched offsets of the staged values
};

__device__ __forceinline__ Tile make_tile(const AdjModel& m, int pitch) {
  const int nbx = (m.nx + ADJ_TILE_X - 1) / ADJ_TILE_X;
  const int b = xcd_block();
  const int by = b / nbx, bx = b - by * nbx;
  const int x0 = bx * ADJ_TILE_X, y0 = by * ADJ_TILE_Y;
  const int tx = threadIdx.x % ADJ_TILE_X, ty = threadIdx.x / ADJ_TILE_X;
  Tile t;
  t.x = x0 + tx;
  t.y = y0 + ty;
  t.l = (ty + 1) * ADJ_HX + tx + 1;
  t.valid = t.x < m.nx && t.y < m.ny;
  t.two = threadIdx.x + ADJ_THREADS < ADJ_HN;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int i = j == 0 || t.two ? threadIdx.x + j * ADJ_THREADS : threadIdx.x;
    const int ly = i / ADJ_HX, lx = i - ly * ADJ_HX;
    const int gx = (x0 + lx - 1 + m.nx) % m.nx;
    int gy = y0 + ly - 1;
    if (m.walls)
      gy = gy < 0 ? 0 : gy >= m.ny ? m.ny - 1 : gy;
    else
      gy = (gy + m.ny) % m.ny;
    t.so[j] = gy * m.nx + gx;
    t.sp[j] = gy * pitch + gx;
  }
  return t;
}

// Copies a plane's values for the tile frame into s; src(dense offset, pitched offset) reads one value.
template <typename T, class S>
__device__ __forceinline__ void stage(T* s, const Tile& t, S src) {
  s[threadIdx.x] = src(t.so[0], t.sp[0]);
  if (t.two) s[threadIdx.x + ADJ_THREADS] = src(t.so[1], t.sp[1]);
}

// 3 x 3 neighbourhood of node (x, y): dense and pitched plane offsets, periodic in x, and in y without walls,
// and s(dx, dy), the index in a staged frame.  With walls a row beyond a plate is the mirror image of the
// boundary row (the forward's ghost rows), and odd(dy) is -1 for such a row: a field that is odd under the
// mirror (u_y in the forward; the adjoint operand of a transposed y-gradient, see below) changes sign there.
struct Nbh {
  int x, y, nx, l;
  int xs[3], ys[3];
  int sg[3];
  __device__ int d(int dx, int dy) const { return ys[dy + 1] * nx + xs[dx + 1]; }
  __device__ int p(int dx, int dy, int pitch) const { return ys[dy + 1] * pitch + xs[dx + 1]; }
  __device__ int s(int dx, int dy) const { return l + dy * ADJ_HX + dx; }
  __device__ int odd(int dy) const { return sg[dy + 1]; }
};

__device__ __forceinline__ Nbh make_nbh(const Tile& t, const AdjModel& m) {
  const int nx = m.nx, ny = m.ny, walls = m.walls;
  Nbh k;
  k.nx = nx;
  k.y = t.y;
  k.x = t.x;
  k.l = t.l;
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

// Transposes of the 9-point operators with the mirror ghost rows of the walls.  On a periodic lattice
// G9x^T = -G9x, G9y^T = -G9y and L9^T = L9.  With walls, the outputs at a boundary row also read the ghost row,
// which is the boundary row itself, and there are no outputs beyond the plate.  Gathering at node j, both
// effects together amount to evaluating the same periodic formula with the adjoint operand continued across
// the plate by its mirror image: even for L9 and G9x (symmetric in y), odd for G9y (antisymmetric in y).
template <typename T, class K, class V>
__device__ __forceinline__ T G9y_T(const K& k, V v) {
  auto w = [&](int dx, int dy) { return T(k.odd(dy)) * v(dx, dy); };
  return G9y<T>(w);
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

// Kernels that need a stencil's result across the 3 x 3 neighbourhood form it on the tile with a one-node ring,
// from their inputs on the tile with a two-node ring (ADJ_N2 values per plane).
constexpr int ADJ_W2 = ADJ_TILE_X + 4, ADJ_N2 = ADJ_W2 * (ADJ_TILE_Y + 4);
static_assert(ADJ_N2 <= 3 * ADJ_THREADS, "three staged values per thread");

// Neighbourhood of a point in the frame with the two-node ring: index l in that frame, and the mirror signs.
struct Nbh2 {
  int l;
  int sg[3];
  __device__ int s(int dx, int dy) const { return l + dy * ADJ_W2 + dx; }
  __device__ int odd(int dy) const { return sg[dy + 1]; }
};

__device__ __forceinline__ Nbh2 make_nbh2(int l, int y, const AdjModel& m) {
  Nbh2 k;
  k.l = l;
  k.sg[0] = m.walls && y == 0 ? -1 : 1;
  k.sg[1] = 1;
  k.sg[2] = m.walls && y == m.ny - 1 ? -1 : 1;
  return k;
}

// This block's tile origin (x0, y0).
__device__ __forceinline__ void tile_origin(const AdjModel& m, int& x0, int& y0) {
  const int nbx = (m.nx + ADJ_TILE_X - 1) / ADJ_TILE_X;
  const int b = xcd_block(), by = b / nbx, bx = b - by * nbx;
  x0 = bx * ADJ_TILE_X;
  y0 = by * ADJ_TILE_Y;
}

// Calls put(i, dense offset, pitched offset) for the values of the frame with the two-node ring that this thread
// stages: periodic images, or with walls the mirrored rows (clamped for lattices of fewer rows than the ring
// reaches; only ring nodes that are not computed read those).
template <class F>
__device__ __forceinline__ void stage2(const AdjModel& m, int pitch, int x0, int y0, F put) {
#pragma unroll
  for (int jj = 0; jj < 3; ++jj) {
    const int i = threadIdx.x + jj * ADJ_THREADS;
    if (i < ADJ_N2) {
      const int ly = i / ADJ_W2, lx = i - ly * ADJ_W2;
      const int gx = (x0 + lx - 2 + 2 * m.nx) % m.nx;
      int gy = y0 + ly - 2;
      if (m.walls) {
        gy = gy < 0 ? -1 - gy : gy >= m.ny ? 2 * m.ny - 1 - gy : gy;
        gy = gy < 0 ? 0 : gy >= m.ny ? m.ny - 1 : gy;
      } else {
        gy = (gy + 2 * m.ny) % m.ny;
      }
      put(i, gy * m.nx + gx, gy * pitch + gx);
    }
  }
}

// With walls, the ring rows beyond a plate take the values of the boundary row (as a plane read at the mirrored
// row gives): copy(i, src) for each such entry i of the one-node-ring frame.  Call after the ring pass, followed
// by a barrier.
template <class F>
__device__ __forceinline__ void ring_ghosts(const AdjModel& m, int y0, F copy) {
  if (!m.walls) return;
  for (int i = threadIdx.x; i < ADJ_HN; i += ADJ_THREADS) {
    const int ly = i / ADJ_HX, lx = i - ly * ADJ_HX;
    const int gy = y0 + ly - 1;
    if (gy >= 0 && gy < m.ny) continue;
    copy(i, ((gy < 0 ? 0 : m.ny - 1) - y0 + 1) * ADJ_HX + lx);
  }
}

// Transpose of the link divergence Div(D c, X) of Eq. (19) at one node, gathered from the links of its
// neighbourhood k: kb (the part multiplying k = D c at the node) and Xb (the part multiplying X).
// Div(k, X)(q) = sum_i W_i (k(q) + k(q + e_i)) (X(q + e_i) - X(q)) / 12, W = 4 on axis links, 1 on diagonals:
// node r enters as q (all links) and as q + e_i of its neighbour q = r - e_i.
template <typename T, class CB, class XH, class KD>
__device__ __forceinline__ void link_adj(CB cb1, XH Xh, KD kD, T& kb, T& Xb) {
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
  kb = (T(4) * kb_ax + kb_dg) * cst<T>(1.0 / 12.0);
  Xb = (T(4) * Xb_ax + Xb_dg) * cst<T>(1.0 / 12.0);
}

// K1 and K2 in one launch.  K1: the adjoint of Eq. (19) (c update, link divergence, production rate) and of
// the phi update of Eq. (18) down to the bracket M; K2: the adjoint of M and X^{n+1/2} down to phi^{n+1/2},
// c^{n+1/2}.  K2 reads K1's M_bar and X^{n+1/2}_bar and the gradients of phi^{n+1/2}, c^{n+1/2} across the 3 x 3
// neighbourhood: they are formed on the tile with a one-node ring.
template <typename T>
__global__ __launch_bounds__(ADJ_THREADS) void k_adj12(AdjModel m, AdjFwd f, AdjPlanes<T> p, const DropDev* drops,
                                                       int ndrop, double* part) {
  __shared__ double red[ADJ_THREADS / 64];
  __shared__ T s_ph[ADJ_N2], s_ch[ADJ_N2], s_pb1[ADJ_N2], s_cb1[ADJ_N2], s_Xh[ADJ_N2];
  __shared__ T s_Mb[ADJ_HN], s_Xhb[ADJ_HN], s_gphx[ADJ_HN], s_gphy[ADJ_HN], s_gchx[ADJ_HN], s_gchy[ADJ_HN];
  const Tile t = make_tile(m, p.pitch);
  int x0, y0;
  tile_origin(m, x0, y0);
  stage2(m, p.pitch, x0, y0, [&](int i, int o, int) {
    s_ph[i] = T(f.ph[o]);
    s_ch[i] = T(f.ch[o]);
    s_pb1[i] = p.pb1[o];
    s_cb1[i] = p.cb1[o];
    s_Xh[i] = T(f.Xh[o]);
  });
  __syncthreads();
  const T D = T(m.D), a = T(m.a), Gamma = T(m.Gamma);
  // on the tile and its one-node ring: M_bar, X^{n+1/2}_bar and the gradients of phi^{n+1/2}, c^{n+1/2}
  for (int i = threadIdx.x; i < ADJ_HN; i += ADJ_THREADS) {
    const int ly = i / ADJ_HX, lx = i - ly * ADJ_HX;
    const int gy = y0 + ly - 1;
    if (m.walls && (gy < 0 || gy >= m.ny)) continue;  // beyond a plate: copied below
    const Nbh2 k = make_nbh2((ly + 1) * ADJ_W2 + lx + 1, (gy + m.ny) % m.ny, m);
    auto ph = [&](int dx, int dy) { return s_ph[k.s(dx, dy)]; };
    auto ch = [&](int dx, int dy) { return s_ch[k.s(dx, dy)]; };
    auto pb1 = [&](int dx, int dy) { return s_pb1[k.s(dx, dy)]; };
    auto cb1 = [&](int dx, int dy) { return s_cb1[k.s(dx, dy)]; };
    auto Xh = [&](int dx, int dy) { return s_Xh[k.s(dx, dy)]; };
    auto kD = [&](int dx, int dy) { return D * ch(dx, dy); };
    s_gphx[i] = G9x<T>(ph);
    s_gphy[i] = G9y<T>(ph);
    s_gchx[i] = G9x<T>(ch);
    s_gchy[i] = G9y<T>(ch);
    // phi^{n+1} = phi^{n+1/2} + Gamma lap9(M)  ->  M_bar = Gamma lap9(phi_bar')
    s_Mb[i] = Gamma * L9<T>(pb1);
    T kb, Xhb;
    link_adj<T>(cb1, Xh, kD, kb, Xhb);
    s_Xhb[i] = Xhb;
  }
  __syncthreads();
  ring_ghosts(m, y0, [&](int i, int src) {
    s_Mb[i] = s_Mb[src];
    s_Xhb[i] = s_Xhb[src];
    s_gphx[i] = s_gphx[src];
    s_gphy[i] = s_gphy[src];
    s_gchx[i] = s_gchx[src];
    s_gchy[i] = s_gchy[src];
  });
  __syncthreads();
  double src = 0.0;
  if (t.valid) {
    const Nbh k = make_nbh(t, m);
    const Nbh2 k2 = make_nbh2((threadIdx.x / ADJ_TILE_X + 2) * ADJ_W2 + threadIdx.x % ADJ_TILE_X + 2, t.y, m);
    const int idx = t.y * m.nx + t.x;
    auto ph = [&](int dx, int dy) { return s_ph[k2.s(dx, dy)]; };
    auto ch = [&](int dx, int dy) { return s_ch[k2.s(dx, dy)]; };
    auto pb1 = [&](int dx, int dy) { return s_pb1[k2.s(dx, dy)]; };
    auto cb1 = [&](int dx, int dy) { return s_cb1[k2.s(dx, dy)]; };
    auto Xh = [&](int dx, int dy) { return s_Xh[k2.s(dx, dy)]; };
    auto kD = [&](int dx, int dy) { return D * ch(dx, dy); };
    // K1 at the node
    const T Mb0 = s_Mb[k.l];
    T phb = pb1(0, 0) + a * Mb0;
    // c^{n+1} = c^{n+1/2} + D lap9(c^{n+1/2}) + Div(D c^{n+1/2}, X^{n+1/2}) - gamma (c^{n+1/2} - c0) + A(n) count
    T kb, Xhb_unused;
    link_adj<T>(cb1, Xh, kD, kb, Xhb_unused);
    const T cb0 = cb1(0, 0);
    T chb = (T(1) - T(m.gamma)) * cb0 + D * L9<T>(cb1) + D * kb;
    // d c^{n+1}(r) / d A0 = min(n, t*) count_n(r)
    if (m.ramp != 0.0 && ndrop > 0) {
      const int cnt = source_count_at((double)k.x, (double)k.y, drops, ndrop, m);
      src = (double)cb0 * m.ramp * (double)cnt;
    }
    // K2: M = a phi^{1/2} + b (phi^n)^3 - B(c^{1/2}) lap9(phi^{1/2}) - B1 grad9 c^{1/2} . grad9 phi^{1/2};
    // X^{1/2} = (B1/2) |grad9 phi^{1/2}|^2
    const T B0 = T(m.B0), B1 = T(m.B1), b = T(m.b);
    auto BM = [&](int dx, int dy) { return (B0 + B1 * ch(dx, dy)) * s_Mb[k.s(dx, dy)]; };
    auto gchxM = [&](int dx, int dy) { const int q = k.s(dx, dy); return s_gchx[q] * s_Mb[q]; };
    auto gchyM = [&](int dx, int dy) { const int q = k.s(dx, dy); return s_gchy[q] * s_Mb[q]; };
    auto gphxX = [&](int dx, int dy) { const int q = k.s(dx, dy); return s_gphx[q] * s_Xhb[q]; };
    auto gphyX = [&](int dx, int dy) { const int q = k.s(dx, dy); return s_gphy[q] * s_Xhb[q]; };
    auto gphxM = [&](int dx, int dy) { const int q = k.s(dx, dy); return s_gphx[q] * s_Mb[q]; };
    auto gphyM = [&](int dx, int dy) { const int q = k.s(dx, dy); return s_gphy[q] * s_Mb[q]; };
    phb = ((phb - L9<T>(BM)) + B1 * (G9x<T>(gchxM) + G9y_T<T>(k, gchyM))) - B1 * (G9x<T>(gphxX) + G9y_T<T>(k, gphyX));
    chb = (chb - B1 * L9<T>(ph) * Mb0) + B1 * (G9x<T>(gphxM) + G9y_T<T>(k, gphyM));
    const T ph0 = p.phi[k.p(0, 0, p.pitch)];
    p.phb[idx] = phb;
    p.chb[idx] = chb;
    p.pb[idx] = T(3) * b * (ph0 * ph0) * Mb0;
  }
  // deterministic per-block partial sum of the A0 contribution, added to the block's running total (steps
  // are taken one after another, so each block's total accumulates in a fixed order)
  for (int o = 32; o > 0; o >>= 1) src += __shfl_xor(src, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = src;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < ADJ_THREADS / 64; ++w) s += red[w];
    part[xcd_block()] += s;
  }
}

template <typename T>
__global__ __launch_bounds__(ADJ_THREADS) void k_adj3(AdjModel m, AdjFwd f, AdjPlanes<T> p) {
  __shared__ T s_ux[ADJ_HN], s_uy[ADJ_HN], s_g[2][ADJ_HN], s_o[2][ADJ_HN];
  const Tile t = make_tile(m, p.pitch);
  stage(s_ux, t, [&](int o, int) { return T(f.ux[o]); });
  stage(s_uy, t, [&](int o, int) { return T(f.uy[o]); });
  stage(s_g[0], t, [&](int, int q) { return p.phi[q]; });
  stage(s_g[1], t, [&](int, int q) { return p.c[q]; });
  stage(s_o[0], t, [&](int o, int) { return p.phb[o]; });
  stage(s_o[1], t, [&](int o, int) { return p.chb[o]; });
  __syncthreads();
  if (!t.valid) return;
  const int N = m.nx * m.ny;
  const Nbh k = make_nbh(t, m);
  const int idx = t.y * m.nx + t.x;
  auto ux = [&](int dx, int dy) { return s_ux[k.s(dx, dy)]; };
  // beyond a plate the forward's advection stencil sees u_y reversed
  auto uy = [&](int dx, int dy) { return T(k.odd(dy)) * s_uy[k.s(dx, dy)]; };
  // With walls the gathered formula below holds as written once ob, g and u_x are continued across a plate by
  // their mirror images and u_y by its negative mirror image (the outputs at a boundary row read the ghost row,
  // and no outputs lie beyond the plate).
  // Advection of Eqs. (16)-(17), o(r) = g - [g divu + ux dgx + uy dgy], divu = (ux(E) - ux(W))/2 +
  // (uy(N) - uy(S))/2, dgx = g - g(W) if ux > 0 else g(E) - g (same in y); gathered at node q.
  T uxb = T(0), uyb = T(0);
  T gb[2];
#pragma unroll
  for (int which = 0; which < 2; ++which) {
    auto G = [&](int dx, int dy) { return s_g[which][k.s(dx, dy)]; };
    auto O = [&](int dx, int dy) { return s_o[which][k.s(dx, dy)]; };
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

// K4 and K5 in one launch.  The adjoint of the force (K4) gives mu_bar and X_bar, which the adjoint of mu_phi and
// X (K5) reads at the 3 x 3 neighbourhood, as it reads the gradients of phi^n, c^n: these are computed on the tile
// with a one-node ring and kept in LDS, from F_bar, phi and c on the tile with a two-node ring.  A ring node takes
// the values of the node it stands for (its periodic image; with walls, a ring row beyond a plate takes the
// boundary row's, as a plane read at the mirrored row gives).  K4's update of phi_bar and c_bar at the tile comes
// first, then K5's.
template <typename T>
__global__ __launch_bounds__(ADJ_THREADS) void k_adj45(AdjModel m, AdjFwd f, AdjPlanes<T> p) {
  __shared__ T s_Fxb[ADJ_N2], s_Fyb[ADJ_N2], s_phi[ADJ_N2], s_c[ADJ_N2];
  __shared__ T s_mub[ADJ_HN], s_Xb[ADJ_HN];
  // the gradients of phi^n, c^n; mu and X, which only K4's update at the tile reads, before the ring pass, occupy
  // two of them until then (43 KB of LDS per workgroup would leave three workgroups per compute unit, 36 KB four)
  __shared__ T s_g[4][ADJ_HN];
  T* const s_gpx = s_g[0];
  T* const s_gpy = s_g[1];
  T* const s_gcx = s_g[2];
  T* const s_gcy = s_g[3];
  T* const s_mu = s_g[2];
  T* const s_X = s_g[3];
  const Tile t = make_tile(m, p.pitch);
  int x0, y0;
  tile_origin(m, x0, y0);
  stage2(m, p.pitch, x0, y0, [&](int i, int o, int q) {
    s_Fxb[i] = p.Fxb[o];
    s_Fyb[i] = p.Fyb[o];
    s_phi[i] = p.phi[q];
    s_c[i] = p.c[q];
  });
  stage(s_mu, t, [&](int o, int) { return T(f.mu[o]); });
  stage(s_X, t, [&](int o, int) { return T(f.X[o]); });
  __syncthreads();
  const Nbh k = make_nbh(t, m);
  const Nbh2 k2 = make_nbh2((threadIdx.x / ADJ_TILE_X + 2) * ADJ_W2 + threadIdx.x % ADJ_TILE_X + 2, t.y, m);
  const int idx = t.y * m.nx + t.x;
  auto Fxb = [&](int dx, int dy) { return s_Fxb[k2.s(dx, dy)]; };
  auto Fyb = [&](int dx, int dy) { return s_Fyb[k2.s(dx, dy)]; };
  T pb = T(0), cb = T(0), fx = T(0), fy = T(0);
  if (t.valid) {  // K4: F = -phi grad9 mu - grad9 c - c grad9 X (Eq. 14)
    auto mu = [&](int dx, int dy) { return s_mu[k.s(dx, dy)]; };
    auto X = [&](int dx, int dy) { return s_X[k.s(dx, dy)]; };
    fx = Fxb(0, 0);
    fy = Fyb(0, 0);
    pb = p.pb[idx];
    cb = p.cb[idx];
    pb -= fx * G9x<T>(mu) + fy * G9y<T>(mu);
    cb += (G9x<T>(Fxb) + G9y_T<T>(k2, Fyb)) - (fx * G9x<T>(X) + fy * G9y<T>(X));
  }
  __syncthreads();
  // mu_bar, X_bar (Eq. 14 transposed) and the gradients of phi^n, c^n on the tile and its one-node ring
  for (int i = threadIdx.x; i < ADJ_HN; i += ADJ_THREADS) {
    const int ly = i / ADJ_HX, lx = i - ly * ADJ_HX;
    const int gy = y0 + ly - 1;
    if (m.walls && (gy < 0 || gy >= m.ny)) continue;  // beyond a plate: copied below
    const Nbh2 k = make_nbh2((ly + 1) * ADJ_W2 + lx + 1, (gy + m.ny) % m.ny, m);
    auto phFx = [&](int dx, int dy) { const int q = k.s(dx, dy); return s_phi[q] * s_Fxb[q]; };
    auto phFy = [&](int dx, int dy) { const int q = k.s(dx, dy); return s_phi[q] * s_Fyb[q]; };
    auto cFx = [&](int dx, int dy) { const int q = k.s(dx, dy); return s_c[q] * s_Fxb[q]; };
    auto cFy = [&](int dx, int dy) { const int q = k.s(dx, dy); return s_c[q] * s_Fyb[q]; };
    auto phi = [&](int dx, int dy) { return s_phi[k.s(dx, dy)]; };
    auto cc = [&](int dx, int dy) { return s_c[k.s(dx, dy)]; };
    s_mub[i] = G9x<T>(phFx) + G9y_T<T>(k, phFy);
    s_Xb[i] = G9x<T>(cFx) + G9y_T<T>(k, cFy);
    s_gpx[i] = G9x<T>(phi);
    s_gpy[i] = G9y<T>(phi);
    s_gcx[i] = G9x<T>(cc);
    s_gcy[i] = G9y<T>(cc);
  }
  __syncthreads();
  ring_ghosts(m, y0, [&](int i, int src) {
    s_mub[i] = s_mub[src];
    s_Xb[i] = s_Xb[src];
    s_gpx[i] = s_gpx[src];
    s_gpy[i] = s_gpy[src];
    s_gcx[i] = s_gcx[src];
    s_gcy[i] = s_gcy[src];
  });
  __syncthreads();
  if (!t.valid) return;
  // K5: mu = a phi + b phi^3 - B(c) lap9 phi - B1 grad9 phi . grad9 c;  X = (B1/2) |grad9 phi|^2 (Eqs. 3, 5)
  const T a = T(m.a), b3 = T(m.b), B0 = T(m.B0), B1 = T(m.B1);
  auto BMu = [&](int dx, int dy) { return (B0 + B1 * s_c[k2.s(dx, dy)]) * s_mub[k.s(dx, dy)]; };
  auto gcxMu = [&](int dx, int dy) { const int q = k.s(dx, dy); return s_gcx[q] * s_mub[q]; };
  auto gcyMu = [&](int dx, int dy) { const int q = k.s(dx, dy); return s_gcy[q] * s_mub[q]; };
  auto gpxMu = [&](int dx, int dy) { const int q = k.s(dx, dy); return s_gpx[q] * s_mub[q]; };
  auto gpyMu = [&](int dx, int dy) { const int q = k.s(dx, dy); return s_gpy[q] * s_mub[q]; };
  auto gpxX = [&](int dx, int dy) { const int q = k.s(dx, dy); return s_gpx[q] * s_Xb[q]; };
  auto gpyX = [&](int dx, int dy) { const int q = k.s(dx, dy); return s_gpy[q] * s_Xb[q]; };
  auto phi = [&](int dx, int dy) { return s_phi[k2.s(dx, dy)]; };
  const T ph = phi(0, 0), mb = s_mub[k.l];
  pb += (((a + T(3) * b3 * (ph * ph)) * mb - L9<T>(BMu)) + B1 * (G9x<T>(gcxMu) + G9y_T<T>(k, gcyMu))) -
        B1 * (G9x<T>(gpxX) + G9y_T<T>(k, gpyX));
  cb += B1 * (G9x<T>(gpxMu) + G9y_T<T>(k, gpyMu)) - B1 * L9<T>(phi) * mb;
  p.pb[idx] = pb;
  p.cb[idx] = cb;
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
  const int nb = adj_blocks(m.nx, m.ny);
  hipLaunchKernelGGL((k_adj12<T>), dim3(nb), dim3(ADJ_THREADS), 0, s, m, f, p, drops_n, ndrop, part);
  hipLaunchKernelGGL((k_adj3<T>), dim3(nb), dim3(ADJ_THREADS), 0, s, m, f, p);
  hipLaunchKernelGGL((k_adj45<T>), dim3(nb), dim3(ADJ_THREADS), 0, s, m, f, p);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_seed(hipStream_t s, int pass, const AdjModel& m, const T* phi, int pitch,
                               const DropDev* drops_prev, int ndrop, int drop, double delta, double sw, T* fb,
                               T* pb, T* cb, double* part) {
  const int nb = adj_blocks(m.nx, m.ny);
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
