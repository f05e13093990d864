// HIP kernels of the two-component D3Q19 Shan-Chen step and its support
// (initial state, population import/export, moments, conserved totals).
//
// Population layout in HBM: structure of arrays, plane (k, i) at element
// offset (k * 19 + i) * Npad, node n = x + nx (y + ny z) inside the plane, so
// consecutive work-items touch consecutive x and every load and store is
// coalesced.  Two grids (A/B ping-pong) hold the state: a step reads the
// pre-collision populations f(t) of one grid and writes f(t + 1) into the
// other (Sec. 3 of the paper describes the same one-step two-grid scheme).
#pragma once

#include "lb_device.h"

namespace lbd {

constexpr int kBlock = 256;

template <int ST>
using store_t = typename StorageTraits<ST>::store_t;
template <int ST>
using real_t = typename StorageTraits<ST>::real;

__device__ __forceinline__ void node_xyz(int n, const Geometry& g, int& x, int& y, int& z) {
  const int plane = g.nx * g.ny;
  z = n / plane;
  const int r = n - z * plane;
  y = r / g.nx;
  x = r - y * g.nx;
}

// Node indices of x + c_i for i = 0..18 with periodic wrap.
__device__ __forceinline__ void neighbours(int x, int y, int z, const Geometry& g, int (&nb)[Q]) {
  const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
  const int X[3] = {xm, x, xp};
  const int Y[3] = {ym, y, yp};
  const int Z[3] = {zm, z, zp};
#pragma unroll
  for (int i = 0; i < Q; ++i) nb[i] = X[CX[i] + 1] + g.nx * (Y[CY[i] + 1] + g.ny * Z[CZ[i] + 1]);
}

// ---------------------------------------------------------------------------
// Tile-major population layout (the fused steps where nx is a multiple of
// 64 and ny of 4): population plane ki = k Q + i of node (x, y, z) at
// element
//   z (38 nx ny) + (tile 38 + ki) 256 + (y mod 4) 64 + (x mod 64),
//   tile = (y / 4) (nx / 64) + x / 64,
// so that one 64 x 4 tile's 38 population rows of one plane are a single
// contiguous block (77,824 bytes in float64), and a workgroup marching that
// tile's column reads one stream instead of 38.  Offsets within a plane stay
// below 2^32 bytes when 38 nx ny times the element size does.
// ---------------------------------------------------------------------------
constexpr int kTileX = 64, kTileY = 4, kTileNodes = kTileX * kTileY;

__device__ __forceinline__ long long tile_major_index(int ki, int x, int y, int z, const Geometry& g) {
  const long long tile = (long long)(y >> 2) * (g.nx >> 6) + (x >> 6);
  return (long long)z * (2LL * Q * g.nx * g.ny) + (tile * (2 * Q) + ki) * kTileNodes + (y & 3) * kTileX + (x & 63);
}

// The 2 x 19 populations of node n, from the structure of arrays or (TILED)
// the tile-major layout.
template <int ST, bool TILED = false>
__device__ __forceinline__ void load_node(const store_t<ST>* __restrict__ f, long long n, const Geometry& g,
                                          const StepCoeffs& c, real_t<ST> (&out)[2][Q]) {
  if constexpr (TILED) {
    int x, y, z;
    node_xyz((int)n, g, x, y, z);
    const long long t = tile_major_index(0, x, y, z, g);
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int i = 0; i < Q; ++i) out[k][i] = decode<ST>(f[t + (long long)(k * Q + i) * kTileNodes], c.shift[k][i]);
  } else {
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int i = 0; i < Q; ++i) out[k][i] = decode<ST>(f[(long long)(k * Q + i) * g.Npad + n], c.shift[k][i]);
  }
}

// ---------------------------------------------------------------------------
// Pass 1: pseudopotential psi_k of every node (0 at solid nodes).
// psi is [2][N] in the arithmetic type.
// ---------------------------------------------------------------------------
// TILED: f in the tile-major layout (psi stays indexed by node).
template <int ST, bool SOLID, bool TILED = false>
__global__ void __launch_bounds__(kBlock) k_psi(const store_t<ST>* __restrict__ f, real_t<ST>* __restrict__ psi,
                                                const uint8_t* __restrict__ mask, Geometry g, StepCoeffs c) {
  using real = real_t<ST>;
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= g.N) return;
  real p[2] = {real(0), real(0)};
  if (!(SOLID && mask[n])) {
    real v[2][Q];
    load_node<ST, TILED>(f, n, g, c, v);
#pragma unroll
    for (int k = 0; k < 2; ++k) p[k] = pseudopotential(density<real>(v[k]), coef_ref<real>(c));
  }
  psi[n] = p[0];
  psi[(long long)g.N + n] = p[1];
}

// ---------------------------------------------------------------------------
// Pass 2: collide every fluid node and push f*_i(x) to x + c_i of the other
// grid; where x + c_i is solid the population bounces back into (x, opp(i)).
// ---------------------------------------------------------------------------
template <int ST, bool SOLID>
__global__ void __launch_bounds__(kBlock) k_collide_push(const store_t<ST>* __restrict__ fin,
                                                         store_t<ST>* __restrict__ fout,
                                                         const real_t<ST>* __restrict__ psi,
                                                         const uint8_t* __restrict__ mask, Geometry g,
                                                         StepCoeffs c) {
  using real = real_t<ST>;
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= g.N) return;
  if (SOLID && mask[n]) return;
  int x, y, z;
  node_xyz(n, g, x, y, z);
  int nb[Q];
  neighbours(x, y, z, g, nb);

  real f[2][Q];
  load_node<ST>(fin, n, g, c, f);
  real pnb[2][Q];
  pnb[0][0] = pnb[1][0] = real(0);
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    pnb[0][i] = psi[nb[i]];
    pnb[1][i] = psi[(long long)g.N + nb[i]];
  }
  const real here[2] = {psi[n], psi[(long long)g.N + n]};
  collide_node<real>(f, pnb, here, c);

#pragma unroll
  for (int k = 0; k < 2; ++k) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      long long dst = (long long)(k * Q + i) * g.Npad + nb[i];
      if (SOLID && i != 0 && mask[nb[i]]) dst = (long long)(k * Q + OPP[i]) * g.Npad + n;
      // w_opp(i) = w_i, so the float16 offset is the same for a bounced value
      fout[dst] = encode<ST>(f[k][i], c.shift[k][i]);
    }
  }
}

// ---------------------------------------------------------------------------
// Initial state: f_i^k = f_i^eq(rho_k, u), zero at solid nodes.
// ---------------------------------------------------------------------------
template <int ST>
__global__ void __launch_bounds__(kBlock) k_init(const double* __restrict__ ra, const double* __restrict__ rb,
                                                 const double* __restrict__ u, const uint8_t* __restrict__ mask,
                                                 store_t<ST>* __restrict__ f, Geometry g, StepCoeffs c) {
  using real = real_t<ST>;
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= g.N) return;
  const bool solid = mask != nullptr && mask[n];
  real ux = real(0), uy = real(0), uz = real(0);
  if (u != nullptr) {
    ux = static_cast<real>(u[n]);
    uy = static_cast<real>(u[(long long)g.N + n]);
    uz = static_cast<real>(u[2LL * g.N + n]);
  }
  const real vv = (ux * ux + uy * uy) + uz * uz;
  const real t15 = real(1.5) * vv;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const real rho = static_cast<real>(k == 0 ? ra[n] : rb[n]);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const real cu = cdot<real>(i, ux, uy, uz);
      real feq = (weight<real>(i) * rho) * (((real(1) + real(3) * cu) + real(4.5) * cu * cu) - t15);
      if (solid) feq = real(0);
      store_t<ST> s = encode<ST>(feq, c.shift[k][i]);
      if (solid) s = store_t<ST>(0);
      f[(long long)(k * Q + i) * g.Npad + n] = s;
    }
  }
}

// Reject non-finite or negative densities and non-finite velocities.
__global__ void __launch_bounds__(kBlock) k_validate_fields(const double* __restrict__ ra,
                                                            const double* __restrict__ rb,
                                                            const double* __restrict__ u, int N, int* flag,
                                                            int need_total) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= N) return;
  bool bad = !(ra[n] >= 0.0 && ra[n] <= 1.0e300) || !(rb[n] >= 0.0 && rb[n] <= 1.0e300);
  if (need_total) bad = bad || !(ra[n] + rb[n] > 0.0);  // the phase field needs rho_A + rho_B > 0
  if (u != nullptr) {
    for (int a = 0; a < 3; ++a) {
      const double v = u[(long long)a * N + n];
      bad = bad || !(v == v) || v > 1.0e300 || v < -1.0e300;
    }
  }
  if (bad) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// Export / import of one population plane (k, i) as float64 [N].
// ---------------------------------------------------------------------------
// Solid nodes export 0 whatever their stored bits (a float16 offset would
// otherwise decode a stored 0 as w_i rho0).
// One population plane as float64 (zero at solid nodes), from the structure
// of arrays or (TILED) the tile-major layout.
template <int ST, bool TILED = false>
__global__ void __launch_bounds__(kBlock) k_decode_plane(const store_t<ST>* __restrict__ f, double* __restrict__ out,
                                                         const uint8_t* __restrict__ mask, int plane, Geometry g,
                                                         StepCoeffs c) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= g.N) return;
  const int k = plane / Q, i = plane % Q;
  long long at = (long long)plane * g.Npad + n;
  if constexpr (TILED) {
    int x, y, z;
    node_xyz(n, g, x, y, z);
    at = tile_major_index(plane, x, y, z, g);
  }
  double v = static_cast<double>(decode<ST>(f[at], c.shift[k][i]));
  if (mask != nullptr && mask[n]) v = 0.0;
  out[n] = v;
}

template <int ST>
__global__ void __launch_bounds__(kBlock) k_encode_plane(const double* __restrict__ in, store_t<ST>* __restrict__ f,
                                                         const uint8_t* __restrict__ mask, int plane, Geometry g,
                                                         StepCoeffs c) {
  using real = real_t<ST>;
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= g.N) return;
  const int k = plane / Q, i = plane % Q;
  store_t<ST> s = encode<ST>(static_cast<real>(in[n]), c.shift[k][i]);
  if (mask != nullptr && mask[n]) s = store_t<ST>(0);
  f[(long long)plane * g.Npad + n] = s;
}

// Non-finite check of imported populations.
__global__ void __launch_bounds__(kBlock) k_check_finite(const double* __restrict__ in, int N, int* flag) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= N) return;
  const double v = in[n];
  if (!(v == v) || v > 1.0e300 || v < -1.0e300) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// Moments: rho_A, rho_B and u = (m_A + m_B + (F_A + F_B) / 2) / (rho_A + rho_B).
// Needs psi of the same state (k_psi).  Outputs are float64; any may be null.
// ---------------------------------------------------------------------------
template <int ST, bool SOLID, bool TILED = false>
__global__ void __launch_bounds__(kBlock) k_moments(const store_t<ST>* __restrict__ f, const real_t<ST>* __restrict__ psi,
                                                    const uint8_t* __restrict__ mask, double* __restrict__ ra,
                                                    double* __restrict__ rb, double* __restrict__ u, Geometry g,
                                                    StepCoeffs c) {
  using real = real_t<ST>;
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= g.N) return;
  if (SOLID && mask[n]) {
    if (ra) ra[n] = 0.0;
    if (rb) rb[n] = 0.0;
    if (u) {
      u[n] = 0.0;
      u[(long long)g.N + n] = 0.0;
      u[2LL * g.N + n] = 0.0;
    }
    return;
  }
  int x, y, z;
  node_xyz(n, g, x, y, z);
  int nb[Q];
  neighbours(x, y, z, g, nb);
  real fv[2][Q];
  load_node<ST, TILED>(f, n, g, c, fv);
  real rho[2], m[2][3];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    rho[k] = density<real>(fv[k]);
    m[k][0] = lattice_sum<0, 0, real>(fv[k]);
    m[k][1] = lattice_sum<1, 0, real>(fv[k]);
    m[k][2] = lattice_sum<2, 0, real>(fv[k]);
  }
  if (ra) ra[n] = static_cast<double>(rho[0]);
  if (rb) rb[n] = static_cast<double>(rho[1]);
  if (!u) return;
  real S[2][3];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    real t[Q];
    t[0] = real(0);
#pragma unroll
    for (int i = 1; i < Q; ++i) t[i] = weight<real>(i) * psi[(long long)(1 - k) * g.N + nb[i]];
    S[k][0] = lattice_sum<0, 1, real>(t);
    S[k][1] = lattice_sum<1, 1, real>(t);
    S[k][2] = lattice_sum<2, 1, real>(t);
  }
  const real G = coef_G<real>(c);
  const real pA = psi[n], pB = psi[(long long)g.N + n];
  const real tot = rho[0] + rho[1];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const real FA = (-G * pA) * S[0][a];
    const real FB = (-G * pB) * S[1][a];
    u[(long long)a * g.N + n] = static_cast<double>(((m[0][a] + m[1][a]) + real(0.5) * (FA + FB)) / tot);
  }
}

// ---------------------------------------------------------------------------
// Conserved totals in float64: per-block partials, then one block folds them.
// Both stages use a fixed order, so results are bitwise repeatable.
// partial layout: [block][8] = rho_A, rho_B, P_x, P_y, P_z, nonfinite count, -, -
// ---------------------------------------------------------------------------
constexpr int kTotals = 6;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// NK: number of population sets (components).  TILED: f in the tile-major
// layout (two components); nodes are visited in the same order either way,
// so the totals are the same bits.
template <int ST, int NK = 2, bool TILED = false>
__global__ void __launch_bounds__(kBlock) k_totals_partial(const store_t<ST>* __restrict__ f,
                                                           const uint8_t* __restrict__ mask, Geometry g, StepCoeffs c,
                                                           double* __restrict__ partial) {
  static_assert(!TILED || NK == 2, "the tile-major layout holds both components");
  double acc[kTotals] = {0, 0, 0, 0, 0, 0};
  for (long long n = (long long)blockIdx.x * kBlock + threadIdx.x; n < g.N; n += (long long)gridDim.x * kBlock) {
    if (mask != nullptr && mask[n]) continue;
    long long t = 0;
    if constexpr (TILED) {
      int x, y, z;
      node_xyz((int)n, g, x, y, z);
      t = tile_major_index(0, x, y, z, g);
    }
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      double v[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const long long at = TILED ? t + (long long)(k * Q + i) * kTileNodes : (long long)(k * Q + i) * g.Npad + n;
        v[i] = static_cast<double>(decode<ST>(f[at], c.shift[k][i]));
        if (!(v[i] - v[i] == 0.0)) acc[5] += 1.0;
      }
      acc[k] += density<double>(v);
      acc[2] += lattice_sum<0, 0, double>(v);
      acc[3] += lattice_sum<1, 0, double>(v);
      acc[4] += lattice_sum<2, 0, double>(v);
    }
  }
  __shared__ double red[kBlock / 64][kTotals];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kTotals; ++j) {
    const double s = wave_sum(acc[j]);
    if (lane == 0) red[wave][j] = s;
  }
  __syncthreads();
  if (threadIdx.x < kTotals) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += red[w][threadIdx.x];
    partial[(long long)blockIdx.x * 8 + threadIdx.x] = s;
  }
}

__global__ void __launch_bounds__(kBlock) k_totals_final(const double* __restrict__ partial, int blocks,
                                                         double* __restrict__ out) {
  double acc[kTotals] = {0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < blocks; b += kBlock)
#pragma unroll
    for (int j = 0; j < kTotals; ++j) acc[j] += partial[(long long)b * 8 + j];
  __shared__ double red[kBlock / 64][kTotals];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kTotals; ++j) {
    const double s = wave_sum(acc[j]);
    if (lane == 0) red[wave][j] = s;
  }
  __syncthreads();
  if (threadIdx.x < kTotals) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += red[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

}  // namespace lbd
