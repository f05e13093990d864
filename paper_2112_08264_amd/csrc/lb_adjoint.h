// Discrete adjoint of one step (reverse-mode derivative), HIP kernels.
//
// Given lam(t+1) = dJ/df(t+1) and the pre-collision state f(t), one adjoint
// step produces lam(t) = dJ/df(t) and the step's contribution to dJ/dG.
// With a_i(x) = lam_i(x + c_i) (lam_opp(i)(x) where x + c_i is solid), and
// per node and component
//   E_i  = 1 + 3 cu + 4.5 cu^2 - 1.5 vv,  cu = c_i . v_k   (f^eq_i = w_i rho_k E_i)
//   A_k  = sum_i a_i om_k w_i E_i                        (through rho in f^eq)
//   V_k  = sum_i a_i om_k w_i rho_k (3 c_i + 9 cu c_i - 3 v_k)   (dJ/dv_k)
//   U    = V_A + V_B,  D = om_A rho_A + om_B rho_B,  a_k = tau_k G psi_k / rho_k
//   W_k  = a_k V_k                                        (= -dJ/dS_k)
// the adjoint is
//   lam_j^k(x) = (1 - om_k) a_j^k + A_k - om_k (U . u') / D
//                - (V_k . S_k) tau_k G g'(rho_k) + c_j . (om_k U / D)
//                - psi'(rho_k) sum_l w_l c_l . W_kbar(x - c_l)
//   dJ/dG     += -sum_k (V_k . S_k) tau_k g(rho_k),   g = psi / rho.
// lam is kept in two parts, lam_j^k(x) = P_j^k(x) + r_k(x): P holds the
// local terms and r_k(x) = -psi'(rho_k(x)) sum_l w_l c_l . W_kbar(x - c_l)
// the stencil term, which is the same for every direction.  One adjoint step
// is then the local kernel (reads P and r of t+1 pulled from x + c_i, writes
// P(t) and W) and a small kernel that turns W into r(t); the moments of f(t)
// come either from a record the forward step wrote or from k_adj_moments.
#pragma once

#include "lb_fused.h"

namespace lbd {

// Adjoint moment record per node: rho_A, rho_B, m_A (3), m_B (3), psi_A, psi_B.
constexpr int kAdjMom = 10;

template <typename real> __device__ __forceinline__ real exp_real(real x);
template <> __device__ __forceinline__ double exp_real<double>(double x) { return exp(x); }
template <> __device__ __forceinline__ float exp_real<float>(float x) { return __expf(x); }

// g = psi / rho and g' = (psi' rho - psi) / rho^2 (limits 1 and -1/(2 ref) at rho = 0), psi' = exp(-rho/ref)
template <typename real>
__device__ __forceinline__ void psi_derivs(real rho, real psi, real ref, real& dpsi, real& g, real& dg) {
  dpsi = exp_real<real>(-rho / ref);
  if (rho == real(0)) {
    g = real(1);
    dg = real(-0.5) / ref;
  } else {
    g = psi / rho;
    dg = (dpsi * rho - psi) / (rho * rho);
  }
}

template <int ST>
__global__ void __launch_bounds__(kBlock) k_adj_moments(const store_t<ST>* __restrict__ f, const uint8_t* __restrict__ mask,
                                                        real_t<ST>* __restrict__ mom, Geometry g, StepCoeffs c) {
  using real = real_t<ST>;
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= g.N) return;
  real out[kAdjMom];
#pragma unroll
  for (int q = 0; q < kAdjMom; ++q) out[q] = real(0);
  if (!(mask != nullptr && mask[n])) {
    real v[2][Q];
    load_node<ST>(f, n, g, c, v);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      out[k] = density<real>(v[k]);
      out[2 + 3 * k + 0] = lattice_sum<0, 0, real>(v[k]);
      out[2 + 3 * k + 1] = lattice_sum<1, 0, real>(v[k]);
      out[2 + 3 * k + 2] = lattice_sum<2, 0, real>(v[k]);
      out[8 + k] = pseudopotential(out[k], coef_ref<real>(c));
    }
  }
#pragma unroll
  for (int q = 0; q < kAdjMom; ++q) mom[(long long)q * g.N + n] = out[q];
}

// Local part.  lam_in = lam(t+1), lam_out = lam(t) without the stencil term;
// W = [6][N] (W_A then W_B); partial[block] += the block's dJ/dG sum of this
// step (float64; each block owns its slot, so the running sums of a whole
// backward pass are folded once, at the end).
// float64: capped at 256 registers for two waves per SIMD (left alone the
// compiler takes 264 and one wave; 8 spills instead: 470 -> ~410 us per
// adjoint step at 128^3).
template <int ST>
__global__ void __launch_bounds__(kBlock, ST == ST_F64 ? 2 : 1) k_adj_local(const real_t<ST>* __restrict__ lam_in, const real_t<ST>* __restrict__ r_in,
                                                      real_t<ST>* __restrict__ lam_out, const real_t<ST>* __restrict__ mom,
                                                      const uint8_t* __restrict__ mask, real_t<ST>* __restrict__ Wout,
                                                      double* __restrict__ partial, Geometry g, StepCoeffs c) {
  using real = real_t<ST>;
  const int n = blockIdx.x * kBlock + threadIdx.x;
  double dG = 0.0;
  if (n < g.N) {
    const bool solid = mask != nullptr && mask[n];
    if (solid) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int j = 0; j < Q; ++j) lam_out[(long long)(k * Q + j) * g.Npad + n] = real(0);
#pragma unroll
      for (int q = 0; q < 6; ++q) Wout[(long long)q * g.N + n] = real(0);
    } else {
      int x, y, z;
      node_xyz(n, g, x, y, z);
      int nb[Q];
      neighbours(x, y, z, g, nb);
      const real ref = coef_ref<real>(c);
      real rho[2], m[2][3], psi[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        rho[k] = mom[(long long)k * g.N + n];
#pragma unroll
        for (int a = 0; a < 3; ++a) m[k][a] = mom[(long long)(2 + 3 * k + a) * g.N + n];
        psi[k] = mom[(long long)(8 + k) * g.N + n];
      }
      // S_k from psi of the other component at the neighbours (solid nodes hold psi = 0)
      real S[2][3];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        S[k][0] = S[k][1] = S[k][2] = real(0);
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          const real t = weight<real>(i) * mom[(long long)(8 + (1 - k)) * g.N + nb[i]];
          S[k][0] += real(CX[i]) * t;
          S[k][1] += real(CY[i]) * t;
          S[k][2] += real(CZ[i]) * t;
        }
      }
      const real om[2] = {coef_om<real>(c, 0), coef_om<real>(c, 1)};
      const real D = om[0] * rho[0] + om[1] * rho[1];
      real up[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) up[a] = (om[0] * m[0][a] + om[1] * m[1][a]) / D;
      real gk[2], dgk[2], ak[2], v[2][3];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        real dpsi;
        psi_derivs<real>(rho[k], psi[k], ref, dpsi, gk[k], dgk[k]);
        ak[k] = coef_tg<real>(c, k) * gk[k];
#pragma unroll
        for (int a = 0; a < 3; ++a) v[k][a] = up[a] - ak[k] * S[k][a];
      }
      // pulled adjoint populations and A_k, V_k
      real am[2][Q];
      real A[2], V[2][3];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        A[k] = real(0);
        V[k][0] = V[k][1] = V[k][2] = real(0);
        const real vv = v[k][0] * v[k][0] + v[k][1] * v[k][1] + v[k][2] * v[k][2];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          long long src = (long long)(k * Q + i) * g.Npad + nb[i];
          long long rsrc = (long long)k * g.N + nb[i];
          if (i != 0 && mask != nullptr && mask[nb[i]]) {
            src = (long long)(k * Q + OPP[i]) * g.Npad + n;
            rsrc = (long long)k * g.N + n;
          }
          const real ai = lam_in[src] + r_in[rsrc];
          am[k][i] = ai;
          const real cu = real(CX[i]) * v[k][0] + real(CY[i]) * v[k][1] + real(CZ[i]) * v[k][2];
          const real E = real(1) + real(3) * cu + real(4.5) * cu * cu - real(1.5) * vv;
          const real aw = ai * om[k] * weight<real>(i);
          A[k] += aw * E;
          const real s = aw * rho[k];
          V[k][0] += s * (real(3) * real(CX[i]) + real(9) * cu * real(CX[i]) - real(3) * v[k][0]);
          V[k][1] += s * (real(3) * real(CY[i]) + real(9) * cu * real(CY[i]) - real(3) * v[k][1]);
          V[k][2] += s * (real(3) * real(CZ[i]) + real(9) * cu * real(CZ[i]) - real(3) * v[k][2]);
        }
      }
      real U[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) U[a] = V[0][a] + V[1][a];
      const real Uu = U[0] * up[0] + U[1] * up[1] + U[2] * up[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const real VS = V[k][0] * S[k][0] + V[k][1] * S[k][1] + V[k][2] * S[k][2];
        const real R = A[k] - om[k] * Uu / D - VS * coef_tg<real>(c, k) * dgk[k];
        real M[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) M[a] = om[k] * U[a] / D;
        const real omc = real(1) - om[k];
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          const real cm = real(CX[j]) * M[0] + real(CY[j]) * M[1] + real(CZ[j]) * M[2];
          lam_out[(long long)(k * Q + j) * g.Npad + n] = omc * am[k][j] + R + cm;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) Wout[(long long)(3 * k + a) * g.N + n] = ak[k] * V[k][a];
        dG += -static_cast<double>(VS) * static_cast<double>(coef_tau<real>(c, k) * gk[k]);
      }
    }
  }
  // deterministic block sum of dG
  __shared__ double red[kBlock / 64];
  const double s = wave_sum(dG);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += red[w];
    partial[blockIdx.x] = partial[blockIdx.x] + t;
  }
}

// Stencil term r_k(x) = -psi'(rho_k(x)) sum_l w_l c_l . W_kbar(x - c_l), zero at solid nodes.
template <int ST>
__global__ void __launch_bounds__(kBlock) k_adj_r(const real_t<ST>* __restrict__ mom, const real_t<ST>* __restrict__ Win,
                                                  const uint8_t* __restrict__ mask, real_t<ST>* __restrict__ r,
                                                  Geometry g, StepCoeffs c) {
  using real = real_t<ST>;
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= g.N) return;
  if (mask != nullptr && mask[n]) {
    r[n] = real(0);
    r[(long long)g.N + n] = real(0);
    return;
  }
  int x, y, z;
  node_xyz(n, g, x, y, z);
  int nb[Q];
  neighbours(x, y, z, g, nb);
  const real ref = coef_ref<real>(c);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int kb = 1 - k;
    real T = real(0);
#pragma unroll
    for (int l = 1; l < Q; ++l) {
      const long long src = nb[OPP[l]];  // x - c_l
      // c_l . W with the zero components left out (adding a zero product
      // changes no finite sum), which halves the gathered loads
      real cw = real(0);
      if (CX[l] != 0) cw = cw + real(CX[l]) * Win[(long long)(3 * kb + 0) * g.N + src];
      if (CY[l] != 0) cw = cw + real(CY[l]) * Win[(long long)(3 * kb + 1) * g.N + src];
      if (CZ[l] != 0) cw = cw + real(CZ[l]) * Win[(long long)(3 * kb + 2) * g.N + src];
      T += weight<real>(l) * cw;
    }
    const real rho = mom[(long long)k * g.N + n];
    r[(long long)k * g.N + n] = -exp_real<real>(-rho / ref) * T;
  }
}

// The same stencil term as k_adj_r, by a z-march over 64 x 4 tiles (nx a
// multiple of 64, ny of 4): W of the planes z - 1 .. z + 2 with a one-node
// halo sit in an LDS ring, so each W value comes from HBM about once instead
// of being gathered from the cache by up to 18 neighbours.  The loads of
// plane z + 2 are issued before plane z is computed and written to the ring
// after it, with one barrier per plane.  Every node sums the same terms in
// the same order as k_adj_r, so the two give the same bits.
template <int ST>
__global__ void __launch_bounds__(256) k_adj_r_march(const real_t<ST>* __restrict__ mom,
                                                     const real_t<ST>* __restrict__ Win,
                                                     const uint8_t* __restrict__ mask, real_t<ST>* __restrict__ r,
                                                     Geometry g, StepCoeffs c, FusedTiling t) {
  using real = real_t<ST>;
  constexpr int TX = 64, TY = 4, RX = TX + 2, RY = TY + 2, NS = 4;
  constexpr int NH = 2 * RX + 2 * TY;  // halo nodes of a plane (140 < 256 threads)
  __shared__ real ring[NS][6][RY][RX];
  const int w = fused_work_item(blockIdx.x, t.total, t.per_round);
  const int chunk = w / (t.tiles_x * t.tiles_y);
  const int tile = w - chunk * (t.tiles_x * t.tiles_y);
  const int ty0 = (tile / t.tiles_x) * TY, tx0 = (tile % t.tiles_x) * TX;
  const int z0 = chunk * t.chunk;
  const int zlen = min(t.chunk, g.nz - z0);
  const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
  const int gx = tx0 + lx, gy = ty0 + ly;  // the host checks nx % 64 == 0 and ny % 4 == 0
  const long long N = g.N;
  const uint32_t plane_n = (uint32_t)g.nx * (uint32_t)g.ny;
  const uint32_t row = (uint32_t)gx + (uint32_t)g.nx * (uint32_t)gy;
  // halo node of this thread: rows -1 and TY (with the corners), then columns -1 and TX
  const bool has_halo = threadIdx.x < NH;
  int hx = 0, hy = 0;
  if (threadIdx.x < 2 * RX) {
    hy = threadIdx.x < RX ? -1 : TY;
    hx = (threadIdx.x % RX) - 1;
  } else if (has_halo) {
    const int cn = threadIdx.x - 2 * RX;
    hx = (cn & 1) ? TX : -1;
    hy = cn >> 1;
  }
  const int hgx = ((tx0 + hx) % g.nx + g.nx) % g.nx, hgy = ((ty0 + hy) % g.ny + g.ny) % g.ny;
  const uint32_t hrow = (uint32_t)hgx + (uint32_t)g.nx * (uint32_t)hgy;
  auto wrapz = [&](int z) { return z < 0 ? z + g.nz : (z >= g.nz ? z - g.nz : z); };
  auto slot = [&](int z) { return (z - z0 + 1 + NS) % NS; };  // ring slot of plane z (z0 - 1 .. z0 + zlen)

  real iw[6], hw[6];
  auto load = [&](int z) {  // W of plane z (interior node and halo node of this thread) into registers
    const long long zo = (long long)plane_n * wrapz(z);
#pragma unroll
    for (int v = 0; v < 6; ++v) iw[v] = Win[(long long)v * N + zo + row];
    if (has_halo)
#pragma unroll
      for (int v = 0; v < 6; ++v) hw[v] = Win[(long long)v * N + zo + hrow];
  };
  auto store = [&](int z) {  // ... into the ring
    const int s = slot(z);
#pragma unroll
    for (int v = 0; v < 6; ++v) ring[s][v][ly + 1][lx + 1] = iw[v];
    if (has_halo)
#pragma unroll
      for (int v = 0; v < 6; ++v) ring[s][v][hy + 1][hx + 1] = hw[v];
  };
  load(z0 - 1);
  store(z0 - 1);
  load(z0);
  store(z0);
  load(z0 + 1);
  store(z0 + 1);
  __syncthreads();
  const real ref = coef_ref<real>(c);
  for (int j = 0; j < zlen; ++j) {
    const int z = z0 + j;
    if (j + 2 <= zlen) load(z + 2);  // plane z0 + zlen is the chunk's far neighbour
    const long long n = (long long)plane_n * z + row;
    const int sm = slot(z - 1), s0 = slot(z), sp = slot(z + 1);
    if (mask != nullptr && mask[n]) {
      r[n] = real(0);
      r[N + n] = real(0);
    } else {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int kb = 1 - k;
        real T = real(0);
#pragma unroll
        for (int l = 1; l < Q; ++l) {
          // W at x - c_l
          const int si = CZ[l] > 0 ? sm : (CZ[l] < 0 ? sp : s0);
          const int yy = ly + 1 - CY[l], xx = lx + 1 - CX[l];
          real cw = real(0);
          if (CX[l] != 0) cw = cw + real(CX[l]) * ring[si][3 * kb + 0][yy][xx];
          if (CY[l] != 0) cw = cw + real(CY[l]) * ring[si][3 * kb + 1][yy][xx];
          if (CZ[l] != 0) cw = cw + real(CZ[l]) * ring[si][3 * kb + 2][yy][xx];
          T += weight<real>(l) * cw;
        }
        const real rho = mom[(long long)k * N + n];
        r[(long long)k * N + n] = -exp_real<real>(-rho / ref) * T;
      }
    }
    if (j + 2 <= zlen) store(z + 2);
    __syncthreads();
  }
}

// dJ/dG of the adjoint steps so far: the blocks' running sums folded in a
// fixed order (single block); acc[0] is overwritten, so folding twice gives
// the same value.
__global__ void __launch_bounds__(kBlock) k_adj_fold(const double* __restrict__ partial, int blocks, double* __restrict__ acc) {
  double s = 0.0;
  for (int b = threadIdx.x; b < blocks; b += kBlock) s += partial[b];
  __shared__ double red[kBlock / 64];
  const double w = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) t += red[q];
    acc[0] = t;
  }
}

// lam(T) seed: lam_i^k(x) = dJ/drho_k(x) (0 at solid nodes).
template <typename real>
__global__ void __launch_bounds__(kBlock) k_adj_seed(const double* __restrict__ ga, const double* __restrict__ gb,
                                                     const uint8_t* __restrict__ mask, real* __restrict__ lam,
                                                     real* __restrict__ r, Geometry g) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= g.N) return;
  const bool solid = mask != nullptr && mask[n];
  r[n] = real(0);
  r[(long long)g.N + n] = real(0);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const real v = solid ? real(0) : static_cast<real>(k == 0 ? (ga ? ga[n] : 0.0) : (gb ? gb[n] : 0.0));
#pragma unroll
    for (int j = 0; j < Q; ++j) lam[(long long)(k * Q + j) * g.Npad + n] = v;
  }
}

// dJ/drho_k(x, 0) = sum_i w_i lam_i^k(x, 0)
template <typename real>
__global__ void __launch_bounds__(kBlock) k_adj_result(const real* __restrict__ lam, const real* __restrict__ r,
                                                       double* __restrict__ ga, double* __restrict__ gb, Geometry g) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= g.N) return;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    double s = 0.0;
    const double rk = static_cast<double>(r[(long long)k * g.N + n]);
#pragma unroll
    for (int i = 0; i < Q; ++i)
      s += weight<double>(i) * (static_cast<double>(lam[(long long)(k * Q + i) * g.Npad + n]) + rk);
    double* out = k == 0 ? ga : gb;
    if (out) out[n] = s;
  }
}

// lam as float64 [2][19][N] (for inspection and tests)
template <typename real>
__global__ void __launch_bounds__(kBlock) k_adj_export(const real* __restrict__ lam, const real* __restrict__ r,
                                                       double* __restrict__ out, Geometry g) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= g.N) return;
  for (int p = 0; p < 2 * Q; ++p)
    out[(long long)p * g.N + n] =
        static_cast<double>(lam[(long long)p * g.Npad + n]) + static_cast<double>(r[(long long)(p / Q) * g.N + n]);
}

}  // namespace lbd
