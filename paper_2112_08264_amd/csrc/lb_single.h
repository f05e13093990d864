// Single-fluid D3Q19 BGK step (the paper's case 1, Sec. 5), HIP kernels.
//
// One population set f_i: rho = sum_i f_i, m = sum_i f_i c_i, u = m / rho,
// BGK relaxation towards f^eq(rho, u) (Sec. 2, Eq. 1; Appendix, Eq. LEQ) and
// push streaming with halfway bounce-back at solid nodes at rest (Appendix,
// Eq. LADDFLBE with the wall velocity set to zero).  Without an
// inter-component force nothing at x depends on its neighbours before the
// collision, so one work-item updates one node: 19 coalesced loads, the
// collision, 19 pushes.  The layout is the two-component one with a single
// component: plane i at element offset i * Npad.
#pragma once

#include "lb_fused.h"
#include "lb_kernels.h"

namespace lbd {

// Work-items take consecutive nodes along x (a block covers 256 of them);
// blocks are renumbered so that each XCD takes one contiguous run of them
// (see fused_work_item with one round), which keeps the partly written
// cache lines at block ends inside one XCD's L2.
template <int ST, bool SOLID>
__global__ void __launch_bounds__(kBlock) k1_step(const store_t<ST>* __restrict__ fin, store_t<ST>* __restrict__ fout,
                                                  const uint8_t* __restrict__ mask, Geometry g, StepCoeffs c) {
  using real = real_t<ST>;
  const int b = fused_work_item(blockIdx.x, gridDim.x, gridDim.x);
  const int n = b * kBlock + threadIdx.x;
  if (n >= g.N) return;
  if (SOLID && mask[n]) return;
  int x, y, z;
  node_xyz(n, g, x, y, z);
  int nb[Q];
  neighbours(x, y, z, g, nb);
  real f[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) f[i] = decode<ST>(fin[(long long)i * g.Npad + n], c.shift[0][i]);
  const real rho = density<real>(f);
  const real ux = lattice_sum<0, 0, real>(f) / rho;
  const real uy = lattice_sum<1, 0, real>(f) / rho;
  const real uz = lattice_sum<2, 0, real>(f) / rho;
  real fs[Q];
  if constexpr (sizeof(real) == 8) {
    // float64: the oracle's operation order, no fused products
    const real om = coef_om<real>(c, 0), omc = coef_omc<real>(c, 0);
    const real t15 = real(1.5) * ((ux * ux + uy * uy) + uz * uz);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const real cu = cdot<real>(i, ux, uy, uz);
      const real feq = (weight<real>(i) * rho) * (((real(1) + real(3) * cu) + real(4.5) * cu * cu) - t15);
      fs[i] = omc * f[i] + om * feq;
    }
  } else {
    relax_f32(f, fs, rho, ux, uy, uz, coef_om<real>(c, 0), coef_omc<real>(c, 0));
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    long long dst = (long long)i * g.Npad + nb[i];
    if (SOLID && i != 0 && mask[nb[i]]) dst = (long long)OPP[i] * g.Npad + n;
    fout[dst] = encode<ST>(fs[i], c.shift[0][i]);  // w_opp(i) = w_i: same float16 offset
  }
}

// Initial state f_i = f_i^eq(rho, u), zero at solid nodes.
template <int ST>
__global__ void __launch_bounds__(kBlock) k1_init(const double* __restrict__ rho_in, const double* __restrict__ u,
                                                  const uint8_t* __restrict__ mask, store_t<ST>* __restrict__ f,
                                                  Geometry g, StepCoeffs c) {
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
  const real rho = static_cast<real>(rho_in[n]);
  const real t15 = real(1.5) * ((ux * ux + uy * uy) + uz * uz);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const real cu = cdot<real>(i, ux, uy, uz);
    const real feq = (weight<real>(i) * rho) * (((real(1) + real(3) * cu) + real(4.5) * cu * cu) - t15);
    f[(long long)i * g.Npad + n] = solid ? store_t<ST>(0) : encode<ST>(feq, c.shift[0][i]);
  }
}

// rho and u = m / rho of the pre-collision state (float64 [N] and [3][N]), zero at solid nodes.
template <int ST>
__global__ void __launch_bounds__(kBlock) k1_moments(const store_t<ST>* __restrict__ f, const uint8_t* __restrict__ mask,
                                                     double* __restrict__ rho_out, double* __restrict__ u, Geometry g,
                                                     StepCoeffs c) {
  using real = real_t<ST>;
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= g.N) return;
  double r = 0.0, v[3] = {0.0, 0.0, 0.0};
  if (!(mask != nullptr && mask[n])) {
    real q[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) q[i] = decode<ST>(f[(long long)i * g.Npad + n], c.shift[0][i]);
    const real rho = density<real>(q);
    r = static_cast<double>(rho);
    v[0] = static_cast<double>(lattice_sum<0, 0, real>(q) / rho);
    v[1] = static_cast<double>(lattice_sum<1, 0, real>(q) / rho);
    v[2] = static_cast<double>(lattice_sum<2, 0, real>(q) / rho);
  }
  if (rho_out != nullptr) rho_out[n] = r;
  if (u != nullptr)
#pragma unroll
    for (int a = 0; a < 3; ++a) u[(long long)a * g.N + n] = v[a];
}

}  // namespace lbd
