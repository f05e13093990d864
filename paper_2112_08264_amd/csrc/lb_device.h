// Device-side building blocks of the two-component D3Q19 steps (Shan-Chen,
// and the colour-gradient constants): lattice constants, the
// pseudopotential's exp, population storage codecs and the per-node
// Shan-Chen collision shared by its step kernels.
//
// Floating-point order.  The float64 path performs the same IEEE operations
// in the same order as the published definition below, with no fused
// multiply-add (the library is built with -ffp-contract=off), so its results
// are reproducible bit for bit by any implementation that follows the same
// order:
//   rho   = ((f_0 + f_1) + f_2) + ... + f_18
//   m_a   = sum_{i=0..18} c_ia f_i accumulated from 0 in index order
//   S_a   = sum_{i=1..18} c_ia (w_i psi(x + c_i)) accumulated from 0 in index order
//   den   = omega_A rho_A + omega_B rho_B;  u'_a = (omega_A m_Aa + omega_B m_Ba) / den
//   a_k   = (tau_k G) (psi_k / rho_k), psi_k / rho_k := 1 at rho_k = 0;  v_ka = u'_a - a_k S_ka
//   vv    = (v_x v_x + v_y v_y) + v_z v_z;  cu = (c_x v_x + c_y v_y) + c_z v_z
//   feq_i = (w_i rho) (((1 + 3 cu) + (4.5 cu) cu) - 1.5 vv)
//   f*_i  = (1 - omega) f_i + omega feq_i
// Terms whose lattice coefficient is zero are left out of the sums; adding
// a signed zero would change nothing but the sign of an exactly zero result.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace lbd {

constexpr int Q = 19;

// D3Q19 (Sec. 2): rest, the six axis neighbours, the twelve face diagonals
// in opposite pairs.  Weights by |c|^2 class from the Appendix table.
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

template <typename T>
__host__ __device__ constexpr T weight(int i) {
  return i == 0 ? T(1) / T(3) : (i <= 6 ? T(1) / T(18) : T(1) / T(36));
}

// ---------------------------------------------------------------------------
// Storage formats
// ---------------------------------------------------------------------------
enum Storage : int { ST_F64 = 0, ST_F32 = 1, ST_F16S = 2 };

template <int ST> struct StorageTraits;
template <> struct StorageTraits<ST_F64> { using store_t = double; using real = double; };
template <> struct StorageTraits<ST_F32> { using store_t = float; using real = float; };
template <> struct StorageTraits<ST_F16S> { using store_t = __half; using real = float; };

// Per-step constants, formed once on the host in float64 (and rounded to
// float32 for the float32 paths).
struct StepCoeffs {
  double om[2];    // omega_k = 1 / tau_k
  double omc[2];   // 1 - omega_k
  double tg[2];    // tau_k * G
  double tau[2];   // tau_k
  double G;
  double psi_ref;
  float omf[2], omcf[2], tgf[2], tauf[2], Gf, psi_reff;
  float shift[2][Q];  // w_i * rho0_k, the float16 storage offset
  // colour-gradient model: 1/nu_k = 1 / ((tau_k - 1/2) / 3), 2.25 sigma (so
  // that A = (2.25 sigma) omega), beta
  double cg_inv_nu[2], cg_s225, cg_beta;
  float cg_inv_nuf[2], cg_s225f, cg_betaf;
};

struct Geometry {
  int nx, ny, nz;
  int N;            // nx * ny * nz
  long long Npad;   // element stride between population planes
};

template <int ST>
__device__ __forceinline__ typename StorageTraits<ST>::real decode(typename StorageTraits<ST>::store_t v, float shift) {
  if constexpr (ST == ST_F16S) {
    return __half2float(v) + shift;
  } else {
    (void)shift;
    return v;
  }
}

template <int ST>
__device__ __forceinline__ typename StorageTraits<ST>::store_t encode(typename StorageTraits<ST>::real v, float shift) {
  if constexpr (ST == ST_F16S) {
    return __float2half_rn(v - shift);
  } else {
    (void)shift;
    return v;
  }
}

// 1.0f in a register whose value the compiler does not know.  With it,
// fma(float(h), one, shift) is selected as one v_fma_mix_f32 (the float16
// operand converted inside the FMA, one rounding of h + shift: the same bits
// as the conversion followed by the float32 addition of `decode`), where
// the visible 1.0 would be folded into a plain addition.
__device__ __forceinline__ float opaque_one() {
  float one;
  asm volatile("v_mov_b32 %0, 1.0" : "=v"(one));
  return one;
}

// The value held by lane l ^ 32, the same node's other component in the
// component-pair kernels: one v_permlane32_swap per 32-bit word (lanes 32-63
// of the first operand trade places with lanes 0-31 of the second), in
// place of an LDS permute.
__device__ __forceinline__ uint32_t other_half_u32(uint32_t x) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
  return (__lane_id() & 32) ? r[0] : r[1];
}
__device__ __forceinline__ float other_half(float v) { return __uint_as_float(other_half_u32(__float_as_uint(v))); }
__device__ __forceinline__ double other_half(double v) {
  const unsigned long long b = __double_as_longlong(v);
  const uint32_t lo = other_half_u32((uint32_t)b), hi = other_half_u32((uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// `decode` for a uniform shift, with `one` from opaque_one().
template <int ST>
__device__ __forceinline__ typename StorageTraits<ST>::real decode_mix(typename StorageTraits<ST>::store_t v,
                                                                      float shift, float one) {
  if constexpr (ST == ST_F16S) {
    return __builtin_fmaf(__half2float(v), one, shift);
  } else {
    (void)shift;
    (void)one;
    return v;
  }
}

// Raw buffer access (gfx9 resource descriptor, stride 0): the wave-uniform
// base goes into the descriptor and the soffset register, the per-lane
// part into a 32-bit voffset, so no 64-bit address is formed per lane.
// Accesses at or beyond `bytes` from the base read 0 and write nothing.
constexpr int kBufferWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufferWord3);
}

template <int ST>
__device__ __forceinline__ typename StorageTraits<ST>::store_t buffer_load(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                                          uint32_t soff) {
  if constexpr (ST == ST_F16S) {
    return __ushort_as_half(__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
  } else if constexpr (ST == ST_F32) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  } else {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  }
}

template <int ST>
__device__ __forceinline__ void buffer_store(typename StorageTraits<ST>::store_t v, __amdgpu_buffer_rsrc_t r,
                                             uint32_t voff, uint32_t soff) {
  if constexpr (ST == ST_F16S) {
    __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(v), r, voff, soff, 0);
  } else if constexpr (ST == ST_F32) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
  } else {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
  }
}

// ---------------------------------------------------------------------------
// e^x (float64): Cody & Waite range reduction, n = rint(x / ln 2),
// r = (x - n ln2_hi) - n ln2_lo, then the degree-13 Taylor polynomial of e^r
// by Horner's rule and e^x = 2^n e^r.  A fixed sequence of IEEE operations,
// so any implementation of the same recipe returns the same bits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double exp_cw(double x) {
  constexpr double INV_LN2 = 0x1.71547652b82fep+0;
  constexpr double LN2_HI = 0x1.62e42fee00000p-1;
  constexpr double LN2_LO = 0x1.a39ef35793c76p-33;
  const double n = rint(x * INV_LN2);
  const double r = (x - n * LN2_HI) - n * LN2_LO;
  double p = 1.0 / 6227020800.0;   // 1/13!
  p = p * r + 1.0 / 479001600.0;   // 1/12!
  p = p * r + 1.0 / 39916800.0;    // 1/11!
  p = p * r + 1.0 / 3628800.0;     // 1/10!
  p = p * r + 1.0 / 362880.0;      // 1/9!
  p = p * r + 1.0 / 40320.0;       // 1/8!
  p = p * r + 1.0 / 5040.0;        // 1/7!
  p = p * r + 1.0 / 720.0;         // 1/6!
  p = p * r + 1.0 / 120.0;         // 1/5!
  p = p * r + 1.0 / 24.0;          // 1/4!
  p = p * r + 1.0 / 6.0;           // 1/3!
  p = p * r + 1.0 / 2.0;           // 1/2!
  p = p * r + 1.0;                 // 1/1!
  p = p * r + 1.0;                 // 1/0!
  return ldexp(p, static_cast<int>(n));
}

// Shan-Chen pseudopotential psi = rho_ref (1 - exp(-rho / rho_ref)).
__device__ __forceinline__ double pseudopotential(double rho, double ref) {
  return ref * (1.0 - exp_cw(-(rho / ref)));
}
__device__ __forceinline__ float pseudopotential(float rho, float ref) {
  return ref * (1.0f - __expf(-(rho / ref)));
}

template <typename real> __device__ __forceinline__ real coef_om(const StepCoeffs& c, int k);
template <> __device__ __forceinline__ double coef_om<double>(const StepCoeffs& c, int k) { return c.om[k]; }
template <> __device__ __forceinline__ float coef_om<float>(const StepCoeffs& c, int k) { return c.omf[k]; }
template <typename real> __device__ __forceinline__ real coef_omc(const StepCoeffs& c, int k);
template <> __device__ __forceinline__ double coef_omc<double>(const StepCoeffs& c, int k) { return c.omc[k]; }
template <> __device__ __forceinline__ float coef_omc<float>(const StepCoeffs& c, int k) { return c.omcf[k]; }
template <typename real> __device__ __forceinline__ real coef_tg(const StepCoeffs& c, int k);
template <> __device__ __forceinline__ double coef_tg<double>(const StepCoeffs& c, int k) { return c.tg[k]; }
template <> __device__ __forceinline__ float coef_tg<float>(const StepCoeffs& c, int k) { return c.tgf[k]; }
template <typename real> __device__ __forceinline__ real coef_tau(const StepCoeffs& c, int k);
template <> __device__ __forceinline__ double coef_tau<double>(const StepCoeffs& c, int k) { return c.tau[k]; }
template <> __device__ __forceinline__ float coef_tau<float>(const StepCoeffs& c, int k) { return c.tauf[k]; }
template <typename real> __device__ __forceinline__ real coef_G(const StepCoeffs& c);
template <> __device__ __forceinline__ double coef_G<double>(const StepCoeffs& c) { return c.G; }
template <> __device__ __forceinline__ float coef_G<float>(const StepCoeffs& c) { return c.Gf; }
template <typename real> __device__ __forceinline__ real coef_ref(const StepCoeffs& c);
template <> __device__ __forceinline__ double coef_ref<double>(const StepCoeffs& c) { return c.psi_ref; }
template <> __device__ __forceinline__ float coef_ref<float>(const StepCoeffs& c) { return c.psi_reff; }

template <typename real> __device__ __forceinline__ real coef_cg_inv_nu(const StepCoeffs& c, int k);
template <> __device__ __forceinline__ double coef_cg_inv_nu<double>(const StepCoeffs& c, int k) { return c.cg_inv_nu[k]; }
template <> __device__ __forceinline__ float coef_cg_inv_nu<float>(const StepCoeffs& c, int k) { return c.cg_inv_nuf[k]; }
template <typename real> __device__ __forceinline__ real coef_cg_s225(const StepCoeffs& c);
template <> __device__ __forceinline__ double coef_cg_s225<double>(const StepCoeffs& c) { return c.cg_s225; }
template <> __device__ __forceinline__ float coef_cg_s225<float>(const StepCoeffs& c) { return c.cg_s225f; }
template <typename real> __device__ __forceinline__ real coef_cg_beta(const StepCoeffs& c);
template <> __device__ __forceinline__ double coef_cg_beta<double>(const StepCoeffs& c) { return c.cg_beta; }
template <> __device__ __forceinline__ float coef_cg_beta<float>(const StepCoeffs& c) { return c.cg_betaf; }

// ---------------------------------------------------------------------------
// Colour-gradient constants (Appendix): the perturbation coefficients B_i by
// |c|^2 class from the Appendix table, |c_i| (1 at rest, where c_i . n = 0),
// and the squared phase-field gradient above which a node counts as
// interface: the perturbation and the recolouring act there only.  float64
// cuts at |grad Theta| = 1e-8, well above its rounding noise in a uniform
// mixture (~1e-16); float arithmetic at 1e-5, above its own (~1e-7).
// ---------------------------------------------------------------------------
template <typename T>
__host__ __device__ constexpr T cg_b(int i) {
  return i == 0 ? T(-2) / T(9) : (i <= 6 ? T(1) / T(54) : T(1) / T(27));
}
template <typename T>
__host__ __device__ constexpr T cg_clen(int i) {
  return i <= 6 ? T(1) : T(1.4142135623730951);
}
template <typename T> __host__ __device__ constexpr T cg_interface_g2();
template <> __host__ __device__ constexpr double cg_interface_g2<double>() { return 1e-16; }
template <> __host__ __device__ constexpr float cg_interface_g2<float>() { return 1e-10f; }

// ---------------------------------------------------------------------------
// Local moments of one component's 19 populations.
// ---------------------------------------------------------------------------
template <typename real>
__device__ __forceinline__ real density(const real (&f)[Q]) {
  real r = f[0];
#pragma unroll
  for (int i = 1; i < Q; ++i) r = r + f[i];
  return r;
}

// sum_i c_i^(axis) g_i accumulated from zero in index order, zero terms left out.
template <int AXIS, int FIRST, typename real>
__device__ __forceinline__ real lattice_sum(const real (&g)[Q]) {
  real s = real(0);
#pragma unroll
  for (int i = FIRST; i < Q; ++i) {
    const int c = AXIS == 0 ? CX[i] : (AXIS == 1 ? CY[i] : CZ[i]);
    if (c == 1) s = s + g[i];
    if (c == -1) s = s - g[i];
  }
  return s;
}

// (c_x v_x + c_y v_y) + c_z v_z for direction i, zero terms left out.
template <typename real>
__device__ __forceinline__ real cdot(int i, real vx, real vy, real vz) {
  real s = real(0);
  if (CX[i] == 1) s = s + vx;
  if (CX[i] == -1) s = s - vx;
  if (CY[i] == 1) s = s + vy;
  if (CY[i] == -1) s = s - vy;
  if (CZ[i] == 1) s = s + vz;
  if (CZ[i] == -1) s = s - vz;
  return s;
}

// ---------------------------------------------------------------------------
// float arithmetic only (float32 and float16-shifted storage, which are not
// bound to the float64 operation order): BGK relaxation of one component's
// 19 populations towards f^eq(rho, v).  Opposite directions i, i + 1 share
// the even part of f^eq, w rho (1 - 1.5 v.v + 4.5 (c.v)^2), and differ in
// the sign of its odd part, 3 w rho c.v; products are fused.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void relax_f32(const float (&f)[Q], float (&fs)[Q], float rho, float vx, float vy,
                                          float vz, float om, float omc) {
  const float vv = fmaf(vz, vz, fmaf(vy, vy, vx * vx));
  const float a0 = fmaf(-1.5f, vv, 1.0f);
  const float orho = om * rho;
  fs[0] = fmaf(omc, f[0], (orho * weight<float>(0)) * a0);
#pragma unroll
  for (int i = 1; i < Q; i += 2) {  // OPP[i] == i + 1
    const float cu = cdot<float>(i, vx, vy, vz);
    const float e = orho * weight<float>(i);
    const float even = e * fmaf(4.5f * cu, cu, a0);
    const float odd = (3.0f * e) * cu;
    fs[i] = fmaf(omc, f[i], even) + odd;
    fs[i + 1] = fmaf(omc, f[i + 1], even) - odd;
  }
}

// ---------------------------------------------------------------------------
// Velocity-shifted BGK collision of both components at one node, in place.
//   f        : the 2 x 19 pre-collision populations (overwritten by f*)
//   psi_nb   : psi_A and psi_B at x + c_i, i = 1..18 (index 0 unused)
//   psi_here : psi_A, psi_B at x
// ---------------------------------------------------------------------------
template <typename real>
__device__ __forceinline__ void collide_node(real (&f)[2][Q], const real (&psi_nb)[2][Q],
                                             const real (&psi_here)[2], const StepCoeffs& c) {
  real rho[2], m[2][3];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    rho[k] = density<real>(f[k]);
    m[k][0] = lattice_sum<0, 0, real>(f[k]);
    m[k][1] = lattice_sum<1, 0, real>(f[k]);
    m[k][2] = lattice_sum<2, 0, real>(f[k]);
  }
  // S_k = sum_i w_i psi_kbar(x + c_i) c_i
  real S[2][3];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    real t[Q];
    t[0] = real(0);
#pragma unroll
    for (int i = 1; i < Q; ++i) t[i] = weight<real>(i) * psi_nb[1 - k][i];
    S[k][0] = lattice_sum<0, 1, real>(t);
    S[k][1] = lattice_sum<1, 1, real>(t);
    S[k][2] = lattice_sum<2, 1, real>(t);
  }
  const real omA = coef_om<real>(c, 0), omB = coef_om<real>(c, 1);
  const real den = omA * rho[0] + omB * rho[1];
  real up[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) up[a] = (omA * m[0][a] + omB * m[1][a]) / den;

#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const real ratio = rho[k] == real(0) ? real(1) : psi_here[k] / rho[k];
    const real ak = coef_tg<real>(c, k) * ratio;
    const real vx = up[0] - ak * S[k][0];
    const real vy = up[1] - ak * S[k][1];
    const real vz = up[2] - ak * S[k][2];
    const real vv = (vx * vx + vy * vy) + vz * vz;
    const real t15 = real(1.5) * vv;
    const real om = coef_om<real>(c, k), omc = coef_omc<real>(c, k);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const real cu = cdot<real>(i, vx, vy, vz);
      const real feq = (weight<real>(i) * rho[k]) * (((real(1) + real(3) * cu) + real(4.5) * cu * cu) - t15);
      f[k][i] = omc * f[k][i] + om * feq;
    }
  }
}

}  // namespace lbd
