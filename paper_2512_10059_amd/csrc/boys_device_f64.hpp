// Device-side FP64 Boys-function evaluation (Algorithm 1, Sec. II F of
// arXiv 2512.10059) for gfx950.  Everything stays in VGPRs; the coefficient
// tables are compile-time constants, so every coefficient becomes an
// instruction literal or an SGPR pair and nothing is looked up in memory.
#pragma once

#include <hip/hip_runtime.h>

#include "boys_coeffs_f64.h"

namespace boys {

constexpr int kF64Kmax = BOYS_F64_KMAX;
constexpr double kX0 = BOYS_F64_X0;  // A = [0, x0)
constexpr double kX1 = BOYS_F64_X1;  // C = (x1, inf), see region_c()
constexpr double kHalfSqrtPi = 0.88622692545275801364908374167057259;

constexpr int kRaN[kF64Kmax + 1] = BOYS_RA_DEG_N_INIT;
constexpr int kRaM[kF64Kmax + 1] = BOYS_RA_DEG_M_INIT;
constexpr double kRaP[kF64Kmax + 1][BOYS_RA_NMAX + 1] = BOYS_RA_P_INIT;
constexpr double kRaQ[kF64Kmax + 1][BOYS_RA_MMAX + 1] = BOYS_RA_Q_INIT;
constexpr double kRbP[BOYS_RB_N + 1] = BOYS_RB_P_INIT;
constexpr double kRbQ[BOYS_RB_M + 1] = BOYS_RB_Q_INIT;

// Region C is open at x1.  The printed x1 is the double nearest the root of
// the equation that defines it (asymptote error = eps_tol for F_32) but lies
// just below the root, where the asymptote misses eps_tol by 8e-30; r_B was
// fitted on the closed interval [x0, x1], so x = x1 is evaluated in B.
__device__ __forceinline__ bool region_c(double x) { return x > kX1; }

// r_{A,K}(x): Horner on numerator and (monic) denominator, one IEEE division.
template <int K>
__device__ __forceinline__ double rational_a(double x) {
  constexpr int n = kRaN[K], m = kRaM[K];
  double p = kRaP[K][n];
#pragma unroll
  for (int i = n - 1; i >= 0; --i) p = __builtin_fma(p, x, kRaP[K][i]);
  double q = x + kRaQ[K][m - 1];
#pragma unroll
  for (int i = m - 2; i >= 0; --i) q = __builtin_fma(q, x, kRaQ[K][i]);
  return p / q;
}

// r_B(x): F_0 on [x0, x1].
__device__ __forceinline__ double rational_b(double x) {
  double p = kRbP[BOYS_RB_N];
#pragma unroll
  for (int i = BOYS_RB_N - 1; i >= 0; --i) p = __builtin_fma(p, x, kRbP[i]);
  double q = x + kRbQ[BOYS_RB_M - 1];
#pragma unroll
  for (int i = BOYS_RB_M - 2; i >= 0; --i) q = __builtin_fma(q, x, kRbQ[i]);
  return p / q;
}

// Negative arguments (outside the domain) become NaN, which then flows
// through region B's arithmetic into every output.
__device__ __forceinline__ double domain(double x) {
  return x >= 0.0 ? x : __builtin_nan("");
}

// F_0..F_K at one argument into F[0..K].
//
// Region A: F_K = r_{A,K}(x), then F_l = (2x F_{l+1} + e^-x) / (2l+1).
// Regions B and C share one upward pass F_{l+1} = ((2l+1) F_l - e) / (2x):
// on B it starts from r_B with e = e^-x, on C from sqrt(pi)/(2 sqrt x) with
// e = 0, which is the asymptotic recurrence F_{l+1} = (l+1/2)/x F_l.
// Divisions by the constants 2l+1 are multiplications by their rounded
// reciprocals and 1/(2x) is formed once; each adds at most one rounding per
// step to the error model of Appendix B.
template <int K>
__device__ __forceinline__ void boys_f64(double x, double (&F)[K + 1]) {
  x = domain(x);
  const double e = ::exp(-x);
  if (x < kX0) {
    F[K] = rational_a<K>(x);
    const double two_x = x + x;
#pragma unroll
    for (int l = K - 1; l >= 0; --l)
      F[l] = __builtin_fma(two_x, F[l + 1], e) * (1.0 / (2 * l + 1));
  } else {
    const bool c = region_c(x);
    const double f0b = rational_b(x);
    const double f0c = kHalfSqrtPi / ::sqrt(x);
    F[0] = c ? f0c : f0b;
    const double eb = c ? 0.0 : e;
    const double inv_2x = 0.5 / x;
#pragma unroll
    for (int l = 0; l < K; ++l)
      F[l + 1] = __builtin_fma(double(2 * l + 1), F[l], -eb) * inv_2x;
  }
}

}  // namespace boys
