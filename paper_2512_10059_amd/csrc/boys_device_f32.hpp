// Device-side FP32 variant of the Boys-function method (orders 0..16) for
// gfx950, with the library's own minimax coefficients (boys_coeffs_f32.h).
//
// Regions A' = [0, x0'), B' = [x0', x1'), C' = [x1', inf) with x0' = x0(16)
// and x1' from the asymptote's error bound at F_16 (the paper's two region
// equations, Sec. II C, at kmax = 16):
//   A': F_K = r'_{A,K}(x) in FP32 (FP32 coefficients, FMA Horner, IEEE
//       division), then the FP32 downward recurrence;
//   B': F_0 = r'_B(x) in FP64, then the FP64 upward recurrence, rounded to
//       FP32 on the way out: upward recurrence subtracts nearly equal
//       numbers when l approaches x, so it keeps the wider type;
//   C': the asymptote sqrt(pi)/(2 sqrt x), F_{l+1} = (2l+1)/(2x) F_l, in FP32.
#pragma once

#include <hip/hip_runtime.h>

#include "boys_coeffs_f32.h"

namespace boys {

constexpr int kF32Kmax = BOYS_F32_KMAX;
constexpr float kX0f = BOYS_F32_X0;
constexpr float kX1f = BOYS_F32_X1;
constexpr float kHalfSqrtPiF = 0.886226925452758013649f;

constexpr int kRa32N[kF32Kmax + 1] = BOYS_F32_RA_DEG_N_INIT;
constexpr int kRa32M[kF32Kmax + 1] = BOYS_F32_RA_DEG_M_INIT;
constexpr float kRa32P[kF32Kmax + 1][BOYS_F32_RA_NMAX + 1] = BOYS_F32_RA_P_INIT;
constexpr float kRa32Q[kF32Kmax + 1][BOYS_F32_RA_MMAX + 1] = BOYS_F32_RA_Q_INIT;
constexpr double kRb32P[BOYS_F32_RB_N + 1] = BOYS_F32_RB_P_INIT;
constexpr double kRb32Q[BOYS_F32_RB_M + 1] = BOYS_F32_RB_Q_INIT;

template <int K>
__device__ __forceinline__ float rational_a32(float x) {
  constexpr int n = kRa32N[K], m = kRa32M[K];
  float p = kRa32P[K][n];
#pragma unroll
  for (int i = n - 1; i >= 0; --i) p = __builtin_fmaf(p, x, kRa32P[K][i]);
  float q = x + kRa32Q[K][m - 1];
#pragma unroll
  for (int i = m - 2; i >= 0; --i) q = __builtin_fmaf(q, x, kRa32Q[K][i]);
  return p / q;
}

__device__ __forceinline__ double rational_b32(double x) {
  double p = kRb32P[BOYS_F32_RB_N];
#pragma unroll
  for (int i = BOYS_F32_RB_N - 1; i >= 0; --i) p = __builtin_fma(p, x, kRb32P[i]);
  double q = x + kRb32Q[BOYS_F32_RB_M - 1];
#pragma unroll
  for (int i = BOYS_F32_RB_M - 2; i >= 0; --i) q = __builtin_fma(q, x, kRb32Q[i]);
  return p / q;
}

// F_0..F_K at one FP32 argument into F[0..K] (FP32 results).
template <int K>
__device__ __forceinline__ void boys_f32(float x, float (&F)[K + 1]) {
  static_assert(K <= kF32Kmax, "the FP32 tables cover orders 0..16");
  x = x >= 0.0f ? x : __builtin_nanf("");
  if (x < kX0f) {
    F[K] = rational_a32<K>(x);
    const float e = ::expf(-x);
    const float two_x = x + x;
#pragma unroll
    for (int l = K - 1; l >= 0; --l)
      F[l] = __builtin_fmaf(two_x, F[l + 1], e) * (1.0f / float(2 * l + 1));
  } else if (!(x >= kX1f)) {  // B' (and NaN, which stays NaN)
    const double xd = double(x);
    const double e = ::exp(-xd);
    const double inv_2x = 0.5 / xd;
    double f = rational_b32(xd);
    F[0] = float(f);
#pragma unroll
    for (int l = 0; l < K; ++l) {
      f = __builtin_fma(double(2 * l + 1), f, -e) * inv_2x;
      F[l + 1] = float(f);
    }
  } else {
    const float inv_2x = 0.5f / x;
    float f = kHalfSqrtPiF / ::sqrtf(x);
    F[0] = f;
#pragma unroll
    for (int l = 0; l < K; ++l) {
      f = (float(2 * l + 1) * f) * inv_2x;
      F[l + 1] = f;
    }
  }
}

}  // namespace boys
