// Runtime-order evaluation helpers for the batched consumer (one order per
// tile, not a compile-time constant), built on the FP64 method of
// boys_device_f64.hpp.
#pragma once

#include "boys_device_f64.hpp"

namespace boys {

// ---------------------------------------------------------------------------
// Runtime-order variants for kernels whose order k is uniform per tile but
// not a compile-time constant (the batched consumer).  The arithmetic is the
// same as boys_f64<K>, step for step.

// r_{A,k}(x) for a wave-uniform k in [0, 32] (a jump on a scalar register).
__device__ __forceinline__ double rational_a_rt(double x, int k) {
  switch (k) {
#define BOYS_RA_CASE(K) \
  case K:               \
    return rational_a<K>(x);
    BOYS_RA_CASE(0) BOYS_RA_CASE(1) BOYS_RA_CASE(2) BOYS_RA_CASE(3) BOYS_RA_CASE(4)
    BOYS_RA_CASE(5) BOYS_RA_CASE(6) BOYS_RA_CASE(7) BOYS_RA_CASE(8) BOYS_RA_CASE(9)
    BOYS_RA_CASE(10) BOYS_RA_CASE(11) BOYS_RA_CASE(12) BOYS_RA_CASE(13) BOYS_RA_CASE(14)
    BOYS_RA_CASE(15) BOYS_RA_CASE(16) BOYS_RA_CASE(17) BOYS_RA_CASE(18) BOYS_RA_CASE(19)
    BOYS_RA_CASE(20) BOYS_RA_CASE(21) BOYS_RA_CASE(22) BOYS_RA_CASE(23) BOYS_RA_CASE(24)
    BOYS_RA_CASE(25) BOYS_RA_CASE(26) BOYS_RA_CASE(27) BOYS_RA_CASE(28) BOYS_RA_CASE(29)
    BOYS_RA_CASE(30) BOYS_RA_CASE(31) BOYS_RA_CASE(32)
#undef BOYS_RA_CASE
    default:
      return __builtin_nan("");
  }
}

// Weighted sums for the batched consumer, with the sum accumulated inside the
// recurrence as in the paper's benchmark consumer (Sec. III, Algorithm 2).
//
// The recurrences run in chunks of kChunk steps whose LDS reads (weights,
// reciprocals) are issued together, so a chunk waits for LDS once rather
// than once per step.  The tables are padded so that chunks may overrun the
// order: w[l] = 0 for l < 0 and l > k, which makes the extra steps add
// exactly zero (their F values stay finite for finite x).  Table layout:
// w = base + kPad, valid for indices -kPad .. kF64Kmax + kPad.
constexpr int kChunk = 4;
constexpr int kPad = kChunk;
constexpr int kTableLen = kF64Kmax + 1 + 2 * kPad;

// Region A: r_{A,k}, then F_l = (2x F_{l+1} + e^-x) * inv[l] downwards;
// inv[l] = 1/(2l+1) rounded (finite for the padded l < 0 too).
__device__ __forceinline__ double wsum_region_a(double x, int k, const double *w,
                                                const double *inv) {
  const double e = ::exp(-x);
  const double two_x = x + x;
  double F = rational_a_rt(x, k);
  double acc = w[k] * F;
  for (int l0 = k - 1; l0 >= 0; l0 -= kChunk) {
    double wl[kChunk], il[kChunk];
#pragma unroll
    for (int s = 0; s < kChunk; ++s) {
      wl[s] = w[l0 - s];
      il[s] = inv[l0 - s];
    }
#pragma unroll
    for (int s = 0; s < kChunk; ++s) {
      F = __builtin_fma(two_x, F, e) * il[s];
      acc = __builtin_fma(wl[s], F, acc);
    }
  }
  return acc;
}

// Upward pass F_{l+1} = (odd[l] F_l - e) * (1/(2x)), odd[l] = 2l+1, from
// F_0 = f0; e = e^-x on region B and 0 on region C.
__device__ __forceinline__ double wsum_upward(double x, double f0, double e, int k,
                                              const double *w, const double *odd) {
  const double inv_2x = 0.5 / x;
  double F = f0;
  double acc = w[0] * F;
  for (int l0 = 0; l0 < k; l0 += kChunk) {
    double wl[kChunk], cl[kChunk];
#pragma unroll
    for (int s = 0; s < kChunk; ++s) {
      wl[s] = w[l0 + s + 1];
      cl[s] = odd[l0 + s];
    }
#pragma unroll
    for (int s = 0; s < kChunk; ++s) {
      F = __builtin_fma(cl[s], F, -e) * inv_2x;
      acc = __builtin_fma(wl[s], F, acc);
    }
  }
  return acc;
}

__device__ __forceinline__ double wsum_region_b(double x, int k, const double *w,
                                                const double *odd) {
  return wsum_upward(x, rational_b(x), ::exp(-x), k, w, odd);
}

// Region C needs 1/sqrt(x) and 1/(2x); both come from one reciprocal square
// root r (about 11 VALU instructions instead of a square root and two
// divisions, about 33): F_0 = (sqrt(pi)/2) r and 1/(2x) = r^2/2, each within
// a few ulps, which the asymptote's own 5e-14 error bound dwarfs.
__device__ __forceinline__ double wsum_region_c(double x, int k, const double *w,
                                                const double *odd) {
  const double r = ::rsqrt(x);
  const double inv_2x = 0.5 * r * r;
  double F = kHalfSqrtPi * r;
  double acc = w[0] * F;
  for (int l0 = 0; l0 < k; l0 += kChunk) {
    double wl[kChunk], cl[kChunk];
#pragma unroll
    for (int s = 0; s < kChunk; ++s) {
      wl[s] = w[l0 + s + 1];
      cl[s] = odd[l0 + s];
    }
#pragma unroll
    for (int s = 0; s < kChunk; ++s) {
      F = (cl[s] * F) * inv_2x;
      acc = __builtin_fma(wl[s], F, acc);
    }
  }
  return acc;
}

}  // namespace boys
