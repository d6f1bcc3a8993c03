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

// fma(a, b, c) for a compile-time (hence wave-uniform) addend c, issued as
// VOP3 v_fma_f64 with c in an SGPR pair.  Written through the compiler's
// builtin, a Horner step with a literal addend becomes v_fmac_f64 (which
// overwrites its addend) plus two v_mov_b32 per step to materialise the
// literal in VGPRs; this form needs no VALU move.  The result is the same
// correctly rounded fused multiply-add.
__device__ __forceinline__ double fma_uniform_addend(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}

// rational_a<K> and rational_b with the Horner steps above (same arithmetic).
template <int K>
__device__ __forceinline__ double rational_a_sc(double x) {
  constexpr int n = kRaN[K], m = kRaM[K];
  double p = kRaP[K][n];
#pragma unroll
  for (int i = n - 1; i >= 0; --i) p = fma_uniform_addend(p, x, kRaP[K][i]);
  double q = x + kRaQ[K][m - 1];
#pragma unroll
  for (int i = m - 2; i >= 0; --i) q = fma_uniform_addend(q, x, kRaQ[K][i]);
  return p / q;
}

__device__ __forceinline__ double rational_b_sc(double x) {
  double p = kRbP[BOYS_RB_N];
#pragma unroll
  for (int i = BOYS_RB_N - 1; i >= 0; --i) p = fma_uniform_addend(p, x, kRbP[i]);
  double q = x + kRbQ[BOYS_RB_M - 1];
#pragma unroll
  for (int i = BOYS_RB_M - 2; i >= 0; --i) q = fma_uniform_addend(q, x, kRbQ[i]);
  return p / q;
}

// r_{A,k}(x) for a wave-uniform k in [0, 32] (a jump on a scalar register).
__device__ __forceinline__ double rational_a_rt(double x, int k) {
  switch (k) {
#define BOYS_RA_CASE(K) \
  case K:               \
    return rational_a_sc<K>(x);
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
// The recurrences run in chunks of kChunk steps whose LDS reads are issued
// together, so a chunk waits for LDS once.  Each step needs a weight and a
// step constant; the per-wave tables hold them as adjacent pairs, one
// 16-byte LDS read per step:
//   down[l] = (w_l, 1/(2l+1))        for the downward pass,
//   up[l]   = (w_{l+1}, 2l+1)        for the upward pass.
// The tables are padded so that chunks may overrun the order: the weight is
// 0 for l < 0 and l > k, which makes the extra steps add exactly zero (their
// F values stay finite for finite x).  Valid indices: -kPad .. kF64Kmax+kPad.
typedef double wpair __attribute__((ext_vector_type(2)));
constexpr int kChunk = 4;
constexpr int kPad = kChunk;
constexpr int kTableLen = kF64Kmax + 1 + 2 * kPad;

// Region A: r_{A,k}, then F_l = (2x F_{l+1} + e^-x) * (1/(2l+1)) downwards.
__device__ __forceinline__ double wsum_region_a(double x, int k, double wk, const wpair *down) {
  const double e = ::exp(-x);
  const double two_x = x + x;
  double F = rational_a_rt(x, k);
  double acc = wk * F;
  for (int l0 = k - 1; l0 >= 0; l0 -= kChunk) {
    wpair t[kChunk];
#pragma unroll
    for (int s = 0; s < kChunk; ++s) t[s] = down[l0 - s];
#pragma unroll
    for (int s = 0; s < kChunk; ++s) {
      F = __builtin_fma(two_x, F, e) * t[s].y;
      acc = __builtin_fma(t[s].x, F, acc);
    }
  }
  return acc;
}

// Region B: r_B, then F_{l+1} = ((2l+1) F_l - e^-x) / (2x) upwards.
__device__ __forceinline__ double wsum_region_b(double x, int k, double w0, const wpair *up) {
  const double e = ::exp(-x);
  const double inv_2x = 0.5 / x;
  double F = rational_b_sc(x);
  double acc = w0 * F;
  for (int l0 = 0; l0 < k; l0 += kChunk) {
    wpair t[kChunk];
#pragma unroll
    for (int s = 0; s < kChunk; ++s) t[s] = up[l0 + s];
#pragma unroll
    for (int s = 0; s < kChunk; ++s) {
      F = __builtin_fma(t[s].y, F, -e) * inv_2x;
      acc = __builtin_fma(t[s].x, F, acc);
    }
  }
  return acc;
}

// Region C needs 1/sqrt(x) and 1/(2x); both come from one reciprocal square
// root r (about 11 VALU instructions instead of a square root and two
// divisions, about 33): F_0 = (sqrt(pi)/2) r and 1/(2x) = r^2/2, each within
// a few ulps, which the asymptote's own 5e-14 error bound dwarfs.
__device__ __forceinline__ double wsum_region_c(double x, int k, double w0, const wpair *up) {
  const double r = ::rsqrt(x);
  const double inv_2x = 0.5 * r * r;
  double F = kHalfSqrtPi * r;
  double acc = w0 * F;
  for (int l0 = 0; l0 < k; l0 += kChunk) {
    wpair t[kChunk];
#pragma unroll
    for (int s = 0; s < kChunk; ++s) t[s] = up[l0 + s];
#pragma unroll
    for (int s = 0; s < kChunk; ++s) {
      F = (t[s].y * F) * inv_2x;
      acc = __builtin_fma(t[s].x, F, acc);
    }
  }
  return acc;
}

}  // namespace boys
