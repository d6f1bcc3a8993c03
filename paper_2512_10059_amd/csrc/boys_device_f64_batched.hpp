// Runtime-order evaluation helpers for the batched consumer (one order per
// tile, not a compile-time constant), built on the FP64 method of
// boys_device_f64.hpp.
#pragma once

#include <type_traits>

#include "boys_device_f64.hpp"
#include "boys_consumer_tables.h"

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

// a + c for a compile-time (hence wave-uniform) c, issued as VOP3 v_add_f64
// with c in an SGPR pair; written as asm so that it is not contracted with
// the product that feeds it.
__device__ __forceinline__ double add_uniform(double a, double c) {
  double r;
  asm("v_add_f64 %0, %1, %2" : "=v"(r) : "v"(a), "s"(c));
  return r;
}

// ---------------------------------------------------------------------------
// e^{-x} for the VALU-bound kernels, without a table: Cody and Waite's
// argument reduction, then a Taylor polynomial.  With n = rint(x/ln2) and
// r = n ln2 - x (ln2 carried as LN2_HI + LN2_LO, |r| <= ln2/2 plus rounding),
//     e^{-x} = 2^(-n) * e^r,
// and e^r from its degree-13 Taylor polynomial, whose truncation is below
// 1e-17 relative.  n LN2_HI - x is exact under the fused multiply-add (both
// terms are multiples of 2^-53 within 1/2 of each other when x >= 1/2, and
// n = 0 below), so the reduction rounds once, in the LN2_LO step.  The result
// is within about 2^-52 relative.  Against about 46 VALU instructions of the
// library routine this takes 21, since the domain needs no overflow,
// underflow or special-value handling: the callers pass 0 <= x < 2^10 or NaN
// (NaN propagates through r; past x = 708 the scaling underflows to 0, on
// lanes whose result is discarded).
constexpr double kExpInvLn2 = BOYS_EXP_INV_LN2;
constexpr double kExpLn2Hi = BOYS_EXP_LN2_HI;
constexpr double kExpLn2Lo = BOYS_EXP_LN2_LO;
constexpr int kExpDegree = BOYS_EXP_DEGREE;
constexpr double kExpTaylor[kExpDegree + 1] = BOYS_EXP_TAYLOR_INIT;

// e^{-x} (see above).  The constants are literals; the Horner steps take
// theirs as SGPR addends.  The top term is a product and a sum, each with
// one SGPR operand, instead of a fused multiply-add with two constants, one
// of which would first be moved into VGPRs; its extra rounding is on a term
// below 2^-52 of the result.
__device__ __forceinline__ double exp_neg(double x) {
  const double nd = __builtin_rint(x * kExpInvLn2);
  double r = __builtin_fma(nd, kExpLn2Hi, -x);
  r = __builtin_fma(nd, kExpLn2Lo, r);
  double p = add_uniform(r * kExpTaylor[kExpDegree], kExpTaylor[kExpDegree - 1]);
#pragma unroll
  for (int j = kExpDegree - 2; j >= 0; --j) p = fma_uniform_addend(p, r, kExpTaylor[j]);
  return __builtin_amdgcn_ldexp(p, -int(nd));
}

// ---------------------------------------------------------------------------
// r_{A,K} and r_B of a table set T at a compile-time order (the pair kernel
// and region B).  The coefficients are indexed as compile-time constants, so
// they are literals materialised where they are used (two scalar moves per
// coefficient, SGPR addends of the Horner steps); read through a pointer they
// became scalar loads hoisted out of the pair loop, which together with the
// weights' 52 SGPRs spilled scalar registers.
template <class T>
constexpr bool monic_rows() {
  for (int k = 0; k <= kF64Kmax; ++k)
    if (T::ra_q[k][T::ra_m[k]] != 1.0) return false;
  return T::rb_q[T::rb_m] == 1.0;
}
static_assert(monic_rows<PaperTables>() && monic_rows<ScreenTables>(), "denominators are monic");

template <int K, class T>
__device__ __forceinline__ double rational_a_t(double x) {
  constexpr int n = T::ra_n[K], m = T::ra_m[K];
  double p = T::ra_p[K][n];
#pragma unroll
  for (int i = n - 1; i >= 0; --i) p = fma_uniform_addend(p, x, T::ra_p[K][i]);
  double q = x + T::ra_q[K][m - 1];
#pragma unroll
  for (int i = m - 2; i >= 0; --i) q = fma_uniform_addend(q, x, T::ra_q[K][i]);
  return p / q;
}

template <class T>
__device__ __forceinline__ double rational_b_t(double x) {
  double p = T::rb_p[T::rb_n];
#pragma unroll
  for (int i = T::rb_n - 1; i >= 0; --i) p = fma_uniform_addend(p, x, T::rb_p[i]);
  double q = x + T::rb_q[T::rb_m - 1];
#pragma unroll
  for (int i = T::rb_m - 2; i >= 0; --i) q = fma_uniform_addend(q, x, T::rb_q[i]);
  return p / q;
}

// ---------------------------------------------------------------------------
// r_{A,k} for a runtime, wave-uniform k (the batched consumer).  The rows of
// a table set live in a constant-memory table read with wide scalar loads at
// the address of row k, instead of a 33-way branch to literal-coded passes.
// Rows are stored for fixed-length Horner passes: P with zeros above n_k, Q
// monic with its leading 1 at m_k and zeros above.  The extra leading steps
// compute 0*x + 0 = 0, then 0*x + 1 = 1, then 1*x + q_{m-1}, which is the
// x + q_{m-1} of the exact-length pass rounded once, so the result is the
// same to the last bit.  Two pass lengths cover the orders: the largest
// (n, m) over all orders for k < kSplitK, and the largest over k >= kSplitK
// for the rest ((8, 13) and (8, 9) for the paper's tables, (7, 10) and
// (7, 7) for the screening set).
constexpr int kSplitK = 8;

template <class T>
constexpr int max_ra_n() {
  int v = 0;
  for (int k = 0; k <= kF64Kmax; ++k) v = T::ra_n[k] > v ? T::ra_n[k] : v;
  return v;
}
template <class T>
constexpr int max_ra_m(int from) {
  int v = 0;
  for (int k = from; k <= kF64Kmax; ++k) v = T::ra_m[k] > v ? T::ra_m[k] : v;
  return v;
}

template <class T>
struct RtRows {
  static constexpr int pad_n = max_ra_n<T>();
  static constexpr int pad_m = max_ra_m<T>(0);
  static constexpr int hi_m = max_ra_m<T>(kSplitK);
  double p[kF64Kmax + 1][pad_n + 1];
  double q[kF64Kmax + 1][pad_m + 1];
};

template <class T>
constexpr RtRows<T> make_rt_rows() {
  RtRows<T> t{};
  for (int k = 0; k <= kF64Kmax; ++k) {
    for (int i = 0; i <= T::ra_n[k]; ++i) t.p[k][i] = T::ra_p[k][i];
    for (int i = 0; i <= T::ra_m[k]; ++i) t.q[k][i] = T::ra_q[k][i];
  }
  return t;
}

static_assert(RtRows<PaperTables>::pad_n == BOYS_RA_NMAX && RtRows<PaperTables>::pad_m == BOYS_RA_MMAX &&
                  RtRows<PaperTables>::hi_m == 9,
              "the paper's rows take the (8, 13) and (8, 9) passes");
static __constant__ const RtRows<PaperTables> kRaRows = make_rt_rows<PaperTables>();
static __constant__ const RtRows<ScreenTables> kRaRowsScreen = make_rt_rows<ScreenTables>();

template <class T>
__device__ __forceinline__ const RtRows<T> &rt_rows() {
  if constexpr (std::is_same_v<T, ScreenTables>) return kRaRowsScreen;
  else return kRaRows;
}

// p(x)/q(x) by Horner passes of NP and NQ steps over P[0..NP], Q[0..NQ].
template <int NP, int NQ>
__device__ __forceinline__ double rational_loaded(double x, const double *P, const double *Q) {
  double p = P[NP];
#pragma unroll
  for (int i = NP - 1; i >= 0; --i) p = fma_uniform_addend(p, x, P[i]);
  double q = Q[NQ];
#pragma unroll
  for (int i = NQ - 1; i >= 0; --i) q = fma_uniform_addend(q, x, Q[i]);
  return p / q;
}

template <class T = PaperTables>
__device__ __forceinline__ double rational_a_rt(double x, int k) {
  using R = RtRows<T>;
  const R &rows = rt_rows<T>();
  const double *P = rows.p[k];
  const double *Q = rows.q[k];
  if (k < kSplitK) return rational_loaded<R::pad_n, R::pad_m>(x, P, Q);
  return rational_loaded<R::pad_n, R::hi_m>(x, P, Q);
}

// ---------------------------------------------------------------------------
// Region C in closed form.  The asymptote F_0 = (sqrt(pi)/2) x^(-1/2) and its
// recurrence F_{l+1} = F_l (l + 1/2)/x give F_l = a_l x^(-l-1/2) with
// a_l = Gamma(l + 1/2)/2, so a weighted sum over orders is
//     sum_l w_l F_l = x^(-1/2) * sum_l (w_l a_l) (1/x)^l,
// a polynomial in 1/x whose coefficients d_l = w_l a_l are formed once per
// batch or call: Horner takes one fused multiply-add per order instead of
// two multiplies and one fused multiply-add.  Each Horner partial sum times
// x^(-1/2) (1/x)^l is a tail sum_{m>=l} w_m F_m, so its rounding stays on the
// scale of sum_m |w_m| F_m, as in the recurrence.
constexpr int kAsymOrders = BOYS_ASYM_ORDERS;
constexpr double kAsymCoefHost[kAsymOrders] = BOYS_ASYM_COEF_INIT;
static __constant__ const double kAsymCoef[kAsymOrders] = BOYS_ASYM_COEF_INIT;
static_assert(kAsymOrders == kF64Kmax + 1, "one coefficient per order");

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
template <class T = PaperTables>
__device__ __forceinline__ double wsum_region_a(double x, int k, double wk, const wpair *down) {
  const double e = exp_neg(x);
  const double two_x = x + x;
  double F = rational_a_rt<T>(x, k);
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
template <class T = PaperTables>
__device__ __forceinline__ double wsum_region_b(double x, int k, double w0, const wpair *up) {
  const double e = exp_neg(x);
  const double inv_2x = 0.5 / x;
  double F = rational_b_t<T>(x);
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

// Region C: x^(-1/2) P(1/x) with P(g) = sum_l d_l g^l, d_l = w_l a_l.  The
// per-wave table holds d_0..d_32 with zeros above k, 16-byte aligned; Horner
// starts at k rounded up to a whole chunk, where the zeros above k leave P = 0
// until d_k.  x^(-1/2) and 1/x come from one reciprocal square root r (1/x =
// r^2, within a few ulps, which the asymptote's own 5e-14 bound dwarfs).
constexpr int kAsymTableLen = kAsymOrders + 1;  // even: rows stay 16-byte aligned
__device__ __forceinline__ double wsum_region_c(double x, int k, const double *asym) {
  const double r = ::rsqrt(x);
  const double g = r * r;
  const int top = (k + kChunk - 1) & ~(kChunk - 1);
  double P = asym[top];
  for (int l0 = top - kChunk; l0 >= 0; l0 -= kChunk) {
    const wpair d01 = *reinterpret_cast<const wpair *>(&asym[l0]);
    const wpair d23 = *reinterpret_cast<const wpair *>(&asym[l0 + 2]);
    P = __builtin_fma(P, g, d23.y);
    P = __builtin_fma(P, g, d23.x);
    P = __builtin_fma(P, g, d01.y);
    P = __builtin_fma(P, g, d01.x);
  }
  return P * r;
}

}  // namespace boys
