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
//
// -n is formed directly as rint(-x/ln2) (rounding to nearest even is
// symmetric, so this is exactly -rint(x/ln2)) and n enters the reduction
// through negated operands, which saves the integer negation of the scale.
__device__ __forceinline__ double exp_neg(double x) {
  const double mn = __builtin_rint(-x * kExpInvLn2);  // -n
  double r = __builtin_fma(-mn, kExpLn2Hi, -x);
  r = __builtin_fma(-mn, kExpLn2Lo, r);
  double p = add_uniform(r * kExpTaylor[kExpDegree], kExpTaylor[kExpDegree - 1]);
#pragma unroll
  for (int j = kExpDegree - 2; j >= 0; --j) p = fma_uniform_addend(p, r, kExpTaylor[j]);
  return __builtin_amdgcn_ldexp(p, int(mn));
}

// 1/x for finite x in the normal range: the hardware reciprocal refined by
// two Newton steps (within about one ulp).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// p/q for the rationals' denominators, which are positive and far from the
// ends of the exponent range on every interval the method uses them: the
// hardware reciprocal of q refined by one Newton step, then one correction
// of the quotient,
//     y = p r,  y' = y + r (p - q y).
// v_rcp_f64 is within 4.7e-8 relatively (measured on gfx950: at most 4.6e-8
// over 6.7e7 arguments spanning [1e-3, 1e6]), so after the Newton step r is
// within e = 2.3e-15 (about 10 ulps).  y is then within about 11 ulps of
// p/q, the residual p - q y is formed with at most a rounding of that small
// quantity, and y' = p/q (1 - e^2) + roundings: half an ulp plus under 1e-13
// ulps, so y' is the correctly rounded quotient except where p/q lies that
// close to a rounding boundary (the same 6.7e7 quotients all matched the
// IEEE division).  A second Newton step would change nothing.  Against the
// IEEE division sequence this also drops the scaling and fix-up steps (6
// instructions instead of 11), which only matter near overflow, underflow
// and for special operands; NaN still propagates.
__device__ __forceinline__ double div_positive(double p, double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = __builtin_fma(r, __builtin_fma(-q, r, 1.0), r);
  const double y = p * r;
  return __builtin_fma(__builtin_fma(-q, y, p), r, y);
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
  if constexpr (m == 0) {
    return p;  // monic of degree 0: q = 1
  } else {
    double q = x + T::ra_q[K][m - 1];
#pragma unroll
    for (int i = m - 2; i >= 0; --i) q = fma_uniform_addend(q, x, T::ra_q[K][i]);
    return p / q;
  }
}

template <class T>
__device__ __forceinline__ double rational_b_t(double x) {
  double p = rb_p_at<T>(T::rb_n);
#pragma unroll
  for (int i = T::rb_n - 1; i >= 0; --i) p = fma_uniform_addend(p, x, rb_p_at<T>(i));
  if constexpr (T::rb_m == 0) {
    return p;
  } else {
    double q = x + rb_q_at<T>(T::rb_m - 1);
#pragma unroll
    for (int i = T::rb_m - 2; i >= 0; --i) q = fma_uniform_addend(q, x, rb_q_at<T>(i));
    return p / q;
  }
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
static __constant__ const RtRows<CentreTables> kRaRowsCentre = make_rt_rows<CentreTables>();
static_assert(monic_rows<CentreTables>(), "denominators are monic");

template <class T>
__device__ __forceinline__ const RtRows<T> &rt_rows() {
  static_assert(std::is_same_v<T, PaperTables> || std::is_same_v<T, ScreenTables> ||
                    std::is_same_v<T, CentreTables>,
                "runtime rows exist for the sets of fixed regions");
  if constexpr (std::is_same_v<T, ScreenTables>) return kRaRowsScreen;
  else if constexpr (std::is_same_v<T, CentreTables>) return kRaRowsCentre;
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

// As rational_loaded, with div_positive for the quotient.
template <int NP, int NQ>
__device__ __forceinline__ double rational_loaded_pos(double x, const double *P, const double *Q) {
  double p = P[NP];
#pragma unroll
  for (int i = NP - 1; i >= 0; --i) p = fma_uniform_addend(p, x, P[i]);
  double q = Q[NQ];
#pragma unroll
  for (int i = NQ - 1; i >= 0; --i) q = fma_uniform_addend(q, x, Q[i]);
  return div_positive(p, q);
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

// r_{A,k}(x) for a runtime k with div_positive (the batched consumer).
template <class T = PaperTables>
__device__ __forceinline__ double rational_a_rt_pos(double x, int k) {
  using R = RtRows<T>;
  const R &rows = rt_rows<T>();
  const double *P = rows.p[k];
  const double *Q = rows.q[k];
  if (k < kSplitK) return rational_loaded_pos<R::pad_n, R::pad_m>(x, P, Q);
  return rational_loaded_pos<R::pad_n, R::hi_m>(x, P, Q);
}

// r_{A,K} of a table set with div_positive for the quotient (literal
// coefficients, SGPR addends, as rational_a_t).
template <int K, class T>
__device__ __forceinline__ double rational_a_lit_pos(double x) {
  constexpr int n = T::ra_n[K], m = T::ra_m[K];
  double p = T::ra_p[K][n];
#pragma unroll
  for (int i = n - 1; i >= 0; --i) p = fma_uniform_addend(p, x, T::ra_p[K][i]);
  if constexpr (m == 0) {
    return p;
  } else {
    double q = x + T::ra_q[K][m - 1];
#pragma unroll
    for (int i = m - 2; i >= 0; --i) q = fma_uniform_addend(q, x, T::ra_q[K][i]);
    return div_positive(p, q);
  }
}

// r_B of a table set with div_positive for the quotient (literal
// coefficients, SGPR addends, as rational_b_t).  A caller in a loop may pass
// the numerator's leading coefficient held in a VGPR: the first Horner step
// has it as its multiplicand, which the literal form moves into VGPRs (two
// moves) on every call.
template <class T>
__device__ __forceinline__ double rational_b_lit_pos(double x, double top = rb_p_at<T>(T::rb_n)) {
  double p = top;
#pragma unroll
  for (int i = T::rb_n - 1; i >= 0; --i) p = fma_uniform_addend(p, x, rb_p_at<T>(i));
  if constexpr (T::rb_m == 0) {
    return p;
  } else {
    double q = x + rb_q_at<T>(T::rb_m - 1);
#pragma unroll
    for (int i = T::rb_m - 2; i >= 0; --i) q = fma_uniform_addend(q, x, rb_q_at<T>(i));
    return div_positive(p, q);
  }
}

// ---------------------------------------------------------------------------
// The batched consumer's view of a table set for a batch of order k: the
// region ends and the two approximants.  Sets with fixed regions use their
// x0 and x1, r_{A,k} from the runtime rows above and the literal-coded r_B.
// The per-kmax set takes x0, x1 and r_B of row k as well, so both rationals
// change with k; they are reached by a binary dispatch on the wave-uniform k
// (five or six scalar compares and branches per call) to literal-coded
// passes of each row's exact degrees.  Padding the rows to common lengths
// instead, as for the fixed sets' region A, would add 10-45% to the
// rationals' steps: the rows' (n, m) vary more than the paper's.
#define BOYS_ORDER_CASE(K) \
  case K:                   \
    return f(std::integral_constant<int, K>{});
template <class F>
__device__ __forceinline__ double order_dispatch(int k, const F &f) {
  static_assert(kF64Kmax == 32, "one case per order 0..32");
  switch (k) {
    BOYS_ORDER_CASE(0) BOYS_ORDER_CASE(1) BOYS_ORDER_CASE(2) BOYS_ORDER_CASE(3) BOYS_ORDER_CASE(4)
    BOYS_ORDER_CASE(5) BOYS_ORDER_CASE(6) BOYS_ORDER_CASE(7) BOYS_ORDER_CASE(8) BOYS_ORDER_CASE(9)
    BOYS_ORDER_CASE(10) BOYS_ORDER_CASE(11) BOYS_ORDER_CASE(12) BOYS_ORDER_CASE(13)
    BOYS_ORDER_CASE(14) BOYS_ORDER_CASE(15) BOYS_ORDER_CASE(16) BOYS_ORDER_CASE(17)
    BOYS_ORDER_CASE(18) BOYS_ORDER_CASE(19) BOYS_ORDER_CASE(20) BOYS_ORDER_CASE(21)
    BOYS_ORDER_CASE(22) BOYS_ORDER_CASE(23) BOYS_ORDER_CASE(24) BOYS_ORDER_CASE(25)
    BOYS_ORDER_CASE(26) BOYS_ORDER_CASE(27) BOYS_ORDER_CASE(28) BOYS_ORDER_CASE(29)
    BOYS_ORDER_CASE(30) BOYS_ORDER_CASE(31)
    default:
      return f(std::integral_constant<int, 32>{});
  }
}
#undef BOYS_ORDER_CASE

template <class T>
constexpr bool kPerKmaxRows = std::is_same_v<T, PerKmaxSet>;

template <class T>
__device__ __forceinline__ double batch_x0(int k) {
  if constexpr (kPerKmaxRows<T>) return PerKmaxSet::x0s[k];
  else return T::x0;
}

template <class T>
__device__ __forceinline__ double batch_x1(int k) {
  if constexpr (kPerKmaxRows<T>) return PerKmaxSet::x1s[k];
  else return T::x1;
}

template <class T>
__device__ __forceinline__ double batch_rational_a(double x, int k) {
  if constexpr (kPerKmaxRows<T>) {
    return order_dispatch(k, [x](auto K) {
      return rational_a_lit_pos<decltype(K)::value, PerKmaxTables<decltype(K)::value>>(x);
    });
  } else {
    return rational_a_rt_pos<T>(x, k);
  }
}

template <class T>
__device__ __forceinline__ double batch_rational_b(double x, int k, double top) {
  if constexpr (kPerKmaxRows<T>) {
    return order_dispatch(
        k, [x](auto K) { return rational_b_lit_pos<PerKmaxTables<decltype(K)::value>>(x); });
  } else {
    return rational_b_lit_pos<T>(x, top);
  }
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

// (2l-1)!! and 1/(2l-1)!!, l = 0..32, for the weight sweeps below.
static __constant__ const double kDFact[kF64Kmax + 1] = BOYS_DFACT_INIT;
static __constant__ const double kInvDFact[kF64Kmax + 1] = BOYS_INV_DFACT_INIT;

// Weighted sums for the batched consumer.  The recurrences of Algorithm 1
// are linear in their seed S (r_{A,k} or r_B) and in e^-x, so the weighted
// sum the paper's benchmark accumulates inside the recurrence (Sec. III,
// Algorithm 2) equals u S + v e^-x, and u and v follow from sweeping the
// weights against the direction of the recurrence, substituting one order at
// a time; neither S nor e^-x is needed until the end.
//
// Region A (downward, F_l = c_l (2x F_{l+1} + e^-x), c_l = 1/(2l+1)): after
// substituting F_0..F_{s-1}, sum = u_s F_s + v_s e^-x + sum_{l>s} w_l F_l with
//     u_0 = w_0, v_0 = 0,  u_{s+1} = w_{s+1} + 2x c_s u_s,  v_{s+1} = v_s + c_s u_s.
// With z_s = u_s (2s-1)!!/(2k-1)!! each step is two fused multiply-adds,
//     v_{s+1} = v_s + z_s (2k-1)!!/(2s+1)!!,
//     z_{s+1} = 2x z_s + w_{s+1} (2s+1)!!/(2k-1)!!,
// and sum = z_k S + v_k e^-x.
// Region B (upward, F_{l+1} = g ((2l+1) F_l - e^-x), g = 1/(2x)): from the top,
//     u_k = w_k, v_k = 0,  u_{l-1} = w_{l-1} + (2l-1) g u_l,  v_{l-1} = v_l - g u_l,
// and with z_l = u_l (2l-1)!!, v' = v/g:
//     v'_{l-1} = v'_l - z_l / (2l-1)!!,   z_{l-1} = g z_l + w_{l-1} (2l-3)!!,
// and sum = z_0 S + g v'_0 e^-x.
// The per-order constants sit in per-wave LDS tables of pairs, one 16-byte
// read per step, formed when a wave enters a batch.  Both sweeps are padded to whole chunks of CH steps by zero entries
// on the side they start from, where they leave z and v at exactly 0.
// Rounding: in region A, u_s is a weighted sum of products of the positive
// factors 2x c_l and the recurrence's own terms, so every step's rounding
// reaches the result as at most a few ulps of sum_l |w_l| F_l, as in the
// recurrence; in region B the sweep's terms are at most (2l-1)!!/(2x)^l <= 1
// times F_0 from x0 on (the recurrence does not amplify there), so its
// absolute error is a few (k+1) ulps of F_0 sum_l |w_l|, and an error in S
// propagates exactly as through the recurrence.
typedef double wpair __attribute__((ext_vector_type(2)));
constexpr int kPolyOrders = BOYS_POLY_ORDERS;
static_assert(kPolyOrders == kF64Kmax + 1, "one constant per order");
constexpr int kChunkMax = 8;                          // longest sweep chunk of any configuration
constexpr int kSweepPadA = kChunkMax;                 // zero entries below s = 0
constexpr int kSweepLenA = kSweepPadA + kF64Kmax + 1; // entries s = -8..32
constexpr int kSweepLenB = kF64Kmax + kChunkMax;      // entries l = 1..40

// h t + c as VOP3 v_fma_f64 with its own destination.  The compiler's
// builtin becomes v_fmac_f64, which accumulates into the addend's register:
// in a chain over loaded constants that leaves the chain in a different
// register each step and costs a move per chain and chunk.
__device__ __forceinline__ double fma_step(double h, double t, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(h), "v"(t), "v"(c));
  return r;
}

// Both sweeps take their first chunk apart from the loop: from z = v = 0
// the first step leaves z = a and v = 0 (exactly, for finite x) and the
// second adds v = z b by a multiply, which drops the two zeroing moves and
// two fused multiply-adds per argument.  Padding entries make the first
// chunk whole at every k.

// Region A.  The tables hold the entries scaled by powers of two so that
// the sweep multiplies by x instead of 2x (saving the add that formed 2x):
// ta[kSweepPadA + s] = 2^(k-s) w_s (2s-1)!!/(2k-1)!!, 2^(s-k-1) (2k-1)!!/(2s-1)!!)
// for 1 <= s <= k, (2^k w_0/(2k-1)!!, 0) for s = 0, zeros for s < 0.  After
// entry s the state is (2^(k-s) z_s, v_s) of the unscaled sweep in 2x, since
// scaling by a power of two commutes with rounding: the same result, bit for
// bit (short of underflow, which the entries' sizes rule out).
template <int CH, class T = PaperTables>
__device__ __forceinline__ double wsum_sweep_a(double x, int k, const wpair *ta) {
  static_assert(CH >= 2, "the peeled first chunk has two steps or more");
  const double e = exp_neg(x);
  const double S = batch_rational_a<T>(x, k);
  const int steps = (k + CH) & ~(CH - 1);  // k + 1 rounded up to whole chunks
  const wpair *t = ta + (kSweepPadA + k + 1 - steps);
  wpair q[CH];
#pragma unroll
  for (int s = 0; s < CH; ++s) q[s] = t[s];
  double z = q[0].x;
  double v = z * q[1].y;
  z = fma_step(x, z, q[1].x);
#pragma unroll
  for (int s = 2; s < CH; ++s) {  // z first: neither step reads the other's result
    const double zs = z;
    z = fma_step(x, zs, q[s].x);
    v = fma_step(zs, q[s].y, v);
  }
  for (int c0 = CH; c0 < steps; c0 += CH) {
#pragma unroll
    for (int s = 0; s < CH; ++s) q[s] = t[c0 + s];
#pragma unroll
    for (int s = 0; s < CH; ++s) {
      const double zs = z;
      z = fma_step(x, zs, q[s].x);
      v = fma_step(zs, q[s].y, v);
    }
  }
  return __builtin_fma(z, S, v * e);
}

// Region B.  Unscaled, tb[l-1] = (w_{l-1} (2l-3)!!, -1/(2l-1)!!) for
// 1 <= l <= k, (w_k (2k-1)!!, 0) for l = k+1, zeros above, swept in
// g = 1/(2x).  The tables hold entry i = l-1 as (2^-i a_i, 2^i b_i) and the
// sweep multiplies by h = 1/x = 2g: after entry i the state is
// (2^-i z_i, v_i / 2) of the unscaled sweep, so z comes out unchanged and
// h (v/2) = g v, bit for bit, and the multiply that formed g is saved.
// top_b is r_B's leading numerator coefficient (see rational_b_lit_pos);
// the per-kmax set ignores it.
template <int CH, class T = PaperTables>
__device__ __forceinline__ double wsum_sweep_b(double x, int k, const wpair *tb, double top_b) {
  static_assert(CH >= 2, "the peeled first chunk has two steps or more");
  const double e = exp_neg(x);
  const double h = recip(x);
  const double S = batch_rational_b<T>(x, k, top_b);
  const int top = (k + CH) & ~(CH - 1);  // k + 1 rounded up to whole chunks
  wpair q[CH];
  const wpair *b0 = tb + (top - CH);  // one base, non-negative offsets
#pragma unroll
  for (int s = 0; s < CH; ++s) q[s] = b0[CH - 1 - s];
  double z = q[0].x;
  double v = z * q[1].y;
  z = fma_step(h, z, q[1].x);
#pragma unroll
  for (int s = 2; s < CH; ++s) {  // z first: neither step reads the other's result
    const double zs = z;
    z = fma_step(h, zs, q[s].x);
    v = fma_step(zs, q[s].y, v);
  }
  for (int l0 = top - CH; l0 > 0; l0 -= CH) {
#pragma unroll
    for (int s = 0; s < CH; ++s) q[s] = tb[l0 - 1 - s];
#pragma unroll
    for (int s = 0; s < CH; ++s) {
      const double zs = z;
      z = fma_step(h, zs, q[s].x);
      v = fma_step(zs, q[s].y, v);
    }
  }
  return __builtin_fma(z, S, (h * v) * e);
}

// Region C: x^(-1/2) P(1/x) with P(g) = sum_l d_l g^l, d_l = w_l a_l.  The
// per-wave table holds d_0..d_32 with zeros above k, 16-byte aligned; Horner
// starts at k rounded up to a whole chunk, where the zeros above k leave P = 0
// until d_k.  x^(-1/2) and 1/x come from one reciprocal square root r (1/x =
// r^2, within a few ulps, which the asymptote's own 5e-14 bound dwarfs).
constexpr int kAsymTableLen = kF64Kmax + kChunkMax;  // zeros above k; even: 16-byte rows
__device__ __forceinline__ double wsum_region_c(double x, int k, const double *asym) {
  constexpr int kChunk = 4;
  const double r = ::rsqrt(x);
  const double g = r * r;
  const int top = (k + kChunk - 1) & ~(kChunk - 1);
  double P = asym[top];
  for (int l0 = top - kChunk; l0 >= 0; l0 -= kChunk) {
    const wpair d01 = *reinterpret_cast<const wpair *>(&asym[l0]);
    const wpair d23 = *reinterpret_cast<const wpair *>(&asym[l0 + 2]);
    P = fma_step(P, g, d23.y);
    P = fma_step(P, g, d23.x);
    P = fma_step(P, g, d01.y);
    P = fma_step(P, g, d01.x);
  }
  return P * r;
}

}  // namespace boys
