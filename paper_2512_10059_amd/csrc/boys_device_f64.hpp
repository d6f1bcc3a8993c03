// Device-side FP64 Boys-function evaluation (Algorithm 1, Sec. II F of
// arXiv 2512.10059) for gfx950.  Everything stays in VGPRs; the coefficient
// tables are compile-time constants, so every coefficient becomes an
// instruction literal or an SGPR pair and nothing is looked up in memory.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "boys_coeffs_f64.h"
#include "boys_coeffs_f64_screen.h"
#include "boys_coeffs_f64_high.h"
#include "boys_coeffs_f64_perk.h"
#include "boys_coeffs_f64_centre.h"

namespace boys {

constexpr int kF64Kmax = BOYS_F64_KMAX;
constexpr double kHalfSqrtPi = 0.88622692545275801364908374167057259;

// A table set of the method: region constants and the coefficients of r_B
// and r_{A,k}, k = 0..kmax, from degree 0 upwards with monic denominators
// (q[m] = 1).  PaperTables are the appendix's (eps_tol = 5e-14, kmax = 32,
// Sec. II F).  The others repeat the construction with the Remez tool and the
// Walsh-table degree choice: ScreenTables at eps_tol = 1e-10 (same x0, which
// depends only on kmax; x1 from the asymptote-error equation at 1e-10), and
// HighTables at 5e-14 for orders up to 40 (x0 and x1 of kmax = 40).
struct PaperTables {
  static constexpr int kmax = kF64Kmax;
  static constexpr double eps = 5e-14;
  static constexpr double x0 = BOYS_F64_X0;  // A = [0, x0)
  static constexpr double x1 = BOYS_F64_X1;  // C = (x1, inf), see region_c()
  static constexpr int rb_n = BOYS_RB_N, rb_m = BOYS_RB_M;
  static constexpr int ra_n[kF64Kmax + 1] = BOYS_RA_DEG_N_INIT;
  static constexpr int ra_m[kF64Kmax + 1] = BOYS_RA_DEG_M_INIT;
  static constexpr double ra_p[kF64Kmax + 1][BOYS_RA_NMAX + 1] = BOYS_RA_P_INIT;
  static constexpr double ra_q[kF64Kmax + 1][BOYS_RA_MMAX + 1] = BOYS_RA_Q_INIT;
  static constexpr double rb_p[BOYS_RB_N + 1] = BOYS_RB_P_INIT;
  static constexpr double rb_q[BOYS_RB_M + 1] = BOYS_RB_Q_INIT;
};

struct ScreenTables {
  static constexpr int kmax = BOYS_SCR_KMAX;
  static constexpr double eps = BOYS_SCR_EPS;
  static constexpr double x0 = BOYS_SCR_X0;
  static constexpr double x1 = BOYS_SCR_X1;
  static constexpr int rb_n = BOYS_SCR_RB_N, rb_m = BOYS_SCR_RB_M;
  static constexpr int ra_n[kF64Kmax + 1] = BOYS_SCR_RA_DEG_N_INIT;
  static constexpr int ra_m[kF64Kmax + 1] = BOYS_SCR_RA_DEG_M_INIT;
  static constexpr double ra_p[kF64Kmax + 1][BOYS_SCR_RA_NMAX + 1] = BOYS_SCR_RA_P_INIT;
  static constexpr double ra_q[kF64Kmax + 1][BOYS_SCR_RA_MMAX + 1] = BOYS_SCR_RA_Q_INIT;
  static constexpr double rb_p[BOYS_SCR_RB_N + 1] = BOYS_SCR_RB_P_INIT;
  static constexpr double rb_q[BOYS_SCR_RB_M + 1] = BOYS_SCR_RB_Q_INIT;
};

constexpr int kHighKmax = BOYS_HIGH_KMAX;
struct HighTables {
  static constexpr int kmax = kHighKmax;
  static constexpr double eps = BOYS_HIGH_EPS;
  static constexpr double x0 = BOYS_HIGH_X0;
  static constexpr double x1 = BOYS_HIGH_X1;
  static constexpr int rb_n = BOYS_HIGH_RB_N, rb_m = BOYS_HIGH_RB_M;
  static constexpr int ra_n[kHighKmax + 1] = BOYS_HIGH_RA_DEG_N_INIT;
  static constexpr int ra_m[kHighKmax + 1] = BOYS_HIGH_RA_DEG_M_INIT;
  static constexpr double ra_p[kHighKmax + 1][BOYS_HIGH_RA_NMAX + 1] = BOYS_HIGH_RA_P_INIT;
  static constexpr double ra_q[kHighKmax + 1][BOYS_HIGH_RA_MMAX + 1] = BOYS_HIGH_RA_Q_INIT;
  static constexpr double rb_p[BOYS_HIGH_RB_N + 1] = BOYS_HIGH_RB_P_INIT;
  static constexpr double rb_q[BOYS_HIGH_RB_M + 1] = BOYS_HIGH_RB_Q_INIT;
};
static_assert(ScreenTables::kmax == kF64Kmax && HighTables::eps == PaperTables::eps,
              "the screening set covers the paper's orders; the high-order set its accuracy");

// The paper's x0 and x1 and accuracy, with r_B and every r_{A,k} refitted at
// the Walsh-table entry nearest the centre of the first feasible
// anti-diagonal (n close to m), the alternative choice of Sec. II D.
struct CentreTables {
  static constexpr int kmax = BOYS_CTR_KMAX;
  static constexpr double eps = BOYS_CTR_EPS;
  static constexpr double x0 = BOYS_CTR_X0;
  static constexpr double x1 = BOYS_CTR_X1;
  static constexpr int rb_n = BOYS_CTR_RB_N, rb_m = BOYS_CTR_RB_M;
  static constexpr int ra_n[kF64Kmax + 1] = BOYS_CTR_RA_DEG_N_INIT;
  static constexpr int ra_m[kF64Kmax + 1] = BOYS_CTR_RA_DEG_M_INIT;
  static constexpr double ra_p[kF64Kmax + 1][BOYS_CTR_RA_NMAX + 1] = BOYS_CTR_RA_P_INIT;
  static constexpr double ra_q[kF64Kmax + 1][BOYS_CTR_RA_MMAX + 1] = BOYS_CTR_RA_Q_INIT;
  static constexpr double rb_p[BOYS_CTR_RB_N + 1] = BOYS_CTR_RB_P_INIT;
  static constexpr double rb_q[BOYS_CTR_RB_M + 1] = BOYS_CTR_RB_Q_INIT;
};
static_assert(CentreTables::kmax == kF64Kmax && CentreTables::x0 == PaperTables::x0 &&
                  CentreTables::x1 == PaperTables::x1 && CentreTables::eps == PaperTables::eps,
              "the centre set keeps the paper's regions and accuracy");

// Per-kmax regions (Sec. II C): x0 and x1 follow from the highest order a
// call evaluates, so a call that stops at K < 32 can use x0(K) and x1(K) of
// its own K, with the two approximants such a call needs: r_B on
// [x0(K), x1(K)] and r_{A,K} on [0, x0(K)].  Row K of every array belongs to
// kmax = K (ra_* row K is r_{A,K} fitted on [0, x0(K)]); row 32 is the
// paper's set.  A runtime-order kernel reading row k takes x0, x1 and r_B of
// the same row.
struct PerKmaxSet {
  static constexpr int kmax = BOYS_PK_KMAX;
  static constexpr double eps = BOYS_PK_EPS;
  static constexpr double x0s[kF64Kmax + 1] = BOYS_PK_X0_INIT;
  static constexpr double x1s[kF64Kmax + 1] = BOYS_PK_X1_INIT;
  static constexpr int rb_ns[kF64Kmax + 1] = BOYS_PK_RB_N_INIT;
  static constexpr int rb_ms[kF64Kmax + 1] = BOYS_PK_RB_M_INIT;
  static constexpr double rb_ps[kF64Kmax + 1][BOYS_PK_RB_NMAX + 1] = BOYS_PK_RB_P_INIT;
  static constexpr double rb_qs[kF64Kmax + 1][BOYS_PK_RB_MMAX + 1] = BOYS_PK_RB_Q_INIT;
  static constexpr int ra_n[kF64Kmax + 1] = BOYS_PK_RA_N_INIT;
  static constexpr int ra_m[kF64Kmax + 1] = BOYS_PK_RA_M_INIT;
  static constexpr double ra_p[kF64Kmax + 1][BOYS_PK_RA_NMAX + 1] = BOYS_PK_RA_P_INIT;
  static constexpr double ra_q[kF64Kmax + 1][BOYS_PK_RA_MMAX + 1] = BOYS_PK_RA_Q_INIT;
};

// The per-kmax set as a table set of one compile-time order K (the
// write-out and pair kernels): row K's regions and r_B; r_{A,K} is row K of
// ra_*, as for every set.
template <int K>
struct PerKmaxTables : PerKmaxSet {
  static constexpr int kmax = K;
  static constexpr double x0 = x0s[K];
  static constexpr double x1 = x1s[K];
  static constexpr int rb_n = rb_ns[K], rb_m = rb_ms[K];
};

// r_B's coefficient i of a table set: rb_p/rb_q, or row kmax of rb_ps/rb_qs
// for the per-kmax set.  Read as an element of the two-dimensional array
// with constant indices, the coefficients fold into instruction literals and
// SGPR operands, as the fixed sets' do; read through a pointer to the row,
// they became scalar loads hoisted out of the kernels' loops.
template <class T, class = void>
struct RbRows : std::false_type {};
template <class T>
struct RbRows<T, std::void_t<decltype(T::rb_ps)>> : std::true_type {};

template <class T>
__host__ __device__ constexpr double rb_p_at(int i) {
  if constexpr (RbRows<T>::value) return T::rb_ps[T::kmax][i];
  else return T::rb_p[i];
}
template <class T>
__host__ __device__ constexpr double rb_q_at(int i) {
  if constexpr (RbRows<T>::value) return T::rb_qs[T::kmax][i];
  else return T::rb_q[i];
}

constexpr bool per_kmax_row32_is_the_papers() {
  if (PerKmaxSet::x0s[kF64Kmax] != PaperTables::x0 || PerKmaxSet::x1s[kF64Kmax] != PaperTables::x1)
    return false;
  if (PerKmaxSet::rb_ns[kF64Kmax] != PaperTables::rb_n || PerKmaxSet::rb_ms[kF64Kmax] != PaperTables::rb_m)
    return false;
  for (int i = 0; i <= PaperTables::rb_n; ++i)
    if (PerKmaxSet::rb_ps[kF64Kmax][i] != PaperTables::rb_p[i]) return false;
  for (int i = 0; i <= PaperTables::rb_m; ++i)
    if (PerKmaxSet::rb_qs[kF64Kmax][i] != PaperTables::rb_q[i]) return false;
  const int n = PaperTables::ra_n[kF64Kmax], m = PaperTables::ra_m[kF64Kmax];
  if (PerKmaxSet::ra_n[kF64Kmax] != n || PerKmaxSet::ra_m[kF64Kmax] != m) return false;
  for (int i = 0; i <= n; ++i)
    if (PerKmaxSet::ra_p[kF64Kmax][i] != PaperTables::ra_p[kF64Kmax][i]) return false;
  for (int i = 0; i <= m; ++i)
    if (PerKmaxSet::ra_q[kF64Kmax][i] != PaperTables::ra_q[kF64Kmax][i]) return false;
  return true;
}
static_assert(PerKmaxSet::kmax == kF64Kmax && PerKmaxSet::eps == PaperTables::eps &&
                  per_kmax_row32_is_the_papers(),
              "the per-kmax set covers the paper's orders at its accuracy; row 32 is the paper's set");

// The table set for a caller's order and error tolerance: the cheapest set
// that covers kmax and whose guarantee is at most tol (1 = screening, 0 = the
// paper's, 2 = high orders), or -1 if none does (tol below 5e-14 or NaN, or
// kmax above 40).
enum TableSet { kSetNone = -1, kSetPaper = 0, kSetScreen = 1, kSetHigh = 2 };
__host__ __device__ constexpr int table_set_for(int kmax, double tol) {
  if (!(tol >= PaperTables::eps) || kmax < 0 || kmax > HighTables::kmax) return kSetNone;
  if (kmax > PaperTables::kmax) return kSetHigh;
  return tol >= ScreenTables::eps ? kSetScreen : kSetPaper;
}

// The paper's set under its short names (the batched consumer uses these).
constexpr double kX0 = PaperTables::x0;
constexpr double kX1 = PaperTables::x1;
static constexpr auto &kRaN = PaperTables::ra_n;
static constexpr auto &kRaM = PaperTables::ra_m;
static constexpr auto &kRaP = PaperTables::ra_p;
static constexpr auto &kRaQ = PaperTables::ra_q;
static constexpr auto &kRbP = PaperTables::rb_p;
static constexpr auto &kRbQ = PaperTables::rb_q;

// Region C is open at x1.  The printed x1 is the double nearest the root of
// the equation that defines it (asymptote error = eps_tol for F_32) but lies
// just below the root, where the asymptote misses eps_tol by 8e-30; r_B was
// fitted on the closed interval [x0, x1], so x = x1 is evaluated in B.  (The
// screening x1 is the root rounded up.)
template <class T = PaperTables>
__device__ __forceinline__ bool region_c(double x) { return x > T::x1; }

// r_{A,K}(x): Horner on numerator and (monic) denominator, one IEEE division.
template <int K, class T = PaperTables>
__device__ __forceinline__ double rational_a(double x) {
  constexpr int n = T::ra_n[K], m = T::ra_m[K];
  double p = T::ra_p[K][n];
#pragma unroll
  for (int i = n - 1; i >= 0; --i) p = __builtin_fma(p, x, T::ra_p[K][i]);
  if constexpr (m == 0) {
    return p;  // monic of degree 0: q = 1
  } else {
    double q = x + T::ra_q[K][m - 1];
#pragma unroll
    for (int i = m - 2; i >= 0; --i) q = __builtin_fma(q, x, T::ra_q[K][i]);
    return p / q;
  }
}

// r_B(x): F_0 on [x0, x1].
template <class T = PaperTables>
__device__ __forceinline__ double rational_b(double x) {
  double p = rb_p_at<T>(T::rb_n);
#pragma unroll
  for (int i = T::rb_n - 1; i >= 0; --i) p = __builtin_fma(p, x, rb_p_at<T>(i));
  if constexpr (T::rb_m == 0) {
    return p;
  } else {
    double q = x + rb_q_at<T>(T::rb_m - 1);
#pragma unroll
    for (int i = T::rb_m - 2; i >= 0; --i) q = __builtin_fma(q, x, rb_q_at<T>(i));
    return p / q;
  }
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
template <int K, class T = PaperTables>
__device__ __forceinline__ void boys_f64(double x, double (&F)[K + 1]) {
  x = domain(x);
  const double e = ::exp(-x);
  if (x < T::x0) {
    F[K] = rational_a<K, T>(x);
    const double two_x = x + x;
#pragma unroll
    for (int l = K - 1; l >= 0; --l)
      F[l] = __builtin_fma(two_x, F[l + 1], e) * (1.0 / (2 * l + 1));
  } else {
    const bool c = region_c<T>(x);
    const double f0b = rational_b<T>(x);
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
