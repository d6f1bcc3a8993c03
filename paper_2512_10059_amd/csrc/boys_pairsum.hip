// boys_pairsum: the paper's benchmark workload (Sec. III, Algorithm 2) on gfx950:
//
//     z_i = sum_{l=0..k} c_l sum_j F_l(x_i + x_j) y_j ,   i, j = 0..n-1,
//
// i.e. n^2 Boys evaluations formed on the fly, with the weighted sum
// accumulated inside the recurrence.  The work is VALU-bound (no per-pair
// memory traffic).
//
// Divergence control: the arguments are first sorted (a bitonic sort of
// (x, index) pairs, below), so the 64 rows of a wave hold nearly equal x_i and, for
// a given j, x_i + x_j falls in one region for the whole wave except within
// a sliver around the region boundaries.  Rows are evaluated in sorted order
// and the results scattered back.  Each thread owns one row i; the j loop
// runs over chunks staged in LDS (x_j, y_j read by all lanes at once) and
// sums every chunk separately before adding it to the row total, which keeps
// the accumulated rounding at (chunk + n/chunk) ulps instead of n.
#include <hip/hip_runtime.h>

#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>
#include <utility>

#include "boys.h"
#include "boys_common.hpp"
#include "boys_device_f64_batched.hpp"

namespace boys {
namespace {

constexpr int kPairChunk = 512;

// Weights up to the highest order of any table set (40).
struct PairWeights {
  double c[kHighKmax + 1];
};

// Region B in closed form.  With g = 1/(2x) the upward recurrence
// F_{l+1} = g ((2l+1) F_l - e^-x) unrolls to F_l = A_l(g) F_0 - e^-x B_l(g),
//     A_l = (2l-1)!! g^l,   B_0 = 0,   B_{l+1} = g ((2l+1) B_l + 1),
// so sum_l c_l F_l = F_0 P(g) - e^-x Q(g) with P(g) = sum_l c_l A_l(g) and
// Q(g) = sum_l c_l B_l(g), polynomials in g whose coefficients depend only on
// the weights (formed once per call on the host).  Two Horner passes take two
// fused multiply-adds per order instead of a multiply and two fused
// multiply-adds.  From x0 on the recurrence does not amplify errors
// (prod (n+1/2)/x <= 1), so |c_l A_l F_0| and |c_l e B_l| stay below
// |c_l| F_0: the absolute rounding stays on the scale of the recurrence's,
// and an error in F_0 propagates as A_l, exactly as through the recurrence.
// The kernel runs both passes in h = 1/x = 2g: the coefficient of g^l is
// stored times 2^-l, so every Horner step is the step in g times a power of
// two, which rounds identically (bit for bit, short of underflow), and the
// multiply forming g is saved.
struct PairBPoly {
  double p[kHighKmax + 1];  // coefficients of P(h/2) in h, degree 0 upwards
  double q[kHighKmax + 1];  // coefficients of Q(h/2) (q[0] = 0)
};

// Region A in closed form.  The downward recurrence from F_K = S,
// F_l = (t F_{l+1} + e^-x)/(2l+1) with t = 2x, unrolls to
// F_l = A_l(t) S + e^-x B_l(t) with
//     A_l = t^(K-l) (2l-1)!!/(2K-1)!!,
//     B_l = sum_{m=l}^{K-1} t^(m-l) (2l-1)!!/(2m+1)!!,
// so sum_l c_l F_l = S U(t) + e^-x V(t), where U = sum c_l A_l has the
// coefficient u_j = c_{K-j} (2K-2j-1)!!/(2K-1)!! of t^j and V = sum c_l B_l
// the coefficient v_j = sum_{l=0}^{K-1-j} c_l (2l-1)!!/(2l+2j+1)!! (v_K = 0):
// two Horner passes, two fused multiply-adds per order instead of the
// recurrence's multiply and two fused multiply-adds.  Every term c_l A_l S
// and c_l B_l e^-x is at most |c_l| F_l in magnitude (both parts of F_l are
// positive), so the rounding of the passes stays on the scale of
// sum_l |c_l| F_l, as in the recurrence; an error in S propagates as A_l,
// exactly as through it.
// As in region B, the passes run in x itself: the coefficient of t^j is
// stored times 2^j (exact), which saves forming t.
struct PairAPoly {
  double u[kHighKmax + 1];  // coefficients of U(2x) in x, degree 0 upwards
  double v[kHighKmax + 1];  // coefficients of V(2x) (v[K] = 0)
};

// e^-v for one operand of a pair argument, or NaN where the product rule
// below must not be used: v < 0 (the pair's sum may still be in the
// domain), v > 700 (the factor would underflow while the pair's sum might
// not) and NaN.  Computed once per row and once per staged x_j.
__device__ __forceinline__ double pair_factor(double v) {
  return v >= 0.0 && v <= 700.0 ? exp_neg(v) : __builtin_nan("");
}

// e^-x of the pair argument x = x_i + x_j from the two operands' factors:
// e^-x_i e^-x_j is one multiply per pair against about 20 instructions of
// exp_neg.  It equals e^-(x_i + x_j) for the exact sum, which differs from
// e^-x at the rounded sum x by at most half an ulp of x relatively (below
// 4e-15 of e^-x in regions A and B), far inside the method's 5e-14.  Where a
// factor is NaN (an operand outside [0, 700], or NaN) the pair falls back to
// exp_neg(x).
__device__ __forceinline__ double pair_exp(double x, double eij) {
  if (!(eij == eij)) eij = exp_neg(x);
  return eij;
}

// The closed forms' coefficient pairs live in LDS and are read through
// pointers of this type.
typedef __attribute__((address_space(3))) const wpair lds_wpair;

// Horner passes of two polynomials of degree K in h whose coefficient pairs
// (a_l, b_l) are read from LDS, fully unrolled (immediate offsets from one
// address register), two pairs at a time and double-buffered: the reads of
// chunk c+1 are issued before the fused multiply-adds of chunk c.  The
// address passes through an empty asm statement that takes the accumulators
// after chunk c-1 as inputs, so no read runs further ahead than that: at
// most four pairs are in registers.  Without it the scheduler issues every
// read at once (4(K+1) more VGPRs), and with the rolled loop this replaces,
// each chunk cost three register moves.  The asm also keeps the reads inside
// the caller's loop, where they would otherwise be hoisted into registers;
// the pointer's value never changes.
template <int K>
__device__ __forceinline__ wpair horner_pairs(double h, lds_wpair *&ab) {
  constexpr int C = 2;
  constexpr int kChunks = (K + C - 1) / C;  // chunk c: l = K-1-cC down to K-C-cC
  const wpair top = ab[K];
  double P = top.x, Q = top.y;
  wpair cur[C], nxt[C];
#pragma unroll
  for (int s = 0; s < C; ++s)
    if (K - 1 - s >= 0) cur[s] = ab[K - 1 - s];
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const int l0 = K - 1 - c * C;
    if (c + 1 < kChunks) {
      asm volatile("" : "+v"(ab) : "v"(P), "v"(Q));
#pragma unroll
      for (int s = 0; s < C; ++s)
        if (l0 - C - s >= 0) nxt[s] = ab[l0 - C - s];
    }
#pragma unroll
    for (int s = 0; s < C; ++s)
      if (l0 - s >= 0) {
        P = __builtin_fma(P, h, cur[s].x);
        Q = __builtin_fma(Q, h, cur[s].y);
      }
#pragma unroll
    for (int s = 0; s < C; ++s)
      if (l0 - C - s >= 0) cur[s] = nxt[s];  // the entries loaded above
  }
  return wpair{P, Q};
}

// Orders up to which region A's coefficients are read as kernel arguments
// (SGPR addends of the Horner steps) rather than as LDS pairs: up to 12 they
// fit in the scalar registers of the pair loop (106 SGPRs at order 12, whose
// 6 spilled ones are read back only outside the loop; at 16, 38 spilled
// inside it), and the paper's benchmark order 12 runs 2.8% faster than with
// LDS pairs; above, LDS pairs (order 24: 190 ms against 230 ms with the
// spills, n = 2^18).
constexpr int kPairSgprOrders = 12;

// sum_{l=0..K} c_l F_l(x) per region with the table set T: regions A and B
// through their closed forms (PairAPoly, PairBPoly), region C by Horner in
// 1/x; eij = e^-x_i e^-x_j (see pair_exp).
template <int K, class T>
__device__ __forceinline__ double pair_weighted(double x, double eij, const PairAPoly &ap,
                                                const PairWeights &dw, lds_wpair *&uv,
                                                lds_wpair *&pq, double rb_top) {
  double acc;
  if (x < T::x0) {  // region A: S U(2x) + e^-x V(2x)
    // e^-x is taken where it is used: formed before the branches, the
    // fallback's -x became a register that the reciprocals then read instead
    // of negating their operand (two more instructions per pair).
    const double S = rational_a_lit_pos<K, T>(x);
    if constexpr (K <= kPairSgprOrders) {
      double U = ap.u[K];
#pragma unroll
      for (int l = K - 1; l >= 0; --l) U = fma_uniform_addend(U, x, ap.u[l]);
      if constexpr (K == 0) {
        acc = U * S;
      } else {  // V has degree K - 1 (v_K = 0)
        double V = ap.v[K - 1];
#pragma unroll
        for (int l = K - 2; l >= 0; --l) V = fma_uniform_addend(V, x, ap.v[l]);
        acc = __builtin_fma(U, S, V * pair_exp(x, eij));
      }
    } else {  // uv[l] = (u_l, v_l)
      const wpair UV = horner_pairs<K>(x, uv);
      acc = __builtin_fma(UV.x, S, UV.y * pair_exp(x, eij));
    }
  } else if (region_c<T>(x)) {
    // x^(-1/2) sum_l (c_l a_l) (1/x)^l by Horner in 1/x (F_l = a_l x^(-l-1/2)
    // beyond x1); x^(-1/2) and 1/x from one reciprocal square root r.
    const double r = ::rsqrt(x);
    const double g = r * r;
    double P = dw.c[K];
#pragma unroll
    for (int l = K - 1; l >= 0; --l) P = fma_uniform_addend(P, g, dw.c[l]);
    acc = P * r;
  } else {  // region B (and NaN): F_0 P(g) - e^-x Q(g), pq[l] = (p_l, q_l) in h = 2g
    const double h = recip(x);
    const double F0 = rational_b_lit_pos<T>(x, rb_top);
    const wpair PQ = horner_pairs<K>(h, pq);
    acc = __builtin_fma(F0, PQ.x, -(pair_exp(x, eij) * PQ.y));
  }
  return acc;
}

// One staged column j in LDS: (x_j, e^-x_j or NaN: pair_factor) and
// (y_j, unused), so one address register serves both reads of a pair.
struct alignas(32) PairCol {
  wpair xe;
  wpair y;
};

template <int K, class T>
__global__ __launch_bounds__(kBlock) void pairsum_kernel(const double *__restrict__ xs,
                                                         const double *__restrict__ ys, int64_t n,
                                                         PairAPoly ap, PairWeights dw, PairBPoly bp,
                                                         double *__restrict__ zs) {
  __shared__ PairCol s_col[kPairChunk];
  __shared__ wpair s_uv[K + 1], s_pq[K + 1];
  if (threadIdx.x <= K) {
    s_uv[threadIdx.x] = wpair{ap.u[threadIdx.x], ap.v[threadIdx.x]};
    s_pq[threadIdx.x] = wpair{bp.p[threadIdx.x], bp.q[threadIdx.x]};
  }
  // Passed through an empty asm statement every pair (and inside
  // horner_pairs), so their reads are not hoisted out of the pair loop.
  lds_wpair *uv = (lds_wpair *)s_uv;
  lds_wpair *pq = (lds_wpair *)s_pq;
  // r_B's leading numerator coefficient, kept in a VGPR across the loop.
  double rb_top = rb_p_at<T>(T::rb_n);
  asm volatile("" : "+v"(rb_top));
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const double xi = i < n ? xs[i] : 0.0;
  const double ei = pair_factor(xi);
  // A negative sum must give NaN (domain()).  Where neither the wave's rows
  // nor the staged chunk hold a negative operand, every sum is >= 0 or NaN,
  // domain() is the identity on it, and the loop without it runs instead.
  const bool rows_nonneg = __ballot(xi < 0.0) == 0;
  double total = 0.0;
  for (int64_t j0 = 0; j0 < n; j0 += kPairChunk) {
    int negatives = 0;
    for (int t = threadIdx.x; t < kPairChunk; t += kBlock) {
      const int64_t j = j0 + t;
      const double xj = j < n ? xs[j] : 0.0;
      s_col[t].xe = wpair{xj, pair_factor(xj)};
      s_col[t].y = wpair{j < n ? ys[j] : 0.0, 0.0};
      negatives += xj < 0.0;
    }
    const bool chunk_nonneg = __syncthreads_count(negatives) == 0;
    const int m = n - j0 < kPairChunk ? int(n - j0) : kPairChunk;
    double part = 0.0;
    if (rows_nonneg && chunk_nonneg) {
      for (int t = 0; t < m; ++t) {
        asm volatile("" : "+v"(uv), "+v"(pq));
        const wpair xe = s_col[t].xe;
        const double y = s_col[t].y.x;
        part = __builtin_fma(y, pair_weighted<K, T>(xi + xe.x, ei * xe.y, ap, dw, uv, pq, rb_top), part);
      }
    } else {
      for (int t = 0; t < m; ++t) {
        asm volatile("" : "+v"(uv), "+v"(pq));
        const wpair xe = s_col[t].xe;
        const double y = s_col[t].y.x;
        part = __builtin_fma(
            y, pair_weighted<K, T>(domain(xi + xe.x), ei * xe.y, ap, dw, uv, pq, rb_top), part);
      }
    }
    total += part;
    __syncthreads();
  }
  if (i < n) zs[i] = total;
}

// ---------------------------------------------------------------------------
// The sort that orders the arguments: a bitonic network over N = 2^p >= n
// records (key, index), where key is the double's bit pattern mapped to an
// unsigned integer of the same order (sign bit set: all bits flipped; else
// the sign bit set) and index the argument's position.  Records compare by
// key, then by index, so the order is total and the result is that of a
// stable sort by x; the N - n padding records (all-ones key and index) sort
// last.  The order only steers divergence: any permutation gives the same
// sums, so correctness needs only that the first n indices be a permutation
// of 0..n-1, which every compare-exchange network preserves.
//
// Stages with a partner distance j >= kSortSeg/2 run as one global kernel
// each (one compare-exchange per thread); the stages below, and the whole
// sort of each kSortSeg-record segment at the start, run in LDS.  At n = 2^19
// that is 45 launches moving about 0.2 GB, against the pair kernel's 0.4 s.
constexpr int kSortSeg = 2048;  // records per LDS segment (24 KB)

__device__ __forceinline__ uint64_t order_key(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  return (b >> 63) ? ~b : (b | (uint64_t(1) << 63));
}

// (ka, ia) after (kb, ib) in the sort order.
__device__ __forceinline__ bool rec_after(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
  return ka > kb || (ka == kb && ia > ib);
}

__global__ void sort_keys_kernel(const double *__restrict__ x, int64_t n, int64_t N,
                                 uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  keys[i] = i < n ? order_key(x[i]) : ~uint64_t(0);
  vals[i] = i < n ? uint32_t(i) : ~uint32_t(0);
}

// Stages (k, j) for k = kmin, 2 kmin, .., kmax and, within each, j from
// min(k/2, jmax) down to 1, on each segment of seg records (seg a power of
// two <= kSortSeg, j < seg).  Direction by the record's global position i:
// ascending where (i & k) == 0.
__global__ __launch_bounds__(kBlock) void sort_segment_kernel(uint64_t *__restrict__ keys,
                                                              uint32_t *__restrict__ vals, int seg,
                                                              int64_t kmin, int64_t kmax, int jmax) {
  __shared__ uint64_t sk[kSortSeg];
  __shared__ uint32_t sv[kSortSeg];
  const int64_t base = int64_t(blockIdx.x) * seg;
  for (int t = threadIdx.x; t < seg; t += kBlock) {
    sk[t] = keys[base + t];
    sv[t] = vals[base + t];
  }
  __syncthreads();
  for (int64_t k = kmin; k <= kmax; k <<= 1) {
    for (int j = int(k >> 1 < jmax ? k >> 1 : jmax); j > 0; j >>= 1) {
      for (int p = threadIdx.x; p < seg / 2; p += kBlock) {
        const int lo = ((p & ~(j - 1)) << 1) | (p & (j - 1));  // bit j clear
        const int hi = lo | j;
        const bool up = ((base + lo) & k) == 0;
        const uint64_t ka = sk[lo], kb = sk[hi];
        const uint32_t ia = sv[lo], ib = sv[hi];
        if (rec_after(ka, ia, kb, ib) == up) {
          sk[lo] = kb;
          sk[hi] = ka;
          sv[lo] = ib;
          sv[hi] = ia;
        }
      }
      __syncthreads();
    }
  }
  for (int t = threadIdx.x; t < seg; t += kBlock) {
    keys[base + t] = sk[t];
    vals[base + t] = sv[t];
  }
}

// One stage (k, j), j >= kSortSeg / 2, over N records: thread p takes the
// pair (lo, lo + j) with bit j of lo clear, p < N/2.
__global__ __launch_bounds__(kBlock) void sort_stage_kernel(uint64_t *__restrict__ keys,
                                                            uint32_t *__restrict__ vals, int64_t half,
                                                            int64_t k, int64_t j) {
  const int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (p >= half) return;
  const int64_t lo = ((p & ~(j - 1)) << 1) | (p & (j - 1));
  const int64_t hi = lo | j;
  const bool up = (lo & k) == 0;
  const uint64_t ka = keys[lo], kb = keys[hi];
  const uint32_t ia = vals[lo], ib = vals[hi];
  if (rec_after(ka, ia, kb, ib) == up) {
    keys[lo] = kb;
    keys[hi] = ka;
    vals[lo] = ib;
    vals[hi] = ia;
  }
}

// The rows in sorted order: x and y permuted by the sorted indices (the
// first n, all below n).
__global__ void gather_kernel(const double *__restrict__ x, const double *__restrict__ y,
                              const uint32_t *__restrict__ idx, double *__restrict__ xs,
                              double *__restrict__ ys, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    const uint32_t r = idx[i];
    xs[i] = x[r];
    ys[i] = y[r];
  }
}

__global__ void scatter_kernel(const double *__restrict__ zs, const uint32_t *__restrict__ idx,
                               double *__restrict__ z, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) z[idx[i]] = zs[i];
}

using PairKernel = void (*)(const double *, const double *, int64_t, PairAPoly, PairWeights,
                            PairBPoly, double *);

template <class T, std::size_t... K>
constexpr auto make_table(std::index_sequence<K...>) {
  return std::array<PairKernel, sizeof...(K)>{{&pairsum_kernel<int(K), T>...}};
}
constexpr auto kPairTable = make_table<PaperTables>(std::make_index_sequence<kF64Kmax + 1>{});
constexpr auto kPairTableScreen = make_table<ScreenTables>(std::make_index_sequence<kF64Kmax + 1>{});
constexpr auto kPairTableCentre = make_table<CentreTables>(std::make_index_sequence<kF64Kmax + 1>{});
// The per-kmax regions: order K with row K of the per-kmax set (row 32 is
// the paper's set, so K = 32 takes the paper's kernel).
template <std::size_t... K>
constexpr auto make_per_kmax_table(std::index_sequence<K...>) {
  return std::array<PairKernel, sizeof...(K) + 1>{
      {&pairsum_kernel<int(K), PerKmaxTables<int(K)>>..., &pairsum_kernel<kF64Kmax, PaperTables>}};
}
constexpr auto kPairTablePerKmax = make_per_kmax_table(std::make_index_sequence<kF64Kmax>{});
// Orders 33..40: the high-order set.
template <std::size_t... I>
constexpr auto make_high_table(std::index_sequence<I...>) {
  return std::array<PairKernel, sizeof...(I)>{{&pairsum_kernel<kF64Kmax + 1 + int(I), HighTables>...}};
}
constexpr auto kPairTableHigh = make_high_table(std::make_index_sequence<kHighKmax - kF64Kmax>{});

// Per-device workspace: sort records (keys, indices), permuted x, y and z.
struct PairState {
  std::mutex mu;
  void *buf = nullptr;
  size_t bytes = 0;
  // Buffers replaced by larger ones; work already enqueued may still use
  // them, so they are freed only by boys_finalize (after a device sync).
  std::vector<void *> retired;
};
constexpr int kMaxDevices = 64;
PairState g_pair[kMaxDevices];

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

void pairsum_release_all() {
  int cur = 0;
  const bool have = hipGetDevice(&cur) == hipSuccess;
  for (int d = 0; d < kMaxDevices; ++d) {
    PairState &s = g_pair[d];
    std::lock_guard<std::mutex> lock(s.mu);
    if (!s.buf && s.retired.empty()) continue;
    if (hipSetDevice(d) != hipSuccess) continue;
    (void)hipDeviceSynchronize();
    if (s.buf) (void)hipFree(s.buf);
    for (void *old : s.retired) (void)hipFree(old);
    s.retired.clear();
    s.buf = nullptr;
    s.bytes = 0;
  }
  if (have) (void)hipSetDevice(cur);
}

}  // namespace boys

extern "C" int boys_pairsum(const double *x, const double *y, int64_t n, const double *c, int kmax,
                            double *z, hipStream_t stream) {
  return boys_pairsum_tol(x, y, n, c, kmax, boys::PaperTables::eps, z, stream);
}

extern "C" int boys_pairsum_tol(const double *x, const double *y, int64_t n, const double *c,
                                int kmax, double tol, double *z, hipStream_t stream) {
  using namespace boys;
  if (n < 0 || n > (int64_t(1) << 31) - 1 || kmax < 0 || kmax > kHighKmax) return BOYS_EINVAL;
  const int set = table_set_for(kmax, tol);
  if (set < 0) return BOYS_EINVAL;
  if (n == 0) return BOYS_OK;
  if (!x || !y || !c || !z) return BOYS_EINVAL;
  if (overlaps(z, n * 8, x, n * 8) || overlaps(z, n * 8, y, n * 8)) return BOYS_EINVAL;
  if (int st = check_device()) return st;
  if (int st = check_not_capturing(stream)) return st;
  int dev = 0;
  BOYS_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return BOYS_ENOTSUP;

  PairWeights dw{};  // c_l a_l for region C
  long double a_hi = kAsymCoefHost[kAsymOrders - 1];  // a_l beyond the table: a_l = a_{l-1} (l - 1/2)
  for (int l = 0; l <= kmax; ++l) {
    if (l >= kAsymOrders) a_hi *= l - 0.5L;
    dw.c[l] = c[l] * (l < kAsymOrders ? kAsymCoefHost[l] : double(a_hi));
  }
  // Region A's polynomials U and V (see PairAPoly), in long double, with
  // df[l] = (2l-1)!! (exact in long double up to l = 20, within a few units
  // of its last place beyond); rounded to double, then scaled by 2^j.
  PairAPoly ap{};
  {
    long double df[kHighKmax + 2];
    df[0] = 1.0L;
    for (int l = 1; l <= kmax + 1; ++l) df[l] = df[l - 1] * (2 * l - 1);
    for (int j = 0; j <= kmax; ++j) {
      const int l = kmax - j;
      ap.u[j] = std::ldexp(double((long double)c[l] * df[l] / df[kmax]), j);
      long double v = 0.0L;
      for (int m = 0; m <= kmax - 1 - j; ++m) v += (long double)c[m] * df[m] / df[m + j + 1];
      ap.v[j] = std::ldexp(double(v), j);
    }
  }
  // Region B's polynomials P and Q (see PairBPoly), in long double:
  // A_l = a_l g^l with a_l = (2l-1)!!, B_l = sum_j b_j g^j; rounded to
  // double, then scaled by 2^-l.
  PairBPoly bp{};
  {
    long double a = 1.0L, b[kHighKmax + 2] = {}, pq_p[kHighKmax + 1] = {}, pq_q[kHighKmax + 1] = {};
    for (int l = 0; l <= kmax; ++l) {
      pq_p[l] = (long double)c[l] * a;
      for (int j = 1; j <= l; ++j) pq_q[j] += (long double)c[l] * b[j];
      // B_{l+1} = g ((2l+1) B_l + 1): shift up by one power of g.
      for (int j = l + 1; j >= 2; --j) b[j] = (2 * l + 1) * b[j - 1];
      b[1] = 1.0L;
      a *= 2 * l + 1;
    }
    for (int l = 0; l <= kmax; ++l) {
      bp.p[l] = std::ldexp(double(pq_p[l]), -l);
      bp.q[l] = std::ldexp(double(pq_q[l]), -l);
    }
  }

  int64_t N = 1;  // records of the sort: the power of two >= n
  while (N < n) N <<= 1;
  const size_t un = size_t(n), uN = size_t(N);
  const size_t off_keys = 0;
  const size_t off_vals = off_keys + align256(8 * uN);
  const size_t off_xs = off_vals + align256(4 * uN);
  const size_t off_ys = off_xs + align256(8 * un);
  const size_t off_zs = off_ys + align256(8 * un);
  size_t need = off_zs + align256(8 * un);

  PairState &s = g_pair[dev];
  std::lock_guard<std::mutex> lock(s.mu);
  const size_t old_bytes = s.bytes;
  if (s.bytes < need) {
    if (s.buf) {
      // Earlier calls may still be using it: retire it rather than wait.
      s.retired.push_back(s.buf);
      s.buf = nullptr;
      s.bytes = 0;
    }
    // Grow geometrically, so the retired buffers stay below the current one.
    need = need > 2 * old_bytes ? need : 2 * old_bytes;
    if (hipMalloc(&s.buf, need) != hipSuccess) {
      (void)hipGetLastError();
      s.buf = nullptr;
      return BOYS_ENOMEM;
    }
    s.bytes = need;
  }
  char *base = static_cast<char *>(s.buf);
  uint64_t *keys = reinterpret_cast<uint64_t *>(base + off_keys);
  uint32_t *vals = reinterpret_cast<uint32_t *>(base + off_vals);
  double *xs = reinterpret_cast<double *>(base + off_xs);
  double *ys = reinterpret_cast<double *>(base + off_ys);
  double *zs = reinterpret_cast<double *>(base + off_zs);

  const unsigned g = unsigned((n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(sort_keys_kernel, dim3(unsigned((N + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream, x,
                     n, N, keys, vals);
  BOYS_TRY_HIP(hipGetLastError());
  // Segments sorted in LDS (directions alternating with the global
  // position), then each merge size k > seg: global stages while j >= seg,
  // the rest in LDS.
  const int seg = int(N < kSortSeg ? N : kSortSeg);
  const unsigned nseg = unsigned(N / seg);
  if (N > 1) {
    hipLaunchKernelGGL(sort_segment_kernel, dim3(nseg), dim3(kBlock), 0, stream, keys, vals, seg, int64_t(2),
                       int64_t(seg), seg);
    BOYS_TRY_HIP(hipGetLastError());
  }
  const unsigned gh = unsigned((N / 2 + kBlock - 1) / kBlock);
  for (int64_t k = int64_t(seg) << 1; k <= N; k <<= 1) {
    for (int64_t j = k >> 1; j >= seg; j >>= 1) {
      hipLaunchKernelGGL(sort_stage_kernel, dim3(gh), dim3(kBlock), 0, stream, keys, vals, N / 2, k, j);
      BOYS_TRY_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(sort_segment_kernel, dim3(nseg), dim3(kBlock), 0, stream, keys, vals, seg, k, k,
                       seg >> 1);
    BOYS_TRY_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(gather_kernel, dim3(g), dim3(kBlock), 0, stream, x, y, vals, xs, ys, n);
  BOYS_TRY_HIP(hipGetLastError());
  PairKernel kernel = kPairTable[kmax < kF64Kmax ? kmax : kF64Kmax];
  if (set == kSetHigh) kernel = kPairTableHigh[kmax - kF64Kmax - 1];
  else if (set == kSetScreen) kernel = kPairTableScreen[kmax];
  else if (table_variant() == BOYS_TABLES_PER_KMAX) kernel = kPairTablePerKmax[kmax];
  else if (table_variant() == BOYS_TABLES_CENTRE) kernel = kPairTableCentre[kmax];
  hipLaunchKernelGGL(kernel, dim3(g), dim3(kBlock), 0, stream, xs, ys, n, ap, dw, bp, zs);
  BOYS_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(scatter_kernel, dim3(g), dim3(kBlock), 0, stream, zs, vals, z, n);
  return hip_status(hipGetLastError());
}
