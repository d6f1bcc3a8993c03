// boys_weighted_sum: batched fused consumer on gfx950.
//
// For every batch b (size n_b, order k_b, weights w_b) and every argument i of
// it:  out[i] = sum_{l=0..k_b} w_{b,l} F_l(x[i]), the weighted sum the paper's
// benchmark accumulates inside the recurrence (Sec. III, Algorithm 2).
//
// Work decomposition.  Each batch is cut into tiles of T = 64*ITEMS
// arguments; a tile has one order, so the recurrence length is uniform over
// it.  A one-block scan kernel turns the batch table into two prefix sums:
// tiles, and cost counted per 64-argument pass (pass_cost below), so partial
// tiles of small batches are not over-weighted.  The main kernel then runs a
// fixed grid of a few workgroups per CU whose waves work independently:
// wave w of W takes the tiles whose cost prefix falls in [w, w+1) * total / W,
// i.e. a contiguous run of tiles of about equal cost, walking the batches in
// order.  There is no shared counter, so the result is deterministic and no
// memory has to be reset between launches.
//
// Divergence.  Argument streams mix all three regions inside every wave, and
// Algorithm 1 takes a different path in each.  With binning enabled the wave
// first sorts its tile by region in LDS (ballot and bit-count ranks), so every
// 64-lane pass except at most two runs a single path; results go back into
// the sorted slots and leave the tile in the original order, each lane
// reading its own items' slots, so the output stores stay coalesced.
//
// The scan and the persistent kernel are launched as one cached hipGraph per
// device; the graph is rebuilt when any argument or the configuration
// changes.  The batch table is read on the device by the graph itself, so
// changing its contents in place is safe.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "boys.h"
#include "boys_common.hpp"
#include "boys_device_f64_batched.hpp"

namespace boys {
namespace {

// Cost of one 64-argument pass of order k, in units of recurrence steps: the
// chunked recurrence runs 4*ceil(k/4) steps, and the region work before it
// (rational, exp, binning, loads and stores) is about 24 steps' worth.
constexpr int kCostBias = 24;
__host__ __device__ __forceinline__ int64_t pass_cost(int k) { return 4 * ((k + 3) / 4) + kCostBias; }
constexpr int kScanThreads = 1024;
constexpr int32_t kMaxBatches = 1 << 24;

struct WsArgs {
  const double *x;
  const int64_t *boff;
  const int32_t *bn;
  const int32_t *bk;
  const double *w;
  const int64_t *woff;
  double *out;
  const int64_t *tile_start;  // [nbatch+1]
  const int64_t *cost_start;  // [nbatch+1]
  int32_t nbatch;
  int32_t taper;  // 0: equal shares per wave; p > 0: shares decreasing with the wave index
};

// Start of wave gw's share of the total cost among W waves.  Waves are
// dispatched in index order, and a SIMD issues from its oldest waves first,
// so the waves of a later round start late and, with equal shares, finish
// last.  With taper p the shares follow F(u) = 1 - (1 - u)^p, u = gw/W:
// the first waves take p times the mean share and the last ones almost
// nothing, so the last round ends soon after the first ones.  Every wave
// computes the boundaries with the same expression, so consecutive shares
// meet exactly; the ends are exact (0 and total).
__device__ __forceinline__ int64_t share_start(int64_t total, int64_t gw, int64_t W, int taper) {
  if (!taper) return total * gw / W;
  const double r = double(W - gw) / double(W);
  double rp = r;
  for (int i = 1; i < taper; ++i) rp *= r;
  return total - int64_t(double(total) * rp);
}

__device__ __forceinline__ int clamp_order(int k) { return k < 0 ? 0 : (k > kF64Kmax ? kF64Kmax : k); }

// A value that is identical in every lane, moved to a scalar register.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v)));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v) >> 32));
  return int64_t((uint64_t(hi) << 32) | lo);
}

// Exclusive prefix sums of tiles and cost over the batches (one workgroup).
// The table is taken in rounds of kScanThreads * kScanPer batches.  Each
// round goes through LDS so that every global access is coalesced:
//   1. the batch sizes and orders are loaded with consecutive lanes on
//      consecutive batches, and each batch's tile count and cost (32-bit: at
//      most 2^24 tiles and 2^25 * 56 cost units for a 2^31-argument batch) are
//      written to LDS;
//   2. thread t reads its kScanPer consecutive batches back and keeps them in
//      registers; thread totals are scanned within each wave by lane
//      shuffles and across the waves in LDS;
//   3. the two 64-bit prefix arrays are staged, one after the other, in the
//      same LDS buffer and written out by consecutive lanes.
// Tiles are powers of two (1 << tile_shift arguments), so every count is an
// add and a shift.
constexpr int kScanPer = 8;
constexpr int kScanRound = kScanThreads * kScanPer;
__global__ __launch_bounds__(kScanThreads) void ws_scan_kernel(const int32_t *__restrict__ bn,
                                                               const int32_t *__restrict__ bk,
                                                               int32_t nbatch, int tile_shift,
                                                               int64_t *__restrict__ tile_start,
                                                               int64_t *__restrict__ cost_start) {
  constexpr int kWaves = kScanThreads / 64;
  // One 64 KB buffer: the per-batch counts (two 32-bit arrays) in step 1,
  // then each 64-bit prefix array in turn in step 3.
  __shared__ __attribute__((aligned(16))) int64_t s_buf[kScanRound];
  __shared__ int64_t s_t[kWaves], s_c[kWaves];
  uint32_t *const s_nt = reinterpret_cast<uint32_t *>(s_buf);
  uint32_t *const s_nc = s_nt + kScanRound;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const uint32_t round_up = (uint32_t(1) << tile_shift) - 1;
  int64_t carry_t = 0, carry_c = 0;  // totals of the earlier rounds
  for (int32_t base = 0; base < nbatch; base += kScanRound) {
    const int32_t m = nbatch - base < kScanRound ? nbatch - base : kScanRound;
    const int32_t *const bnr = bn + base;
    const int32_t *const bkr = bk + base;
    // 1. Coalesced loads from indices clamped into the table (all in flight
    // together); batches past the end count as empty.
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
      const int j = i * kScanThreads + tid;
      const uint32_t jc = uint32_t(j < m ? j : m - 1);
      const int32_t nr = bnr[jc];
      const int kr = bkr[jc];
      const uint32_t n = j < m && nr > 0 ? uint32_t(nr) : 0u;
      s_nt[j] = (n + round_up) >> tile_shift;
      s_nc[j] = ((n + 63u) >> 6) * uint32_t(pass_cost(clamp_order(kr)));
    }
    __syncthreads();
    // 2. Thread t owns batches kScanPer*t .. kScanPer*t + kScanPer-1.
    uint32_t ct[kScanPer], cc[kScanPer];
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
      ct[i] = s_nt[tid * kScanPer + i];
      cc[i] = s_nc[tid * kScanPer + i];
    }
    int64_t st = 0, sc = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
      st += ct[i];
      sc += cc[i];
    }
    int64_t it = st, ic = sc;  // inclusive scan over the wave
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t ut = __shfl_up(it, off);
      const int64_t uc = __shfl_up(ic, off);
      if (lane >= off) {
        it += ut;
        ic += uc;
      }
    }
    if (lane == 63) {
      s_t[wv] = it;
      s_c[wv] = ic;
    }
    __syncthreads();  // also: every thread has read its counts from s_buf
    int64_t tot_t = 0, tot_c = 0;
    for (int w = 0; w < kWaves; ++w) {
      if (w < wv) {
        it += s_t[w];
        ic += s_c[w];
      }
      tot_t += s_t[w];
      tot_c += s_c[w];
    }
    // 3. Exclusive prefixes, staged in LDS and stored by consecutive lanes.
    int64_t r = carry_t + it - st;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
      s_buf[tid * kScanPer + i] = r;
      r += ct[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
      const int j = i * kScanThreads + tid;
      if (j < m) tile_start[base + uint32_t(j)] = s_buf[j];
    }
    __syncthreads();
    r = carry_c + ic - sc;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
      s_buf[tid * kScanPer + i] = r;
      r += cc[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
      const int j = i * kScanThreads + tid;
      if (j < m) cost_start[base + uint32_t(j)] = s_buf[j];
    }
    __syncthreads();  // s_buf, s_t and s_c are rewritten by the next round
    carry_t += tot_t;
    carry_c += tot_c;
  }
  if (tid == 0) {
    tile_start[nbatch] = carry_t;
    cost_start[nbatch] = carry_c;
  }
}

// The batch-table fields a wave needs for batch b.  Every lane loads the same
// addresses (one request each) and the values are moved to SGPRs.
struct BatchFields {
  int64_t cost0, tiles, off, woff;
  int32_t n, k;
};

__device__ __forceinline__ BatchFields load_batch(const WsArgs &a, int32_t b) {
  BatchFields f;
  f.cost0 = uniform(a.cost_start[b]);
  f.tiles = uniform(a.tile_start[b + 1] - a.tile_start[b]);
  f.off = uniform(a.boff[b]);
  f.woff = uniform(a.woff[b]);
  f.n = uniform(a.bn[b]);
  f.k = uniform(clamp_order(a.bk[b]));
  return f;
}

// Forms the wave's LDS tables for a batch of order k with weights w (see the
// weight sweeps in boys_device_f64_batched.hpp), one entry per lane; with
// D_l = (2l-1)!!:
//   ta[8 + s] = (2^(k-s) w_s D_s / D_k, 2^(s-k-1) D_k / D_s)  1 <= s <= k;
//               (2^k w_0 / D_k, 0) at s = 0;
//   tb[i]     = (2^-i w_i (2i-1)!!, -2^i / (2i+1)!!)  0 <= i < k;
//               (2^-k w_k (2k-1)!!, 0) at i = k;
//   tc[l]     = w_l a_l  l <= k  (region C);
// zeros elsewhere (the powers of two let the sweeps run in x and 1/x).  The
// weight loads use indices clamped into the batch's range, so they are
// unconditional and in flight together.
__device__ __forceinline__ void load_tables(const double *w, int k, int lane, wpair *ta, wpair *tb,
                                            double *tc) {
  // Every load is unconditional, from an index clamped into its table; the
  // entries outside their orders are zeroed by selects.
  const int s = lane - kSweepPadA;  // ta's order
  const int sc = s < 0 ? 0 : (s > k ? k : s);
  const int lc = lane > k ? k : lane;  // tb's l - 1 and tc's l
  const int lp = lane + 1 > k ? k : lane + 1;
  const double ws = w[sc], wl = w[lc];
  const double dfs = kDFact[sc], ids = kInvDFact[sc], dfl = kDFact[lc], idp = kInvDFact[lp];
  const double al = kAsymCoef[lc];
  const double dk = kDFact[k], idk = kInvDFact[k];
  const bool in_a = s >= 0 && s <= k, in_b = lane <= k;
  const wpair ea{__builtin_amdgcn_ldexp(in_a ? ws * (dfs * idk) : 0.0, k - s),
                 __builtin_amdgcn_ldexp(in_a && s >= 1 ? ids * dk : 0.0, s - k - 1)};
  const wpair eb{__builtin_amdgcn_ldexp(in_b ? wl * dfl : 0.0, -lane),
                 __builtin_amdgcn_ldexp(lane + 1 <= k ? -idp : 0.0, lane)};
  const double ec = in_b ? wl * al : 0.0;
  if (lane < kSweepLenA) ta[lane] = ea;
  if (lane < kSweepLenB) tb[lane] = eb;
  if (lane < kAsymTableLen) tc[lane] = ec;
}

// Largest b in [0, nbatch] with cost_start[b] <= lo, searched by one wave:
// each round probes 64 evenly spaced entries, so 8192 batches take 3 rounds
// of dependent loads instead of 13.
__device__ __forceinline__ int32_t wave_search(const int64_t *cost_start, int32_t nbatch,
                                               int64_t lo, int lane) {
  int32_t L = 0, H = nbatch;
  while (H > L) {
    const int64_t span = H - L;
    const int32_t pos = L + int32_t((span * (lane + 1) + 63) / 64);
    const uint64_t m = __ballot(cost_start[pos] <= lo);
    const int cnt = __popcll(m);  // the probes that pass form a prefix of the lanes
    const int32_t p_first = L + int32_t((span + 63) / 64);
    if (cnt == 0) {
      H = p_first - 1;
    } else {
      const int32_t p_last = L + int32_t((span * cnt + 63) / 64);
      const int32_t p_next = cnt < 64 ? L + int32_t((span * (cnt + 1) + 63) / 64) - 1 : H;
      L = p_last;
      H = p_next;
    }
  }
  return L;
}

// Mask of lanes 0..r-1 (r <= 0: none, r >= 64: all).
__device__ __forceinline__ uint64_t lane_prefix_mask(int r) {
  return r >= 64 ? ~uint64_t(0) : (r <= 0 ? uint64_t(0) : (uint64_t(1) << r) - 1);
}

// Orders LDS accesses of one wave (the hardware executes a wave's LDS
// instructions in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Waves per workgroup of the persistent kernel.  Every wave is an
// independent worker with its own LDS slice, so the workgroup only groups
// waves for dispatch: a workgroup's slot on a CU is freed when its last wave
// ends.
constexpr int kWsWaves = 4;
constexpr int kWsBlock = 64 * kWsWaves;

// Persistent kernel in which every wave is an independent worker: wave gw of
// W takes the tiles whose cost prefix lies in [gw, gw+1) * total / W.  A tile
// is 64*ITEMS arguments of one batch.  With BIN the wave sorts its tile by
// region (ballots and lane prefix counts, no atomics) into its LDS slice, so
// each 64-lane pass over the sorted tile runs a single region path except at
// the two region boundaries.  CH is the sweep chunk: the constant pairs of
// CH orders are read together, so a chunk waits for LDS once.  No workgroup
// barrier follows the set-up.
//
// With PF the wave loads the next tile's arguments of the same batch into
// registers right after taking the current tile's, so their latency hides
// behind the current tile's binning, passes and stores (8 more VGPR pairs
// at tile 512).
template <int ITEMS, bool BIN, int CH, class TS, bool PF = false>
__global__ __launch_bounds__(kWsBlock) void ws_kernel(WsArgs a) {
  static_assert((ITEMS & (ITEMS - 1)) == 0, "tiles are powers of two: the scan counts them by shifts");
  static_assert(CH <= kChunkMax, "the tables are padded for chunks up to kChunkMax");
  constexpr int T = 64 * ITEMS;
  __shared__ wpair s_ta[kWsWaves][kSweepLenA];  // region A's sweep constants
  __shared__ wpair s_tb[kWsWaves][kSweepLenB];  // region B's sweep constants
  __shared__ double s_x[kWsWaves][BIN ? T : 1];  // sorted arguments, then their results
  __shared__ __attribute__((aligned(16))) double s_tc[kWsWaves][kAsymTableLen];  // w_l a_l: region C

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const uint32_t lane8 = uint32_t(lane) * 8u;  // the lane's byte offset in a 64-double row
  // The wave index is the same in every lane; saying so keeps the per-wave
  // cost range, the batch fields and the order k in scalar registers, so
  // loops over k and the choice of r_A,k branch on scalar conditions.
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  wpair *const ta = s_ta[wv];
  wpair *const tb = s_tb[wv];
  double *const tc = s_tc[wv];

  const int64_t gw = int64_t(blockIdx.x) * kWsWaves + wv;
  const int64_t W = int64_t(gridDim.x) * kWsWaves;
  const int64_t total = uniform(a.cost_start[a.nbatch]);
  const int64_t lo = uniform(share_start(total, gw, W, a.taper));
  const int64_t hi = uniform(share_start(total, gw + 1, W, a.taper));
  int32_t b = uniform(wave_search(a.cost_start, a.nbatch, lo, lane));
  BatchFields f{};
  int64_t j = 0;
  if (b < a.nbatch) {
    f = load_batch(a, b);
    const int64_t cost = ITEMS * pass_cost(f.k);  // a full tile
    j = (lo - f.cost0 + cost - 1) / cost;
  }
  bool reload = true;
  double xn[ITEMS];        // PF: the next tile's arguments
  // r_B's leading numerator coefficient in a VGPR for the whole kernel
  // instead of two literal moves per region-B pass (fixed-region sets).
  double top_b = 0.0;
  if constexpr (!kPerKmaxRows<TS>) {
    top_b = rb_p_at<TS>(TS::rb_n);
    asm volatile("" : "+v"(top_b));
  }
  bool have_next = false;  // PF: xn holds the tile this iteration takes

  for (;;) {
    while (b < a.nbatch && j >= f.tiles) {  // past this batch: next non-empty one
      ++b;
      j = 0;
      reload = true;
      if (b < a.nbatch) f = load_batch(a, b);
    }
    if (b >= a.nbatch || f.cost0 + j * ITEMS * pass_cost(f.k) >= hi) break;
    const int64_t first = f.off + j * T;
    const int64_t rem = int64_t(f.n) - j * T;
    const int count = int(rem < T ? rem : T);
    const int k = f.k;
    // Region ends of this batch (the set's own, or row k's for the per-kmax
    // set): uniform, so they stay in scalar registers.
    const double x0v = batch_x0<TS>(k);
    const double x1v = batch_x1<TS>(k);
    ++j;
    if (reload) {
      wave_sync();  // the previous batch's passes have read the tables
      load_tables(a.w + f.woff, k, lane, ta, tb, tc);
      reload = false;
    }
    // Argument loads: one wave-uniform base (the tile's first argument) and
    // a 32-bit byte offset per lane, so the loads take the scalar-base form
    // with the item's 512-byte step as immediate offset.  In a partial tile
    // the offsets are clamped to the last argument, so every load stays in
    // the tile and all ITEMS loads are in flight together; lanes past the end
    // are never evaluated or stored.
    const char *const tx = reinterpret_cast<const char *>(a.x + first);
    double xv[ITEMS];
    if (PF && have_next) {
#pragma unroll
      for (int it = 0; it < ITEMS; ++it) xv[it] = xn[it];
    } else if (count == T) {
#pragma unroll
      for (int it = 0; it < ITEMS; ++it)
        xv[it] = *reinterpret_cast<const double *>(tx + (lane8 + uint32_t(it) * 512u));
    } else {
      const uint32_t last8 = uint32_t(count - 1) * 8u;
#pragma unroll
      for (int it = 0; it < ITEMS; ++it) {
        const uint32_t o = lane8 + uint32_t(it) * 512u;
        xv[it] = *reinterpret_cast<const double *>(tx + (o < last8 ? o : last8));
      }
    }
    if constexpr (PF) {
      // The next tile (j, after the increment above) when it is in this
      // batch and starts inside this wave's share: exactly the tile the next
      // iteration takes, since neither the batch advance nor the share test
      // then fires.  Offsets clamped as for a partial tile.
      have_next = j < f.tiles && f.cost0 + j * ITEMS * pass_cost(k) < hi;
      if (have_next) {
        const int64_t nrem = int64_t(f.n) - j * T;
        const uint32_t nlast8 = uint32_t((nrem < T ? nrem : T) - 1) * 8u;
        const char *const nx = reinterpret_cast<const char *>(a.x + f.off + j * T);
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
          const uint32_t o = lane8 + uint32_t(it) * 512u;
          xn[it] = *reinterpret_cast<const double *>(nx + (o < nlast8 ? o : nlast8));
        }
      }
    }
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) xv[it] = domain(xv[it]);
    if constexpr (BIN) {
      // Classes in the order A, C, B: the two 64-lane passes that straddle a
      // class boundary then pair the cheap asymptote path with one of the
      // rational paths instead of both rational paths.  Class c goes to
      // [start_c, start_c + count_c).  A first sweep counts classes A and C
      // (ballots of one compare each per item); B is the rest of the valid
      // lanes.  A second sweep gives each lane its slot: the running base of
      // its class plus its rank in the class among the item's lanes, where
      // the ranks in A and C are lane-prefix counts of their masks and the
      // rank in B is the lane index minus both (valid lanes form a prefix).
      // The slot is chosen by selects, not branches.  Each lane keeps the
      // slots of its items; results are written back into them, then stored
      // in the original order with coalesced stores.
      int nA = 0, nC = 0;
      int slot[ITEMS];
      auto bin = [&](auto full) {
        constexpr bool kFull = decltype(full)::value;
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
          const uint64_t valid = kFull ? ~uint64_t(0) : lane_prefix_mask(count - it * 64);
          nA += __popcll(__ballot(xv[it] < x0v) & valid);
          nC += __popcll(__ballot(xv[it] > x1v) & valid);
        }
        int bA = 0, bC = nA, bB = nA + nC;
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
          // The compares again, rather than 2*ITEMS masks held in scalar
          // registers across the sweeps.
          double xr = xv[it];
          asm volatile("" : "+v"(xr));
          const uint64_t valid = kFull ? ~uint64_t(0) : lane_prefix_mask(count - it * 64);
          const bool isA = xr < x0v;
          const bool isC = xr > x1v;  // C = (x1, inf); x1 > x0: never with isA
          const uint64_t mA = __ballot(isA) & valid;
          const uint64_t mC = __ballot(isC) & valid;
          const int rA = int(__builtin_amdgcn_mbcnt_hi(uint32_t(mA >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mA), 0u)));
          const int rC = int(__builtin_amdgcn_mbcnt_hi(uint32_t(mC >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mC), 0u)));
          int sl = isC ? bC + rC : bB + (lane - rA - rC);
          sl = isA ? bA + rA : sl;
          if constexpr (kFull) {
            s_x[wv][sl] = xv[it];
          } else {
            // Lanes past the tile's end take slot 0: their rank in B would
            // count them past the tile, and the slot is read again before the
            // store.
            const bool in = it * 64 + lane < count;
            sl = in ? sl : 0;
            if (in) s_x[wv][sl] = xv[it];
          }
          slot[it] = sl;
          const int cA = __popcll(mA), cC = __popcll(mC);
          const int cV = kFull ? 64 : __popcll(valid);
          bA += cA;
          bC += cC;
          bB += cV - cA - cC;
        }
      };
      if (count == T) bin(std::true_type{});
      else bin(std::false_type{});
      const int nAC = nA + nC;
      wave_sync();
      // The passes cover the items holding a valid slot.  In the last one of
      // a partial tile, lanes past the tile's end (slots from count on,
      // after every class) evaluate their stale slot on region B's path and
      // write it back, where no store reads it: those lanes were masked off
      // in the same wave instructions before, so they cost nothing, and each
      // pass saves the bounds compare and its exec-mask updates.  The paths
      // touch no memory that depends on the argument.
      const int passes = (count + 63) >> 6;
#pragma unroll 1
      for (int it = 0; it < passes; ++it) {
        const int q = it * 64 + lane;
        const double xq = s_x[wv][q];
        double acc;
        if (q < nA) acc = wsum_sweep_a<CH, TS>(xq, k, ta);
        else if (q < nAC) acc = wsum_region_c(xq, k, tc);
        else acc = wsum_sweep_b<CH, TS>(xq, k, tb, top_b);
        s_x[wv][q] = acc;
      }
      wave_sync();
      // Non-temporal stores: the output is not read again by the kernel.
      char *const to = reinterpret_cast<char *>(a.out + first);
      if (count == T) {
#pragma unroll
        for (int it = 0; it < ITEMS; ++it)
          __builtin_nontemporal_store(s_x[wv][slot[it]],
                                      reinterpret_cast<double *>(to + (lane8 + uint32_t(it) * 512u)));
      } else {
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
          const double v = s_x[wv][slot[it]];
          if (it * 64 + lane < count)
            __builtin_nontemporal_store(v, reinterpret_cast<double *>(to + (lane8 + uint32_t(it) * 512u)));
        }
      }
      wave_sync();
    } else {
      wave_sync();
#pragma unroll 1
      for (int it = 0; it < ITEMS; ++it) {
        const int p = it * 64 + lane;
        if (p < count) {
          const double xq = xv[it];
          double acc;
          if (xq < x0v) acc = wsum_sweep_a<CH, TS>(xq, k, ta);
          else if (xq > x1v) acc = wsum_region_c(xq, k, tc);
          else acc = wsum_sweep_b<CH, TS>(xq, k, tb, top_b);
          a.out[first + p] = acc;
        }
      }
      wave_sync();
    }
  }
}

// ---------------------------------------------------------------------------
// Configurations (the autotuner's search space).

using WsKernel = void (*)(WsArgs);

// The table sets of the batched consumer: the paper's, the screening set
// (eps_tol = 1e-10), the per-kmax regions and the centre-of-anti-diagonal
// refit (boys_set_tables).
enum WsSet { kWsPaper = 0, kWsScreen = 1, kWsPerKmax = 2, kWsCentre = 3, kWsSets = 4 };

// The set for a call at tolerance tol (>= 5e-14): the screening set from
// 1e-10 on, else the process-wide variant of the 5e-14 tables.
int ws_set_for(double tol) {
  if (tol >= ScreenTables::eps) return kWsScreen;
  switch (table_variant()) {
    case BOYS_TABLES_PER_KMAX: return kWsPerKmax;
    case BOYS_TABLES_CENTRE: return kWsCentre;
    default: return kWsPaper;
  }
}

struct WsConfig {
  WsKernel kernel[kWsSets];  // by WsSet
  int items;               // arguments per lane per tile (tile = 64 * items)
  int bin;                 // region binning in LDS
  int chunk;               // sweep chunk (orders whose constants are read together)
  int rounds;              // grid = rounds x the workgroups resident per CU x CUs
  int taper;               // per-wave shares decreasing with the wave index
  const char *name;
};

// Grids are counted in rounds of resident workgroups.
#define BOYS_WS_CONFIG_PF(ITEMS, BIN, CH, PF, R, TAPER, NAME)                                         \
  {{&ws_kernel<ITEMS, BIN, CH, PaperTables, PF>, &ws_kernel<ITEMS, BIN, CH, ScreenTables, PF>,         \
    &ws_kernel<ITEMS, BIN, CH, PerKmaxSet, PF>, &ws_kernel<ITEMS, BIN, CH, CentreTables, PF>}, \
   ITEMS, BIN, CH, R, TAPER, NAME}
#define BOYS_WS_CONFIG(ITEMS, BIN, CH, R, TAPER, NAME) BOYS_WS_CONFIG_PF(ITEMS, BIN, CH, false, R, TAPER, NAME)
const WsConfig kConfigs[] = {
    BOYS_WS_CONFIG(8, true, 4, 3, 2, "tile512-bin-ch4-3rounds-taper2"),
    BOYS_WS_CONFIG(8, true, 4, 3, 0, "tile512-bin-ch4-3rounds"),
    BOYS_WS_CONFIG(8, true, 4, 2, 2, "tile512-bin-ch4-2rounds-taper2"),
    BOYS_WS_CONFIG(8, true, 4, 2, 3, "tile512-bin-ch4-2rounds-taper3"),
    BOYS_WS_CONFIG(8, true, 4, 3, 3, "tile512-bin-ch4-3rounds-taper3"),
    BOYS_WS_CONFIG(8, true, 4, 4, 3, "tile512-bin-ch4-4rounds-taper3"),
    BOYS_WS_CONFIG(8, true, 8, 2, 2, "tile512-bin-ch8-2rounds-taper2"),
    BOYS_WS_CONFIG(8, true, 8, 3, 3, "tile512-bin-ch8-3rounds-taper3"),
    BOYS_WS_CONFIG(4, true, 4, 3, 2, "tile256-bin-ch4-3rounds-taper2"),
    BOYS_WS_CONFIG(4, false, 4, 2, 0, "tile256-nobin-ch4-2rounds"),
    BOYS_WS_CONFIG_PF(8, true, 4, true, 2, 3, "tile512-bin-ch4-pf-2rounds-taper3"),
    BOYS_WS_CONFIG_PF(8, true, 4, true, 3, 3, "tile512-bin-ch4-pf-3rounds-taper3"),
    BOYS_WS_CONFIG_PF(4, true, 4, true, 3, 3, "tile256-bin-ch4-pf-3rounds-taper3"),
};
#undef BOYS_WS_CONFIG
#undef BOYS_WS_CONFIG_PF
constexpr int kNumConfigs = int(sizeof(kConfigs) / sizeof(kConfigs[0]));
constexpr int kDefaultConfig = 0;  // tile512-bin-ch4-3rounds-taper2

// ---------------------------------------------------------------------------
// Per-device state: workspace, one cached graph per configuration (so the
// tuner can alternate between them without rebuilding), chosen configuration.

struct GraphKey {
  const void *ptrs[7];
  int32_t nbatch;
  int config;
  int set;  // WsSet
  const void *ws;
  bool operator==(const GraphKey &o) const { return std::memcmp(this, &o, sizeof(*this)) == 0; }
};

struct GraphSlot {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  GraphKey key;
  bool has_key = false;
};

// A graph replaced by a newer one.  Its launches may still be queued, so it is
// destroyed once an event recorded behind them (on the stream of the call
// that replaced it: calls on one device are ordered by the caller) has
// completed, checked without waiting at later calls.
struct RetiredGraph {
  hipGraph_t graph;
  hipGraphExec_t exec;
  hipEvent_t done;
};

struct DeviceState {
  std::mutex mu;
  void *ws = nullptr;  // see Workspace
  int64_t ws_cap = 0;
  // Workspaces replaced by larger ones.  Graphs already enqueued may still
  // read them, so they are freed only by boys_finalize (which synchronises
  // the device); capacities double, so together they stay below the current
  // one.
  std::vector<void *> retired;
  std::vector<RetiredGraph> retired_graphs;
  GraphSlot slot[kWsSets][kNumConfigs];  // [table set][configuration]
  int config = -1;  // -1: not chosen yet (one choice serves both sets)
  int cus = 0;
  char arch[32] = {};  // the device's architecture name (up to the first ':')
  int resident[kWsSets][kNumConfigs] = {};  // workgroups per CU, 0: not queried yet
  void *scratch_ptr = nullptr;         // this device's copy of `scratch`
  bool has_graphs() const {
    for (const auto &row : slot)
      for (const GraphSlot &g : row)
        if (g.exec || g.graph) return true;
    return !retired_graphs.empty();
  }
};

constexpr int kMaxDevices = 64;
DeviceState g_dev[kMaxDevices];

// Destroys a slot's graph at once: for graphs never launched, or after a
// device synchronisation.
void drop_slot(GraphSlot &g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g.exec = nullptr;
  g.graph = nullptr;
  g.has_key = false;
}

// Moves a slot's graph to the retired list behind an event recorded on
// `stream`; if the event cannot be made, waits for the stream instead.
int retire_slot(DeviceState &s, GraphSlot &g, hipStream_t stream) {
  if (!g.exec && !g.graph) return BOYS_OK;
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(ev, stream) != hipSuccess) {
    if (ev) (void)hipEventDestroy(ev);
    BOYS_TRY_HIP(hipStreamSynchronize(stream));
    drop_slot(g);
    return BOYS_OK;
  }
  s.retired_graphs.push_back(RetiredGraph{g.graph, g.exec, ev});
  g.exec = nullptr;
  g.graph = nullptr;
  g.has_key = false;
  return BOYS_OK;
}

int retire_graphs(DeviceState &s, hipStream_t stream) {
  for (auto &row : s.slot)
    for (GraphSlot &g : row)
      if (int st = retire_slot(s, g, stream)) return st;
  return BOYS_OK;
}

// Destroys the retired graphs whose event has completed (never waits).
void reap_graphs(DeviceState &s) {
  size_t keep = 0;
  for (RetiredGraph &r : s.retired_graphs) {
    if (hipEventQuery(r.done) == hipSuccess) {
      (void)hipGraphExecDestroy(r.exec);
      (void)hipGraphDestroy(r.graph);
      (void)hipEventDestroy(r.done);
    } else {
      s.retired_graphs[keep++] = r;
    }
  }
  s.retired_graphs.resize(keep);
  (void)hipGetLastError();  // a query of a pending event reports hipErrorNotReady
}

// After a device synchronisation: destroys every graph.
void drop_graphs(DeviceState &s) {
  for (auto &row : s.slot)
    for (GraphSlot &g : row) drop_slot(g);
  for (RetiredGraph &r : s.retired_graphs) {
    (void)hipGraphExecDestroy(r.exec);
    (void)hipGraphDestroy(r.graph);
    (void)hipEventDestroy(r.done);
  }
  s.retired_graphs.clear();
}

// The tuning cache: the file named by BOYS_TUNE_CACHE holds lines
//     weighted_sum <arch> <table set> <bucket> <configuration name>
// (bucket = floor(log2 nbatch)).  A lookup takes the last line whose device
// architecture, table set and bucket match this call and whose name is one of
// this build's configurations; anything else (no variable, no file, other
// devices or builds, malformed lines) leaves the default.  Names rather than
// indices keep entries valid when the configuration table changes.
int nbatch_bucket(int32_t nbatch) { return nbatch > 0 ? int(std::log2(double(nbatch))) : 0; }

int config_by_name(const char *name) {
  for (int c = 0; c < kNumConfigs; ++c)
    if (std::strcmp(kConfigs[c].name, name) == 0) return c;
  return -1;
}

int cached_config(const char *arch, int32_t nbatch, int set) {
  const char *path = std::getenv("BOYS_TUNE_CACHE");
  int best = kDefaultConfig;
  if (!path || !arch[0]) return best;
  FILE *f = std::fopen(path, "r");
  if (!f) return best;
  const int bucket = nbatch_bucket(nbatch);
  char line[256];
  while (std::fgets(line, sizeof(line), f)) {
    char tag[32], a[32], name[96];
    int st = -1, bk = -1;
    char extra;
    if (std::sscanf(line, "%31s %31s %d %d %95s %c", tag, a, &st, &bk, name, &extra) != 5) continue;
    if (std::strcmp(tag, "weighted_sum") != 0 || std::strcmp(a, arch) != 0 || st != set || bk != bucket)
      continue;
    const int c = config_by_name(name);
    if (c >= 0) best = c;
  }
  std::fclose(f);
  return best;
}

void store_config(const char *arch, int32_t nbatch, int set, int cfg) {
  const char *path = std::getenv("BOYS_TUNE_CACHE");
  if (!path || !arch[0]) return;
  if (FILE *f = std::fopen(path, "a")) {
    std::fprintf(f, "weighted_sum %s %d %d %s\n", arch, set, nbatch_bucket(nbatch), kConfigs[cfg].name);
    std::fclose(f);
  }
}

// The workspace of one call: the scan's prefix arrays of tiles and cost,
// [cap] each (cap >= nbatch + 1), carved from one allocation or from
// `scratch`.
struct Workspace {
  int64_t *tile_start;
  int64_t *cost_start;
};

constexpr size_t workspace_bytes(int64_t cap) { return size_t(cap) * 2 * sizeof(int64_t); }

Workspace carve(void *base, int64_t cap) {
  int64_t *p = static_cast<int64_t *>(base);
  return Workspace{p, p + cap};
}

struct Call {
  const double *x;
  const int64_t *boff;
  const int32_t *bn;
  const int32_t *bk;
  const double *w;
  const int64_t *woff;
  int32_t nbatch;
  double *out;
};

// Makes sure the workspace holds nbatch + 1 entries.
int ensure_workspace(DeviceState &s, int32_t nbatch, hipStream_t stream) {
  const int64_t need = int64_t(nbatch) + 1;
  if (s.ws_cap >= need) return BOYS_OK;
  if (s.ws) {
    // An earlier graph may still be reading the old workspace: retire it
    // rather than wait for the device.
    s.retired.push_back(s.ws);
    s.ws = nullptr;
    s.ws_cap = 0;
  }
  if (int st = retire_graphs(s, stream)) return st;
  int64_t cap = 1024;
  while (cap < need) cap *= 2;
  if (hipMalloc(&s.ws, workspace_bytes(cap)) != hipSuccess) {
    (void)hipGetLastError();
    s.ws = nullptr;
    return BOYS_ENOMEM;
  }
  s.ws_cap = cap;
  return BOYS_OK;
}

// Grid of the persistent kernel: `rounds` rounds of the workgroups that fit
// on every CU at once.
int main_grid(DeviceState &s, int cfg, int set, unsigned *grid) {
  const WsConfig &conf = kConfigs[cfg];
  int &resident = s.resident[set][cfg];
  if (resident == 0) {
    const WsKernel kern = conf.kernel[set];
    int r = 0;
    BOYS_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, reinterpret_cast<const void *>(kern),
                                                              kWsBlock, 0));
    resident = r < 1 ? 1 : r;
  }
  *grid = unsigned(s.cus * resident * conf.rounds);
  return BOYS_OK;
}

// Builds (or reuses) the graph {scan -> persistent kernel} for this call.
int prepare_graph(DeviceState &s, const Call &c, int cfg, int set, hipStream_t stream) {
  GraphKey key;
  std::memset(&key, 0, sizeof(key));
  const void *p[7] = {c.x, c.boff, c.bn, c.bk, c.w, c.woff, c.out};
  std::memcpy(key.ptrs, p, sizeof(p));
  key.nbatch = c.nbatch;
  key.config = cfg;
  key.set = set;
  key.ws = s.ws;
  GraphSlot &g = s.slot[set][cfg];
  if (g.has_key && g.exec && key == g.key) return BOYS_OK;
  if (int st = retire_slot(s, g, stream)) return st;

  const WsConfig &conf = kConfigs[cfg];
  const Workspace ws = carve(s.ws, s.ws_cap);
  int64_t *tile_start = ws.tile_start;
  int64_t *cost_start = ws.cost_start;
  int tile_shift = __builtin_ctz(unsigned(64 * conf.items));  // items is a power of two

  BOYS_TRY_HIP(hipGraphCreate(&g.graph, 0));
  hipGraphNode_t scan_node, main_node;

  const int32_t *bn = c.bn, *bk = c.bk;
  int32_t nbatch = c.nbatch;
  void *scan_args[] = {&bn, &bk, &nbatch, &tile_shift, &tile_start, &cost_start};
  hipKernelNodeParams sp = {};
  sp.func = reinterpret_cast<void *>(&ws_scan_kernel);
  sp.gridDim = dim3(1);
  sp.blockDim = dim3(kScanThreads);
  sp.sharedMemBytes = 0;
  sp.kernelParams = scan_args;
  sp.extra = nullptr;
  BOYS_TRY_HIP(hipGraphAddKernelNode(&scan_node, g.graph, nullptr, 0, &sp));

  WsArgs args{c.x, c.boff, c.bn, c.bk, c.w, c.woff, c.out, tile_start, cost_start, c.nbatch, conf.taper};
  void *main_args[] = {&args};
  hipKernelNodeParams mp = {};
  const WsKernel kern = conf.kernel[set];
  unsigned grid = 0;
  if (int st = main_grid(s, cfg, set, &grid)) return st;
  mp.gridDim = dim3(grid);
  mp.func = reinterpret_cast<void *>(kern);
  mp.blockDim = dim3(kWsBlock);
  mp.sharedMemBytes = 0;
  mp.kernelParams = main_args;
  mp.extra = nullptr;
  BOYS_TRY_HIP(hipGraphAddKernelNode(&main_node, g.graph, &scan_node, 1, &mp));

  BOYS_TRY_HIP(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
  g.key = key;
  g.has_key = true;
  return BOYS_OK;
}

int validate(const Call &c) {
  if (c.nbatch < 0 || c.nbatch > kMaxBatches) return BOYS_EINVAL;
  if (c.nbatch == 0) return BOYS_OK;
  if (!c.x || !c.boff || !c.bn || !c.bk || !c.w || !c.woff || !c.out) return BOYS_EINVAL;
  return BOYS_OK;
}

int device_state(DeviceState **out) {
  int dev = 0;
  BOYS_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return BOYS_ENOTSUP;
  DeviceState &s = g_dev[dev];
  if (s.cus == 0) {
    int cus = 0;
    BOYS_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    hipDeviceProp_t prop;
    BOYS_TRY_HIP(hipGetDeviceProperties(&prop, dev));
    size_t i = 0;
    for (; i + 1 < sizeof(s.arch) && prop.gcnArchName[i] && prop.gcnArchName[i] != ':'; ++i)
      s.arch[i] = prop.gcnArchName[i];
    s.arch[i] = 0;
    s.cus = cus > 0 ? cus : 1;
  }
  *out = &s;
  return BOYS_OK;
}

// Enqueues one evaluation with configuration cfg and table set `set` (state
// lock held).
int launch(DeviceState &s, const Call &c, int cfg, int set, hipStream_t stream) {
  if (!s.retired_graphs.empty()) reap_graphs(s);
  if (int st = ensure_workspace(s, c.nbatch, stream)) return st;
  if (int st = prepare_graph(s, c, cfg, set, stream)) {
    drop_slot(s.slot[set][cfg]);  // built here, never launched
    return st;
  }
  BOYS_TRY_HIP(hipGraphLaunch(s.slot[set][cfg].exec, stream));
  return BOYS_OK;
}

int weighted_sum_with_set(const Call &c, int set, hipStream_t stream) {
  if (int st = validate(c)) return st;
  if (c.nbatch == 0) return BOYS_OK;
  if (int st = check_device()) return st;
  if (int st = check_not_capturing(stream)) return st;
  DeviceState *s = nullptr;
  if (int st = device_state(&s)) return st;
  std::lock_guard<std::mutex> lock(s->mu);
  if (s->config < 0) s->config = cached_config(s->arch, c.nbatch, set);
  return launch(*s, c, s->config, set, stream);
}

// ---------------------------------------------------------------------------
// Allocation-free variant (boys_weighted_sum_noalloc): the scan's two prefix
// arrays live in a fixed device array instead of the grown workspace, and the
// two kernels are launched directly on the caller's stream instead of through
// a cached graph, so the call allocates nothing and can be captured.  Every
// call's scan rewrites all prefix entries the main kernel then reads, so
// nothing has to be cleared between calls; calls that overlap on one device
// share the array and race.
constexpr int32_t kNoAllocMaxBatches = BOYS_NOALLOC_MAX_BATCHES;
constexpr int64_t kNoAllocCap = int64_t(kNoAllocMaxBatches) + 1;
static_assert(workspace_bytes(kNoAllocCap) % sizeof(int64_t) == 0, "whole int64 entries");
__device__ __align__(256) int64_t scratch[workspace_bytes(kNoAllocCap) / sizeof(int64_t)];

// This device's address of `scratch` (looked up once per device, with the
// device current; the array's name is only a host-side stand-in).
int scratch_address(DeviceState &s, void **out) {
  if (!s.scratch_ptr) {
    void *p = nullptr;
    BOYS_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    s.scratch_ptr = p;
  }
  *out = s.scratch_ptr;
  return BOYS_OK;
}

int launch_direct(DeviceState &s, const Call &c, int cfg, int set, const Workspace &ws,
                  hipStream_t stream) {
  const WsConfig &conf = kConfigs[cfg];
  const int tile_shift = __builtin_ctz(unsigned(64 * conf.items));
  unsigned grid = 0;
  if (int st = main_grid(s, cfg, set, &grid)) return st;
  hipLaunchKernelGGL(ws_scan_kernel, dim3(1), dim3(kScanThreads), 0, stream, c.bn, c.bk, c.nbatch,
                     tile_shift, ws.tile_start, ws.cost_start);
  BOYS_TRY_HIP(hipGetLastError());
  const WsArgs args{c.x, c.boff, c.bn, c.bk, c.w, c.woff, c.out, ws.tile_start, ws.cost_start, c.nbatch,
                    conf.taper};
  hipLaunchKernelGGL(conf.kernel[set], dim3(grid), dim3(kWsBlock), 0, stream, args);
  BOYS_TRY_HIP(hipGetLastError());
  return BOYS_OK;
}

}  // namespace
}  // namespace boys

extern "C" {

int boys_weighted_sum_noalloc(const double *x, const int64_t *batch_off, const int32_t *batch_n,
                              const int32_t *batch_kmax, const double *w, const int64_t *w_off,
                              int32_t nbatch, double *out, hipStream_t stream) {
  using namespace boys;
  const Call c{x, batch_off, batch_n, batch_kmax, w, w_off, nbatch, out};
  if (nbatch > kNoAllocMaxBatches) return BOYS_EINVAL;
  if (int st = validate(c)) return st;
  if (nbatch == 0) return BOYS_OK;
  if (int st = check_device()) return st;
  DeviceState *s = nullptr;
  if (int st = device_state(&s)) return st;
  std::lock_guard<std::mutex> lock(s->mu);
  void *base = nullptr;
  if (int st = scratch_address(*s, &base)) return st;
  const int cfg = s->config < 0 ? kDefaultConfig : s->config;
  return launch_direct(*s, c, cfg, ws_set_for(PaperTables::eps), carve(base, kNoAllocCap), stream);
}

int boys_weighted_sum(const double *x, const int64_t *batch_off, const int32_t *batch_n,
                      const int32_t *batch_kmax, const double *w, const int64_t *w_off,
                      int32_t nbatch, double *out, hipStream_t stream) {
  using namespace boys;
  return weighted_sum_with_set(Call{x, batch_off, batch_n, batch_kmax, w, w_off, nbatch, out},
                               ws_set_for(PaperTables::eps), stream);
}

int boys_weighted_sum_tol(const double *x, const int64_t *batch_off, const int32_t *batch_n,
                          const int32_t *batch_kmax, const double *w, const int64_t *w_off,
                          int32_t nbatch, double tol, double *out, hipStream_t stream) {
  using namespace boys;
  const int set = table_set_for(kF64Kmax, tol);
  if (set < 0) return BOYS_EINVAL;
  return weighted_sum_with_set(Call{x, batch_off, batch_n, batch_kmax, w, w_off, nbatch, out},
                               ws_set_for(tol), stream);
}

int boys_tune_weighted_sum(const double *x, const int64_t *batch_off, const int32_t *batch_n,
                           const int32_t *batch_kmax, const double *w, const int64_t *w_off,
                           int32_t nbatch, double *out, hipStream_t stream, int *best_config,
                           float *best_ms) {
  using namespace boys;
  const Call c{x, batch_off, batch_n, batch_kmax, w, w_off, nbatch, out};
  if (int st = validate(c)) return st;
  if (nbatch == 0) return BOYS_OK;
  if (int st = check_device()) return st;
  if (int st = check_not_capturing(stream)) return st;
  DeviceState *s = nullptr;
  if (int st = device_state(&s)) return st;
  std::lock_guard<std::mutex> lock(s->mu);

  hipEvent_t e0, e1;
  BOYS_TRY_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_status(hipGetLastError());
  }
  // Rounds over all configurations, keeping each one's best time: timing
  // them one after another would favour the first ones, measured while the
  // clocks are still at their boost level.
  constexpr int kRounds = 3;
  const int set = ws_set_for(PaperTables::eps);  // the variant of the paper's accuracy in use
  float tmin[kNumConfigs] = {};
  int st = BOYS_OK;
  for (int cfg = 0; cfg < kNumConfigs && st == BOYS_OK; ++cfg)
    st = launch(*s, c, cfg, set, stream);  // warm-up (and graph build)
  for (int r = 0; r < kRounds && st == BOYS_OK; ++r) {
    for (int cfg = 0; cfg < kNumConfigs && st == BOYS_OK; ++cfg) {
      float t = 0.0f;
      if ((st = hip_status(hipEventRecord(e0, stream)))) break;
      if ((st = launch(*s, c, cfg, set, stream))) break;
      if ((st = hip_status(hipEventRecord(e1, stream)))) break;
      if ((st = hip_status(hipEventSynchronize(e1)))) break;
      if ((st = hip_status(hipEventElapsedTime(&t, e0, e1)))) break;
      if (r == 0 || t < tmin[cfg]) tmin[cfg] = t;
    }
  }
  int best = 0;
  for (int cfg = 1; cfg < kNumConfigs; ++cfg)
    if (tmin[cfg] < tmin[best]) best = cfg;
  const float best_t = tmin[best];
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != BOYS_OK) return st;
  s->config = best;
  store_config(s->arch, nbatch, set, best);
  if ((st = launch(*s, c, best, set, stream))) return st;  // leaves the graph of the winner cached
  if (best_config) *best_config = best;
  if (best_ms) *best_ms = best_t;
  return BOYS_OK;
}

int boys_weighted_sum_num_configs(void) { return boys::kNumConfigs; }

const char *boys_weighted_sum_config_name(int config) {
  if (config < 0 || config >= boys::kNumConfigs) return "invalid";
  return boys::kConfigs[config].name;
}

int boys_weighted_sum_get_config(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= boys::kMaxDevices) return -1;
  std::lock_guard<std::mutex> lock(boys::g_dev[dev].mu);
  const int c = boys::g_dev[dev].config;
  return c < 0 ? boys::kDefaultConfig : c;
}

int boys_weighted_sum_set_config(int config) {
  if (config < -1 || config >= boys::kNumConfigs) return BOYS_EINVAL;
  int dev = 0;
  BOYS_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= boys::kMaxDevices) return BOYS_ENOTSUP;
  std::lock_guard<std::mutex> lock(boys::g_dev[dev].mu);
  boys::g_dev[dev].config = config;
  return BOYS_OK;
}

void boys_finalize(void) {
  using namespace boys;
  int cur = 0;
  const bool have_cur = hipGetDevice(&cur) == hipSuccess;
  for (int d = 0; d < kMaxDevices; ++d) {
    DeviceState &s = g_dev[d];
    std::lock_guard<std::mutex> lock(s.mu);
    if (!s.ws && !s.has_graphs() && s.retired.empty()) continue;
    if (hipSetDevice(d) != hipSuccess) continue;
    (void)hipDeviceSynchronize();
    drop_graphs(s);
    if (s.ws) (void)hipFree(s.ws);
    for (void *old : s.retired) (void)hipFree(old);
    s.retired.clear();
    s.ws = nullptr;
    s.ws_cap = 0;
  }
  if (have_cur) (void)hipSetDevice(cur);
  pairsum_release_all();
}

}  // extern "C"
