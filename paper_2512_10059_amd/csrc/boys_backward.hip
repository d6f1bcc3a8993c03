// boys_backward: gradient of F_0..F_kmax with respect to x on gfx950.
//
// dF_k/dx = -F_{k+1} (differentiate the defining integral under the integral
// sign), so for upstream gradients G
//
//     grad_x[i] = - sum_{k=0..kmax} G[i, k] F_{k+1}(x[i]).
//
// The kernel recomputes F_0..F_{kmax+1} in VGPRs with the FP64 method at
// order kmax+1 (the paper's tables up to order 32, the high-order set for
// 33..40) instead of reading values saved by the forward pass: x is 8 bytes
// per argument while the saved rows would be 8*(kmax+1).  G rows are the
// dominant traffic (8*(kmax+1) bytes per argument); each wave reads its 64
// rows as one contiguous stream into an LDS slice whose row stride is an odd
// number of doubles, so that the per-lane row reads that follow are free of
// bank conflicts.  Packed rows come with 16-byte loads, issued before the
// evaluation so that their latency hides behind it, or for long odd rows by
// LDS-DMA loads that land in LDS during the evaluation.
#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <type_traits>
#include <utility>

#include "boys.h"
#include "boys_common.hpp"
#include "boys_device_f64.hpp"

namespace boys {
namespace {

typedef double d2 __attribute__((ext_vector_type(2)));

// Waves per workgroup: orders whose recomputation needs the high-order table
// set (kmax+1 > 32) stage rows of 34..40 doubles, so their groups have two
// waves (about 42 KB of LDS) instead of four (84 KB, one group per CU).
constexpr int backward_waves(int K) { return K + 1 > kF64Kmax ? 2 : kWavesPerBlock; }

template <int K, class T>
__global__ __launch_bounds__(64 * backward_waves(K)) void backward_kernel(
    const double *__restrict__ x, const double *__restrict__ g, int64_t n, int64_t ld,
    double *__restrict__ grad, int packed) {
  constexpr int C = K + 1;                  // columns of G used
  constexpr int WB = backward_waves(K);
  constexpr int CP = (C % 2 == 0) ? C + 1 : C;  // padded LDS row stride
  // Packed rows go to LDS by LDS-DMA loads for odd row lengths from 19 on.
  // There the rows held in VGPRs across the evaluation would cap the waves
  // per SIMD at two or three; the DMA path runs kmax 18..30 7-17% faster,
  // while at kmax <= 16 the register path, whose loads overlap the
  // evaluation entirely, is 3-5% faster.
  constexpr bool kDma = C % 2 == 1 && C >= 19;
  // Per-wave slice: 64 rows, plus (DMA) the slack that the last LDS-DMA
  // instruction's surplus lanes write: 128 J doubles are written in all.
  constexpr int SL = kDma ? 128 * ((32 * C + 63) / 64) : 64 * CP;
  __shared__ __attribute__((aligned(16))) double stage[WB * SL];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  double *slice = stage + wave * SL;

  for (int64_t blk = blockIdx.x; blk * (64 * WB) < n; blk += gridDim.x) {
    const int64_t row0 = blk * (64 * WB) + int64_t(wave) * 64;
    const int64_t i = row0 + lane;
    const int rows = n - row0 < 64 ? int(n - row0 > 0 ? n - row0 : 0) : 64;
    double F[C + 1];
    if constexpr (kDma) {
      if (rows == 64 && packed) {
        // Full wave, packed 16-byte-aligned rows of odd length: the LDS slice
        // (stride C) is an exact copy of the wave's 64*C consecutive doubles,
        // so the rows go straight from memory to LDS (16-byte LDS-DMA loads,
        // 1 KiB per instruction) while the wave evaluates, holding no VGPRs.
        // x is awaited before the DMA loads are issued: the compiler's wait
        // for x would otherwise also wait for every DMA load in flight.
        constexpr int U = 32 * C;
        constexpr int J = (U + 63) / 64;
        const double xv = x[i];
        asm volatile("" : : "v"(xv));  // x has arrived
        __builtin_amdgcn_sched_barrier(0);
        const d2 *src = reinterpret_cast<const d2 *>(g + row0 * C);
#pragma unroll
        for (int jj = 0; jj < J; ++jj) {
          // Every lane takes part (no branch, so the load counter stays
          // exact).  In the last instruction the lanes past the wave's rows
          // re-read its last unit and land in the slice's slack.
          const int u = lane + 64 * jj;
          __builtin_amdgcn_global_load_lds(
              (const __attribute__((address_space(1))) void *)(src + (u < U ? u : U - 1)),
              (__attribute__((address_space(3))) void *)(slice + 128 * jj), 16, 0, 0);
        }
        boys_f64<K + 1, T>(xv, F);
        __builtin_amdgcn_s_waitcnt(0);  // the LDS-DMA loads have landed
      } else {
        // Strided rows or a partial wave: evaluate first, then copy the rows
        // to LDS element by element (64 consecutive elements per load when
        // the rows are packed), so that the register budget stays that of
        // the DMA path.
        boys_f64<K + 1, T>(i < n ? x[i] : 0.0, F);
#pragma unroll 4
        for (int e = lane; e < rows * C; e += 64) {
          const int r = e / C, c = e - r * C;
          slice[r * CP + c] = g[(row0 + r) * ld + c];
        }
      }
    } else if constexpr (C > kF64Kmax) {
      // Even row lengths of the high orders: rows held across the evaluation
      // would take over 300 VGPRs, so evaluate first, then read the rows
      // (16-byte loads when packed, else element by element).
      boys_f64<K + 1, T>(i < n ? x[i] : 0.0, F);
      if (rows == 64 && packed) {
        constexpr int U = 32 * C;
        constexpr int J = (U + 63) / 64;
        const d2 *src = reinterpret_cast<const d2 *>(g + row0 * C);
#pragma unroll
        for (int jj = 0; jj < J; ++jj) {
          const int u = lane + 64 * jj;
          if (u < U) {
            const d2 v = __builtin_nontemporal_load(src + u);
            const int e = 2 * u, r = e / C, c = e - r * C;  // C even: no straddle
            slice[r * CP + c] = v.x;
            slice[r * CP + c + 1] = v.y;
          }
        }
      } else {
#pragma unroll 4
        for (int e = lane; e < rows * C; e += 64) {
          const int r = e / C, c = e - r * C;
          slice[r * CP + c] = g[(row0 + r) * ld + c];
        }
      }
    } else if (rows == 64 && packed) {
      // Full wave, packed 16-byte-aligned rows: the wave's 64 rows are 32*C
      // consecutive 16-byte units, read with 16-byte loads (1 KiB per
      // instruction) into VGPRs, all issued before the evaluation so that
      // their latency hides behind it, then written to the slice.  A unit
      // may straddle two rows when C is odd; its halves go to their own rows.
      constexpr int U = 32 * C;
      constexpr int J = (U + 63) / 64;
      const d2 *src = reinterpret_cast<const d2 *>(g + row0 * C);
      d2 gv[J];
#pragma unroll
      for (int jj = 0; jj < J; ++jj) {
        const int u = lane + 64 * jj;
        gv[jj] = __builtin_nontemporal_load(src + (u < U ? u : U - 1));
      }
      boys_f64<K + 1, T>(x[i], F);
#pragma unroll
      for (int jj = 0; jj < J; ++jj) {
        const int u = lane + 64 * jj;
        if (u < U) {
          const int e = 2 * u, r = e / C, c = e - r * C;
          slice[r * CP + c] = gv[jj].x;
          const int r1 = (e + 1) / C, c1 = e + 1 - r1 * C;
          slice[r1 * CP + c1] = gv[jj].y;
        }
      }
    } else if (rows == 64) {
      // Full wave, strided rows: all C loads of this wave's 64 rows of G (64
      // consecutive elements per instruction when the rows are packed) issued
      // before the evaluation, so their latency hides behind it.
      double gv[C];
#pragma unroll
      for (int jj = 0; jj < C; ++jj) {
        const int e = lane + 64 * jj, r = e / C, c = e - r * C;
        gv[jj] = __builtin_nontemporal_load(g + (row0 + r) * ld + c);
      }
      boys_f64<K + 1, T>(x[i], F);
#pragma unroll
      for (int jj = 0; jj < C; ++jj) {
        const int e = lane + 64 * jj, r = e / C, c = e - r * C;
        slice[r * CP + c] = gv[jj];
      }
    } else {
      for (int e = lane; e < rows * C; e += 64) {
        const int r = e / C, c = e - r * C;
        slice[r * CP + c] = g[(row0 + r) * ld + c];
      }
      boys_f64<K + 1, T>(i < n ? x[i] : 0.0, F);
    }
    __syncthreads();
    if (i < n) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < C; ++k) acc = __builtin_fma(slice[lane * CP + k], F[k + 1], acc);
      grad[i] = -acc;
    }
    __syncthreads();
  }
}

using BackwardKernel = void (*)(const double *, const double *, int64_t, int64_t, double *, int);

// kmax 0..31 recompute orders up to 32 with the paper's tables; kmax 32..39
// recompute orders 33..40 with the high-order set.
constexpr int kBackwardKmax = kHighKmax - 1;
template <int K>
using BackwardSet = std::conditional_t<(K + 1 > kF64Kmax), HighTables, PaperTables>;
template <std::size_t... K>
constexpr auto make_table(std::index_sequence<K...>) {
  return std::array<BackwardKernel, sizeof...(K)>{
      {&backward_kernel<int(K), BackwardSet<int(K)>>...}};
}
constexpr auto kBackwardTable = make_table(std::make_index_sequence<kBackwardKmax + 1>{});
// The screening set recomputes orders up to 32 (kmax up to 31).
template <std::size_t... K>
constexpr auto make_screen_table(std::index_sequence<K...>) {
  return std::array<BackwardKernel, sizeof...(K)>{{&backward_kernel<int(K), ScreenTables>...}};
}
constexpr auto kBackwardTableScreen = make_screen_table(std::make_index_sequence<kF64Kmax>{});

}  // namespace
}  // namespace boys

extern "C" int boys_backward(const double *x, const double *grad_f, int64_t n, int kmax,
                             int64_t ld_g, double *grad_x, hipStream_t stream) {
  return boys_backward_tol(x, grad_f, n, kmax, ld_g, boys::PaperTables::eps, grad_x, stream);
}

extern "C" int boys_backward_tol(const double *x, const double *grad_f, int64_t n, int kmax,
                                 int64_t ld_g, double tol, double *grad_x, hipStream_t stream) {
  using namespace boys;
  if (n < 0 || kmax < 0 || kmax > kBackwardKmax || ld_g < kmax + 1) return BOYS_EINVAL;
  // The set of the recomputation order kmax+1 (orders above 32: the
  // high-order set for any valid tol).
  const int set = table_set_for(kmax + 1, tol);
  if (set < 0) return BOYS_EINVAL;
  if (n == 0) return BOYS_OK;
  if (!x || !grad_f || !grad_x) return BOYS_EINVAL;
  if (n - 1 > (INT64_MAX / 8 - (kmax + 1)) / ld_g) return BOYS_EINVAL;
  const int64_t g_bytes = ((n - 1) * ld_g + kmax + 1) * 8;
  if (overlaps(grad_x, n * 8, x, n * 8) || overlaps(grad_x, n * 8, grad_f, g_bytes))
    return BOYS_EINVAL;
  if (int st = check_device()) return st;

  const int block = 64 * backward_waves(kmax);
  int64_t blocks = (n + block - 1) / block;
  if (blocks > kMaxBlocks) blocks = kMaxBlocks;
  const int packed = ld_g == kmax + 1 && (reinterpret_cast<uintptr_t>(grad_f) & 15) == 0;
  const BackwardKernel kernel = set == kSetScreen ? kBackwardTableScreen[kmax] : kBackwardTable[kmax];
  hipLaunchKernelGGL(kernel, dim3(unsigned(blocks)), dim3(block), 0, stream, x, grad_f, n, ld_g,
                     grad_x, packed);
  return hip_status(hipGetLastError());
}
