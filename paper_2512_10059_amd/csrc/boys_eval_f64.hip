// boys_eval_f64: FP64 write-out of F_0..F_kmax (Algorithm 1, Sec. II F of
// arXiv 2512.10059) on gfx950.
//
// One lane evaluates one argument with everything in VGPRs (boys_f64).  The
// output row of an argument is kmax+1 contiguous doubles, so a wave's 64 rows
// form one contiguous block of 64*(kmax+1) doubles; direct stores from the
// lanes would hit 64 different cache lines per instruction.  Each wave
// therefore stages its rows in its own LDS slice and writes the block back
// with 16-byte stores that cover 1 KiB of consecutive addresses per
// instruction.  The LDS row stride is the odd number kmax+1 or kmax+2, which
// maps 16 consecutive lanes onto 32 distinct banks (conflict-free 64-bit
// writes).  The stores are non-temporal: nothing re-reads the output here.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <array>
#include <utility>

#include "boys.h"
#include "boys_common.hpp"
#include "boys_device_f64.hpp"

namespace boys {
namespace {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

// Streaming stores: non-temporal, at device scope (the nt and sc1 bits of
// the store).  The output is written once and read only after the kernel
// ends.  Measured at 2^26 arguments and kmax 32: 2.84 ms per launch
// (6.42 TB/s) against 3.07 ms with the non-temporal bit alone (what the
// compiler's non-temporal store builtin sets), 2.98 ms with nt at workgroup
// scope (sc0) and 3.26 ms at system scope without nt.  Only the buffer-store
// builtin takes the scope bits, so a wave's 64 contiguous rows are written
// through a buffer resource that spans exactly those rows: every offset is
// inside it, and the compiler sees an ordinary store (its hazards and waits
// included).
constexpr int kStreamPolicy = 2 | 16;  // nt | sc1
constexpr int kRawBufferFlags = 0x00020000;  // dword 3 of a raw gfx9 buffer resource

// Waves per workgroup of the write-out kernel for order K.  The LDS stage
// takes 64*(K+1)*8 bytes per wave; four-wave groups at orders above 32
// (84 KB per group at order 40) fit one group, four waves, per CU, too few
// to keep the stores in flight.  Those orders run two-wave groups (three to
// four groups per CU).  Measured at 2^26 arguments: order 40 in 4.19 ms with
// two-wave groups against 4.79 ms with four and 4.24 ms with one; staging 32
// rows at a time to raise occupancy further, or a persistent grid, was slower.
constexpr int eval_waves(int K) { return K > kF64Kmax ? 2 : kWavesPerBlock; }

template <int K, class T>
__global__ __launch_bounds__(64 * eval_waves(K)) void eval_f64_kernel(
    const double *__restrict__ x, int64_t n, double *__restrict__ out, int64_t ld,
    int contiguous) {
  constexpr int C = K + 1;                      // doubles per output row
  constexpr int CP = (C % 2 == 0) ? C + 1 : C;  // LDS row stride (odd)
  constexpr int WB = eval_waves(K);
  __shared__ __attribute__((aligned(16))) double stage[WB * 64 * CP];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: the buffer base below
  double *slice = stage + wave * 64 * CP;

  for (int64_t blk = blockIdx.x; blk * (64 * WB) < n; blk += gridDim.x) {
    const int64_t row0 = blk * (64 * WB) + int64_t(wave) * 64;
    const int64_t i = row0 + lane;
    double F[C];
    // From kmax 8 on, where the store stream sets the time, waves evaluate
    // at raised issue priority and store at the default: a wave still
    // evaluating gets the SIMD ahead of waves in their store bursts, so it
    // reaches its own stores sooner and the stream stays fed.  Measured on
    // 2^26 arguments in alternating processes: kmax 32 2.825-2.827 ms
    // against 2.901-2.909 ms without, kmax 16 1.583-1.591 against
    // 1.691-1.693, kmax 8 0.925-0.928 against 0.963-0.978, kmax 12 and 24
    // even; at kmax 0-4, bound by the evaluation, 1.5-2.5% slower, so not
    // there.  Raising the priority for the stores instead was slower.
    if constexpr (K >= 8) __builtin_amdgcn_s_setprio(3);
    boys_f64<K, T>(i < n ? x[i] : 0.0, F);
#pragma unroll
    for (int l = 0; l < C; ++l) slice[lane * CP + l] = F[l];
    __syncthreads();
    if constexpr (K >= 8) __builtin_amdgcn_s_setprio(0);
    const int64_t rows = n - row0 < 64 ? n - row0 : 64;
    if (contiguous && rows == 64) {
      // The wave's 64 rows are 64*C contiguous doubles = 32*C 16-byte units.
      const __amdgpu_buffer_rsrc_t rows_rsrc =
          __builtin_amdgcn_make_buffer_rsrc(out + row0 * C, 0, 64 * C * 8, kRawBufferFlags);
#pragma unroll
      for (int j = 0; j < (32 * C + 63) / 64; ++j) {
        const int u = lane + 64 * j;
        if (u < 32 * C) {
          d2 v;
          if constexpr (CP == C) {
            v = reinterpret_cast<const d2 *>(slice)[u];
          } else {  // even C: a unit never straddles two rows
            const int r = (2 * u) / C, c = 2 * u - r * C;
            v = d2{slice[r * CP + c], slice[r * CP + c + 1]};
          }
          __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), rows_rsrc, u * 16, 0,
                                                 kStreamPolicy);
        }
      }
    } else if (rows > 0) {
      const int total = int(rows) * C;
      for (int e = lane; e < total; e += 64) {
        const int r = e / C, c = e - r * C;
        __builtin_nontemporal_store(slice[r * CP + c], out + (row0 + r) * ld + c);
      }
    }
    __syncthreads();
  }
}

using EvalKernel = void (*)(const double *, int64_t, double *, int64_t, int);

template <class T, std::size_t... K>
constexpr auto make_table(std::index_sequence<K...>) {
  return std::array<EvalKernel, sizeof...(K)>{{&eval_f64_kernel<int(K), T>...}};
}
constexpr auto kEvalTable = make_table<PaperTables>(std::make_index_sequence<kF64Kmax + 1>{});
constexpr auto kEvalTableScreen =
    make_table<ScreenTables>(std::make_index_sequence<kF64Kmax + 1>{});
constexpr auto kEvalTableCentre =
    make_table<CentreTables>(std::make_index_sequence<kF64Kmax + 1>{});

// The per-kmax regions: order K with row K of the per-kmax set (row 32 is
// the paper's set, so K = 32 takes the paper's kernel).
template <std::size_t... K>
constexpr auto make_per_kmax_table(std::index_sequence<K...>) {
  return std::array<EvalKernel, sizeof...(K) + 1>{
      {&eval_f64_kernel<int(K), PerKmaxTables<int(K)>>..., &eval_f64_kernel<kF64Kmax, PaperTables>}};
}
constexpr auto kEvalTablePerKmax = make_per_kmax_table(std::make_index_sequence<kF64Kmax>{});

// Orders above 32: the high-order set (its orders up to 32 are not needed:
// the paper's tables cover them at the same accuracy).
template <std::size_t... I>
constexpr auto make_high_table(std::index_sequence<I...>) {
  return std::array<EvalKernel, sizeof...(I)>{
      {&eval_f64_kernel<kF64Kmax + 1 + int(I), HighTables>...}};
}
constexpr auto kEvalTableHigh =
    make_high_table(std::make_index_sequence<kHighKmax - kF64Kmax>{});

}  // namespace
}  // namespace boys

extern "C" int boys_eval_f64(const double *x, int64_t n, int kmax, double *out, int64_t ld_out,
                             hipStream_t stream) {
  return boys_eval_f64_tol(x, n, kmax, boys::PaperTables::eps, out, ld_out, stream);
}

extern "C" int boys_eval_f64_tol(const double *x, int64_t n, int kmax, double tol, double *out,
                                 int64_t ld_out, hipStream_t stream) {
  using namespace boys;
  const int set = table_set_for(kmax, tol);
  if (set < 0) return BOYS_EINVAL;
  if (n < 0 || ld_out < kmax + 1) return BOYS_EINVAL;
  if (n == 0) return BOYS_OK;
  if (!x || !out) return BOYS_EINVAL;
  if (n - 1 > (INT64_MAX / 8 - (kmax + 1)) / ld_out) return BOYS_EINVAL;
  const int64_t out_bytes = ((n - 1) * ld_out + kmax + 1) * 8;
  if (overlaps(x, n * 8, out, out_bytes)) return BOYS_EINVAL;
  if (int st = check_device()) return st;

  const int contiguous = ld_out == kmax + 1 && (reinterpret_cast<uintptr_t>(out) & 15) == 0;
  const int block = 64 * eval_waves(kmax);
  int64_t blocks = (n + block - 1) / block;
  if (blocks > kMaxBlocks) blocks = kMaxBlocks;
  EvalKernel kernel = kEvalTable[kmax < kF64Kmax ? kmax : kF64Kmax];
  if (set == kSetHigh) kernel = kEvalTableHigh[kmax - kF64Kmax - 1];
  else if (set == kSetScreen) kernel = kEvalTableScreen[kmax];
  else if (table_variant() == BOYS_TABLES_PER_KMAX) kernel = kEvalTablePerKmax[kmax];
  else if (table_variant() == BOYS_TABLES_CENTRE) kernel = kEvalTableCentre[kmax];
  hipLaunchKernelGGL(kernel, dim3(unsigned(blocks)), dim3(block), 0, stream, x, n, out, ld_out,
                     contiguous);
  return hip_status(hipGetLastError());
}
