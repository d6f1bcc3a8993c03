// boys_eval_f32: FP32 write-out of F_0..F_kmax (kmax <= 16) on gfx950.
//
// Same structure as the FP64 write-out: one lane per argument, values in
// VGPRs, each wave's 64 rows staged in its LDS slice (odd row stride, free of
// bank conflicts) and written back as 16-byte non-temporal stores covering
// consecutive addresses.  Per argument 4 bytes are read and 4*(kmax+1)
// written, half the traffic of the FP64 path.
#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <utility>

#include "boys.h"
#include "boys_common.hpp"
#include "boys_device_f32.hpp"

namespace boys {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

template <int K>
__global__ __launch_bounds__(kBlock) void eval_f32_kernel(const float *__restrict__ x, int64_t n,
                                                          float *__restrict__ out, int64_t ld,
                                                          int contiguous) {
  constexpr int C = K + 1;                      // floats per output row
  constexpr int CP = (C % 2 == 0) ? C + 1 : C;  // LDS row stride (odd)
  __shared__ __attribute__((aligned(16))) float stage[kWavesPerBlock * 64 * CP];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  float *slice = stage + wave * 64 * CP;

  for (int64_t blk = blockIdx.x; blk * kBlock < n; blk += gridDim.x) {
    const int64_t row0 = blk * kBlock + int64_t(wave) * 64;
    const int64_t i = row0 + lane;
    float F[C];
    boys_f32<K>(i < n ? x[i] : 0.0f, F);
#pragma unroll
    for (int l = 0; l < C; ++l) slice[lane * CP + l] = F[l];
    __syncthreads();
    const int64_t rows = n - row0 < 64 ? n - row0 : 64;
    if (contiguous && rows == 64) {
      // 64*C floats = 16*C units of 16 bytes.
      f4 *dst = reinterpret_cast<f4 *>(out + row0 * C);
#pragma unroll
      for (int j = 0; j < (16 * C + 63) / 64; ++j) {
        const int u = lane + 64 * j;
        if (u < 16 * C) {
          f4 v;
          if constexpr (CP == C) {
            // Unpadded rows (odd C): the wave's rows are contiguous in LDS,
            // so unit u is floats 4u..4u+3 of the slice, 16-byte aligned
            // (slices start at multiples of 256 C bytes).
            v = reinterpret_cast<const f4 *>(slice)[u];
          } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              const int e = 4 * u + t, r = e / C, c = e - r * C;
              v[t] = slice[r * CP + c];
            }
          }
          __builtin_nontemporal_store(v, dst + u);
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

using EvalKernel = void (*)(const float *, int64_t, float *, int64_t, int);

template <std::size_t... K>
constexpr auto make_table(std::index_sequence<K...>) {
  return std::array<EvalKernel, sizeof...(K)>{{&eval_f32_kernel<int(K)>...}};
}
constexpr auto kEvalTable = make_table(std::make_index_sequence<kF32Kmax + 1>{});

}  // namespace
}  // namespace boys

extern "C" int boys_eval_f32(const float *x, int64_t n, int kmax, float *out, int64_t ld_out,
                             hipStream_t stream) {
  using namespace boys;
  if (n < 0 || kmax < 0 || kmax > kF32Kmax || ld_out < kmax + 1) return BOYS_EINVAL;
  if (n == 0) return BOYS_OK;
  if (!x || !out) return BOYS_EINVAL;
  if (n - 1 > (INT64_MAX / 4 - (kmax + 1)) / ld_out) return BOYS_EINVAL;
  const int64_t out_bytes = ((n - 1) * ld_out + kmax + 1) * 4;
  if (overlaps(x, n * 4, out, out_bytes)) return BOYS_EINVAL;
  if (int st = check_device()) return st;

  const int contiguous = ld_out == kmax + 1 && (reinterpret_cast<uintptr_t>(out) & 15) == 0;
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > kMaxBlocks) blocks = kMaxBlocks;
  hipLaunchKernelGGL(kEvalTable[kmax], dim3(unsigned(blocks)), dim3(kBlock), 0, stream, x, n, out,
                     ld_out, contiguous);
  return hip_status(hipGetLastError());
}
