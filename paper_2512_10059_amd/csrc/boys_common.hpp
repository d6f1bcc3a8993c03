// Host-side plumbing shared by the entry points of libboys.so: status codes,
// HIP error capture and the per-device architecture check.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "boys.h"

namespace boys {

// Records `err` as this thread's last HIP error and returns BOYS_EHIP, or
// BOYS_OK for hipSuccess.
int hip_status(hipError_t err);

// BOYS_OK when the current device is gfx950, BOYS_ENOTSUP otherwise
// (cached per device), BOYS_EHIP if the device cannot be queried.
int check_device();

// BOYS_OK when `stream` is not under graph capture, BOYS_ECAPTURE when it is
// (capturing or invalidated), BOYS_EHIP if the query fails.  The entry points
// that keep a per-device workspace or cached graph refuse captured streams:
// their workspace may have to grow, and a graph replayed later would share it.
int check_not_capturing(hipStream_t stream);

// The process-wide variant of the 5e-14 tables for orders up to 32
// (boys_set_tables): BOYS_TABLES_PAPER, BOYS_TABLES_PER_KMAX or
// BOYS_TABLES_CENTRE.
int table_variant();

// Frees the workspaces of boys_pairsum on every device (boys_finalize).
void pairsum_release_all();

// True when [a, a+abytes) and [b, b+bbytes) overlap.
inline bool overlaps(const void *a, int64_t abytes, const void *b, int64_t bbytes) {
  const auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  return pa < pb + static_cast<uintptr_t>(bbytes) && pb < pa + static_cast<uintptr_t>(abytes);
}

// Blocks of 256 threads (4 wave64) for the streaming kernels.
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;

// Launch-size cap for grid-stride kernels: 2^20 workgroups is far more than
// the 256 CUs need to stay busy, and keeps the grid within limits for any n.
constexpr int64_t kMaxBlocks = int64_t(1) << 20;

#define BOYS_TRY_HIP(expr)                                   \
  do {                                                       \
    hipError_t boys_err_ = (expr);                           \
    if (boys_err_ != hipSuccess) return ::boys::hip_status(boys_err_); \
  } while (0)

}  // namespace boys
