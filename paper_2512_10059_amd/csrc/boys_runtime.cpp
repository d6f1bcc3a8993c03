// Status codes, error capture and device checks of libboys.so.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>
#include <mutex>

#include "boys.h"
#include "boys_common.hpp"

namespace boys {

namespace {
thread_local int g_last_hip_error = 0;
constexpr int kMaxDevices = 64;
// 0 = unknown, 1 = gfx950, -1 = other architecture.
int g_arch_ok[kMaxDevices] = {0};
std::mutex g_arch_mutex;
std::atomic<int> g_table_variant{BOYS_TABLES_PAPER};
}  // namespace

int table_variant() { return g_table_variant.load(std::memory_order_relaxed); }

int hip_status(hipError_t err) {
  if (err == hipSuccess) return BOYS_OK;
  g_last_hip_error = static_cast<int>(err);
  return BOYS_EHIP;
}

int check_device() {
  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return hip_status(err);
  if (dev < 0 || dev >= kMaxDevices) return BOYS_ENOTSUP;
  {
    std::lock_guard<std::mutex> lock(g_arch_mutex);
    if (g_arch_ok[dev] != 0) return g_arch_ok[dev] > 0 ? BOYS_OK : BOYS_ENOTSUP;
  }
  hipDeviceProp_t prop;
  err = hipGetDeviceProperties(&prop, dev);
  if (err != hipSuccess) return hip_status(err);
  const bool ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
  std::lock_guard<std::mutex> lock(g_arch_mutex);
  g_arch_ok[dev] = ok ? 1 : -1;
  return ok ? BOYS_OK : BOYS_ENOTSUP;
}

int check_not_capturing(hipStream_t stream) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t err = hipStreamIsCapturing(stream, &cs);
  if (err != hipSuccess) return hip_status(err);
  return cs == hipStreamCaptureStatusNone ? BOYS_OK : BOYS_ECAPTURE;
}

}  // namespace boys

extern "C" {

const char *boys_strerror(int status) {
  switch (status) {
    case BOYS_OK: return "success";
    case BOYS_EINVAL: return "invalid argument";
    case BOYS_EHIP: return "HIP runtime error";
    case BOYS_ENOTSUP: return "device not supported (libboys needs gfx950)";
    case BOYS_ENOMEM: return "workspace allocation failed";
    case BOYS_ECAPTURE: return "stream is under graph capture (this entry point keeps cached workspaces and graphs)";
    default: return "unknown status";
  }
}

int boys_last_hip_error(void) { return boys::g_last_hip_error; }

int boys_set_tables(int variant) {
  if (variant != BOYS_TABLES_PAPER && variant != BOYS_TABLES_PER_KMAX && variant != BOYS_TABLES_CENTRE)
    return BOYS_EINVAL;
  boys::g_table_variant.store(variant, std::memory_order_relaxed);
  return BOYS_OK;
}

int boys_get_tables(void) { return boys::table_variant(); }

}  // extern "C"
