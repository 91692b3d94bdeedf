// Host-side helpers shared by the C-ABI translation units of libssfm: the
// thread-local error message behind ssfm_last_error() and a guard that
// restores the caller's current device.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

namespace ssfm {

// Record a formatted message for ssfm_last_error() and return `code`.
int api_fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
// api_fail(SSFM_EHIP, ...) with the HIP error's name and number.
int api_fail_hip(hipError_t e, const char* what);
// The message of the last failing call on this thread.
const std::string& api_last_error();
// Clear it (every C-ABI entry point does on entry).
void api_clear_error();

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  hipError_t status = hipSuccess;
  explicit DeviceGuard(int dev) {
    status = hipGetDevice(&prev);
    if (status == hipSuccess && prev != dev) status = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
  DeviceGuard(const DeviceGuard&) = delete;
  DeviceGuard& operator=(const DeviceGuard&) = delete;
};

}  // namespace ssfm
