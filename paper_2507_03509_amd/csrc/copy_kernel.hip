// Plain device-to-device copy: the achievable-bandwidth reference of the
// measurements.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "host_common.hpp"
#include "ssfm.h"

namespace {

// One pass, no grid-stride loop: workgroup g copies the 1024 vectors
// [1024 g, 1024 g + 1024) in four rounds of 256 consecutive 16-byte vectors
// (each load instruction fully coalesced), all four loads before the stores.
__global__ __launch_bounds__(256) void stream_copy(float4* __restrict__ dst,
                                                   const float4* __restrict__ src, int64_t n) {
  const int64_t i0 = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  if (i0 + 768 < n) {
    const float4 a = src[i0], b = src[i0 + 256], c = src[i0 + 512], d = src[i0 + 768];
    dst[i0] = a;
    dst[i0 + 256] = b;
    dst[i0 + 512] = c;
    dst[i0 + 768] = d;
  } else {
    for (int k = 0; k < 4; ++k)
      if (i0 + 256 * k < n) dst[i0 + 256 * k] = src[i0 + 256 * k];
  }
}

}  // namespace

extern "C" int ssfm_stream_copy(void* dst, const void* src, int64_t bytes, void* stream) {
  ssfm::api_clear_error();
  if (!dst || !src) return ssfm::api_fail(SSFM_EINVAL, "NULL copy buffer");
  if ((((uintptr_t)dst | (uintptr_t)src) & 15) != 0 || bytes < 0 || bytes % 16 != 0)
    return ssfm::api_fail(SSFM_EINVAL, "copy needs 16-byte aligned buffers and size (got %lld)",
                          (long long)bytes);
  if (bytes == 0) return SSFM_OK;
  const int64_t n = bytes / 16;
  const int64_t blocks64 = (n + 1023) / 1024;
  if (blocks64 > 0x7fffffff) return ssfm::api_fail(SSFM_EINVAL, "copy of %lld bytes too large", (long long)bytes);
  const unsigned blocks = (unsigned)blocks64;
  hipLaunchKernelGGL(stream_copy, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                     static_cast<float4*>(dst), static_cast<const float4*>(src), n);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SSFM_OK : ssfm::api_fail_hip(e, "stream_copy launch");
}
