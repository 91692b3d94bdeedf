// Measurement utility: the cost of the two ways of ordering the dependent
// passes of a split-step call -- a kernel boundary (graph replay or direct
// launches of dependent kernels on one stream) against a device-wide barrier
// inside one persistent cooperative kernel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "host_common.hpp"
#include "ssfm.h"

namespace {

// Device-wide barrier of the cooperative probe: lane 0 of every workgroup
// takes the generation, arrives on the counter (the last arrival resets it
// and advances the generation) and waits, with a bounded spin, for the
// generation to move.  Returns false once any workgroup's spin ran out.
__device__ __forceinline__ bool grid_barrier(unsigned* count, unsigned* gen, int* err,
                                             unsigned spin_max) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    ok = 1;
    const unsigned g = __hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned arrived =
        __hip_atomic_fetch_add(count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == gridDim.x - 1) {
      __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned it = 0;
      while (__hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (++it > spin_max) {
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
  }
  __syncthreads();
  return ok != 0;
}

// sync: [0] arrival counter, [32] generation (own 128-byte lines), [64] error
__global__ __launch_bounds__(256) void barrier_rounds(unsigned* sync, int rounds,
                                                      unsigned spin_max) {
  int* err = reinterpret_cast<int*>(sync + 64);
  for (int r = 0; r < rounds; ++r) {
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
    if (!grid_barrier(sync, sync + 32, err, spin_max)) break;
  }
}

// a kernel with no work: its launches measure the boundary alone
__global__ __launch_bounds__(256) void empty_pass(int* never) {
  if (threadIdx.x == 0x7fffffff) *never = 0;
}

}  // namespace

extern "C" int ssfm_orchestration_probe(int method, int32_t workgroups, int32_t rounds,
                                        void* stream, double* us_per_round) {
  ssfm::api_clear_error();
  if (!us_per_round) return ssfm::api_fail(SSFM_EINVAL, "us_per_round is NULL");
  *us_per_round = 0.0;
  if (method < 0 || method > 2) return ssfm::api_fail(SSFM_EINVAL, "method %d not 0, 1 or 2", method);
  if (rounds < 1 || rounds > 65536)
    return ssfm::api_fail(SSFM_EINVAL, "rounds %d outside [1, 65536]", rounds);
  hipStream_t st = static_cast<hipStream_t>(stream);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return ssfm::api_fail_hip(e, "hipGetDevice");
  int cus = 0, per_cu = 0;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return ssfm::api_fail_hip(e, "hipDeviceGetAttribute");
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, barrier_rounds, 256, 0)) !=
      hipSuccess)
    return ssfm::api_fail_hip(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
  // the cooperative kernel needs every workgroup resident at once
  const int64_t cap = method == 2 ? (int64_t)cus * per_cu : 65536;
  if (workgroups < 1 || workgroups > cap)
    return ssfm::api_fail(SSFM_EINVAL, "workgroups %d outside [1, %lld]", workgroups,
                          (long long)cap);
  unsigned* sync = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_st = nullptr;
  int herr = 0;
  auto cleanup = [&] {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_st) (void)hipStreamDestroy(cap_st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (sync) (void)hipFree(sync);
  };
  if ((e = hipMalloc(&sync, 512)) != hipSuccess) {
    cleanup();
    return ssfm::api_fail(SSFM_ENOMEM, "probe buffer");
  }
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipMemsetAsync(sync, 0, 512, st);
  int* never = reinterpret_cast<int*>(sync + 96);
  if (e == hipSuccess && method == 0) {
    // graph of `rounds` dependent launches, captured on a stream of its own
    e = hipStreamCreateWithFlags(&cap_st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap_st, hipStreamCaptureModeThreadLocal);
    for (int r = 0; r < rounds && e == hipSuccess; ++r) {
      hipLaunchKernelGGL(empty_pass, dim3(workgroups), dim3(256), 0, cap_st, never);
      e = hipGetLastError();
    }
    if (cap_st) {
      const hipError_t ec = hipStreamEndCapture(cap_st, &graph);
      if (e == hipSuccess) e = ec;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(exec, st);  // warm-up
  }
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  if (e == hipSuccess) {
    if (method == 0) {
      e = hipGraphLaunch(exec, st);
    } else if (method == 1) {
      for (int r = 0; r < rounds && e == hipSuccess; ++r) {
        hipLaunchKernelGGL(empty_pass, dim3(workgroups), dim3(256), 0, st, never);
        e = hipGetLastError();
      }
    } else {
      // ~0.1 s of polling at most per barrier before the probe gives up
      unsigned spin_max = 1u << 21;
      void* args[] = {&sync, &rounds, &spin_max};
      e = hipLaunchCooperativeKernel(reinterpret_cast<void*>(barrier_rounds), dim3(workgroups),
                                     dim3(256), args, 0, st);
    }
  }
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess && method == 2)
    e = hipMemcpy(&herr, sync + 64, sizeof(int), hipMemcpyDeviceToHost);
  cleanup();
  if (e != hipSuccess) return ssfm::api_fail_hip(e, "orchestration probe");
  if (herr) return ssfm::api_fail(SSFM_EHIP, "grid barrier wait ran out");
  *us_per_round = 1e3 * (double)ms / rounds;
  return SSFM_OK;
}
