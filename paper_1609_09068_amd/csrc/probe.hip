// Achievable read bandwidth of the device: the ceiling the solve's
// gather-bound kernels are measured against.  One pass reads the buffer with
// 16-byte loads, four in flight per thread, and folds them into one float per
// thread (written out so the loads are not dropped).
#include <chrono>

#include "internal.h"

namespace prlib {
namespace {

constexpr int kProbeThreads = 256;

__global__ __launch_bounds__(kProbeThreads) void k_read_probe(const float4* __restrict__ a, int64_t n16,
                                                              float* __restrict__ sink) {
  const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
  int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
  float s = 0.f;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const float4 v0 = a[i], v1 = a[i + stride], v2 = a[i + 2 * stride], v3 = a[i + 3 * stride];
    s += ((v0.x + v1.y) + (v2.z + v3.w));
  }
  for (; i < n16; i += stride) s += a[i].x;
  sink[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

}  // namespace
}  // namespace prlib

using namespace prlib;

extern "C" int32_t pr_bandwidth_probe(const void* buf_dev, int64_t bytes, int32_t reps, void* hip_stream,
                                      double* ms_out) {
  if (!buf_dev || bytes < 16 || reps <= 0 || !ms_out || ((uintptr_t)buf_dev & 15u)) {
    set_error("bad arguments (need a 16-byte aligned buffer of at least 16 bytes, reps > 0, ms_out)");
    return PR_EINVAL;
  }
  int dev = 0, cus = 0;
  PR_HIP_CHECK(hipGetDevice(&dev));
  PR_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const hipStream_t s = (hipStream_t)hip_stream;
  const int64_t n16 = bytes / 16;
  const int grid = std::max(1, cus) * 8;
  float* sink = nullptr;
  PR_HIP_CHECK(hipMalloc(&sink, sizeof(float) * (size_t)grid * kProbeThreads));
  hipEvent_t e0, e1;
  PR_HIP_CHECK(hipEventCreate(&e0));
  PR_HIP_CHECK(hipEventCreate(&e1));
  const float4* a = reinterpret_cast<const float4*>(buf_dev);
  for (int w = 0; w < 2; ++w) k_read_probe<<<grid, kProbeThreads, 0, s>>>(a, n16, sink);
  PR_HIP_CHECK(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) k_read_probe<<<grid, kProbeThreads, 0, s>>>(a, n16, sink);
  PR_HIP_CHECK(hipEventRecord(e1, s));
  PR_HIP_CHECK(hipEventSynchronize(e1));
  float ms = 0.f;
  PR_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(sink);
  PR_HIP_CHECK(hipGetLastError());
  *ms_out = (double)ms / reps;
  return PR_OK;
}
