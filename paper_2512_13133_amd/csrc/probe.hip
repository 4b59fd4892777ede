// A plain streaming read of a device buffer, timed with HIP events on the
// caller's stream: the HBM read bandwidth an ordinary kernel reaches on this
// device, the practical ceiling to set beside the published peak when
// reading the roofline of the alignment kernels.  A measurement aid; no part
// of the method uses it.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/clipalign.h"

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_BLOCKS = 8192;  // 32 workgroups per compute unit

// Written only when a block's fold hits one 32-bit value, which keeps the
// loads live without adding traffic (external linkage, so the compiler cannot
// drop the store and the loads behind it).
__device__ uint32_t clipalign_probe_sink[PROBE_BLOCKS];

namespace {

// Grid-stride over 16-byte words, sixteen loads in flight per thread.
__global__ void __launch_bounds__(PROBE_THREADS) read_probe_kernel(const uint4* __restrict__ p, int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * PROBE_THREADS;
  uint32_t acc = 0;
  int64_t t = (int64_t)blockIdx.x * PROBE_THREADS + threadIdx.x;
  for (; t + 15 * stride < n16; t += 16 * stride) {
    uint4 v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = p[t + u * stride];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (; t < n16; t += stride) {
    const uint4 a = p[t];
    acc ^= a.x ^ a.y ^ a.z ^ a.w;
  }
  if (acc == 0x9e3779b9u) clipalign_probe_sink[blockIdx.x] = acc;
}

}  // namespace

extern "C" ca_status ca_probe_read_bandwidth(void* stream, const void* buf, uint64_t bytes, int32_t reps,
                                             double* ms_per_read) {
  if (!buf || !ms_per_read || bytes == 0 || (bytes & 15) || ((uintptr_t)buf & 15) || reps < 1) return CA_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n16 = (int64_t)(bytes / 16);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return CA_EDEVICE;
  }
  ca_status st = CA_OK;
  float ms = 0.0f;
  hipLaunchKernelGGL(read_probe_kernel, dim3(PROBE_BLOCKS), dim3(PROBE_THREADS), 0, s, (const uint4*)buf, n16);
  if (hipGetLastError() != hipSuccess || hipEventRecord(e0, s) != hipSuccess) st = CA_EDEVICE;
  for (int r = 0; st == CA_OK && r < reps; ++r) {
    hipLaunchKernelGGL(read_probe_kernel, dim3(PROBE_BLOCKS), dim3(PROBE_THREADS), 0, s, (const uint4*)buf, n16);
    if (hipGetLastError() != hipSuccess) st = CA_EDEVICE;
  }
  if (st == CA_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                      hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    st = CA_EDEVICE;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == CA_OK) *ms_per_read = (double)ms / reps;
  return st;
}
