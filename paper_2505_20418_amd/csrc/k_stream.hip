// Streaming copy: the practical HBM ceiling of this device for a kernel
// that reads and writes every byte once (the traffic pattern of the CG
// sweeps and update kernels), measured on footprints far beyond the L2 and
// the Infinity Cache. Each thread moves 16-byte vectors with plain vector
// loads and stores; the grid is a few workgroups per CU, striding over the
// buffer, so every wavefront keeps several loads in flight.
#include <algorithm>

#include "device_util.h"

namespace maze {

namespace {

constexpr int kStreamThreads = 256;
constexpr int kStreamUnroll = 4;

__global__ __launch_bounds__(kStreamThreads) void k_stream_copy(const uint4* __restrict__ src,
                                                                uint4* __restrict__ dst,
                                                                long long n) {
  const long long stride = (long long)gridDim.x * kStreamThreads;
  long long i = (long long)blockIdx.x * kStreamThreads + threadIdx.x;
  for (; i + (kStreamUnroll - 1) * stride < n; i += kStreamUnroll * stride) {
    uint4 v[kStreamUnroll];
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) v[u] = src[i + u * stride];
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) dst[i + u * stride] = v[u];
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, int cus,
                              hipStream_t st) {
  const long long n = (long long)(bytes / sizeof(uint4));
  if (n <= 0) return hipSuccess;
  const long long want = (long long)std::max(cus, 1) * 8;
  const long long need = (n + kStreamThreads - 1) / kStreamThreads;
  const int blocks = (int)std::max(1LL, std::min(want, need));
  hipLaunchKernelGGL(k_stream_copy, dim3(blocks), dim3(kStreamThreads), 0, st,
                     static_cast<const uint4*>(src), static_cast<uint4*>(dst), n);
  return hipGetLastError();
}

}  // namespace maze
