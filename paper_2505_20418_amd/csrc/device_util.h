// Device helpers shared by the HIP kernels: deterministic wavefront and
// workgroup reductions (fixed shuffle tree, fixed LDS order), partial-slot
// sums, and the XCD-aware workgroup remapping.
#pragma once

#include <hip/hip_runtime.h>

#include "maze_internal.h"

namespace maze {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;  // valid in lane 0
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  return v;
}

// Sum over the 256 threads of a workgroup; every thread gets the result.
// sm: at least 4 doubles of LDS. Fixed order: shuffle tree per wave, then
// waves 0..3 in order.
__device__ __forceinline__ double block_sum(double v, double* sm) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sm[w] = v;
  __syncthreads();
  double s = sm[0];
#pragma unroll
  for (int i = 1; i < kThreads / 64; ++i) s += sm[i];
  return s;
}

__device__ __forceinline__ double block_max(double v, double* sm) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sm[w] = v;
  __syncthreads();
  double s = sm[0];
#pragma unroll
  for (int i = 1; i < kThreads / 64; ++i) s = fmax(s, sm[i]);
  return s;
}

// Deterministic sum of n partials (each thread a strided subsequence in
// order, then the fixed workgroup tree). Identical in every workgroup.
__device__ __forceinline__ double sum_partials(const double* part, int n, double* sm) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) v += part[i];
  return block_sum(v, sm);
}

__device__ __forceinline__ double max_partials(const double* part, int n, double* sm) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) v = fmax(v, part[i]);
  return block_max(v, sm);
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b % 8). Remap so that each XCD receives a contiguous range of logical
// workgroup ids: neighbouring segments of the same x planes then share one
// XCD's L2, which serves their overlapping halo rows.
__device__ __forceinline__ int xcd_remap(int b, int nwg) {
  constexpr int X = 8;
  const int q = nwg / X, rem = nwg % X;
  const int xcd = b % X, i = b / X;
  return (xcd < rem) ? xcd * (q + 1) + i : rem * (q + 1) + (xcd - rem) * q + i;
}

__device__ __forceinline__ volatile int32_t* vol(int32_t* p) { return p; }

// Access to the device scalars (Scalars) that one kernel writes and a later
// kernel reads. Plain uniform loads of them may be compiled to scalar-cache
// loads, and the scalar cache is not kept coherent with vector stores of an
// earlier kernel, so every such access is an agent-scope relaxed atomic:
// a vector load or store that reaches the coherent level of the hierarchy.
template <typename T>
__device__ __forceinline__ T ctl_ld(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void ctl_st(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Whether either of two control words (the done and error flags of a
// solve) is set, decided once for the whole workgroup: thread 0 reads them
// and shares the answer through a word of the caller's LDS (slot), which
// is the caller's again on return. A solve's leader may set its done flag
// while other workgroups of the same launch are starting; if each thread
// read it for itself, part of a workgroup could leave while the rest went
// on to a workgroup reduction short of the leavers' shares. The slot is
// borrowed rather than declared: a static LDS word would raise a kernel's
// LDS just past what lets four 256-thread workgroups share a CU. Every
// thread of the workgroup must call it (it holds two barriers).
__device__ __forceinline__ bool wg_flags_set(const int32_t* a, const int32_t* b, int32_t* slot) {
  if (threadIdx.x == 0) *slot = (ctl_ld(a) != 0 || ctl_ld(b) != 0) ? 1 : 0;
  __syncthreads();
  const bool set = *slot != 0;
  __syncthreads();
  return set;
}

}  // namespace maze
