// Device helpers: deterministic wavefront / workgroup reductions and the
// "last workgroup finishes the reduction" pattern (integer ticket only, no
// floating-point atomics, so every sum has a fixed order).
#pragma once
#include <hip/hip_runtime.h>
#include "common.h"

namespace msp {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ float wave_sumf(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the workgroup; sh must hold NT/64 + 1 doubles.  All threads get
// the result.  Fixed order: butterfly inside waves, then waves in order.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  static_assert(NT % 64 == 0, "workgroup must be whole waves");
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) r += sh[i];
    sh[NT / 64] = r;
  }
  __syncthreads();
  const double r = sh[NT / 64];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double load_coherent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Returns true in exactly one workgroup: the last one to arrive.  The
// partial results written before the call are visible to it.  The caller's
// last workgroup must reset *counter to 0 (thread 0) when done.
__device__ __forceinline__ bool last_block(unsigned int* counter,
                                           unsigned int nblocks,
                                           unsigned int* sh_ticket) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) *sh_ticket = atomicAdd(counter, 1u);
  __syncthreads();
  const bool last = (*sh_ticket == nblocks - 1);
  if (last) __threadfence();
  return last;
}

// Fixed-order sum of nb partials (stride between consecutive partials:
// `stride` doubles) inside the last workgroup.
template <int NT>
__device__ __forceinline__ double reduce_partials(const double* part, int nb,
                                                  int stride, double* sh) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += NT) s += load_coherent(part + (long long)i * stride);
  return block_sum<NT>(s, sh);
}

__device__ __forceinline__ bool finite(double v) {
  return __builtin_isfinite(v);
}

}  // namespace msp
