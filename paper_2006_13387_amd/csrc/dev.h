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

// Two sums over the workgroup at once, each in block_sum's order; sh must
// hold 2 (NT/64) doubles.  All threads get both results.
template <int NT>
__device__ __forceinline__ double2 block_sum2(double a, double b, double* sh) {
  static_assert(NT % 64 == 0, "workgroup must be whole waves");
  constexpr int W = NT / 64;
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[w] = a;
    sh[W + w] = b;
  }
  __syncthreads();
  double ra = 0.0, rb = 0.0;
#pragma unroll
  for (int i = 0; i < W; ++i) {
    ra += sh[i];
    rb += sh[W + i];
  }
  __syncthreads();
  return make_double2(ra, rb);
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

// Block-uniform read of the CG "done" word (another workgroup of the same
// kernel may write it while this one runs; the value is read once by thread
// 0 and broadcast through LDS so that every thread takes the same branch).
__device__ __forceinline__ int block_read_done(const CGScalars* sc, int* sh) {
  if (threadIdx.x == 0)
    *sh = __hip_atomic_load(&sc->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const int d = *sh;
  __syncthreads();
  return d;
}

// Convergence test after the update x += alpha p, r -= alpha q: every
// workgroup sums the update kernel's partials of r.r in the same fixed
// order; the leader (the problem's workgroup 0) records the outcome.
// Returns true when the iteration is over (converged, iteration limit or
// non-finite residual).  The done word, the counters and the partials are
// read together (one memory latency); a workgroup that finds the solve
// already over ignores the sum.  The counters are read before any leader
// can advance them in this launch, so every workgroup decides alike.  Only
// threads below NLD read partials (a workgroup whose other waves have
// copies in flight keeps their memory counters to those copies).
template <int NT, int NLD = NT>
__device__ bool cg_check_done(CGScalars* sc, const double* part_upd, int nb_upd,
                              double* red, int* sh, bool leader) {
  int d0 = DONE_RUNNING, it0 = 0, maxit = 0;
  double tol2 = 0.0, ff = 0.0;
  if (threadIdx.x == 0) {
    d0 = __hip_atomic_load(&sc->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    it0 = __hip_atomic_load(&sc->iter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    maxit = sc->maxit;
    tol2 = sc->tol2;
    ff = sc->ff;
  }
  double s = 0.0;
  if ((int)threadIdx.x < NLD)
    for (int i = threadIdx.x; i < nb_upd; i += NLD) s += load_coherent(part_upd + i);
  const double rr = block_sum<NT>(s, red);
  if (threadIdx.x == 0) {
    int d = d0;
    if (d0 == DONE_RUNNING) {
      const int it1 = it0 + 1;
      if (!finite(rr)) d = DONE_BREAKDOWN;
      else if (rr <= tol2 * ff) d = DONE_CONVERGED;
      else if (it1 >= maxit) d = DONE_MAXIT;
      if (d != DONE_RUNNING && leader) {
        sc->rr = rr;
        sc->iter = it1;
        if (d == DONE_BREAKDOWN) sc->status = -5;
        __hip_atomic_store(&sc->done, d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    *sh = d;
  }
  __syncthreads();
  const bool over = *sh != DONE_RUNNING;
  __syncthreads();
  return over;
}

}  // namespace msp
