// Small dense helpers shared by the heat eigen iterations: a counter-based
// uniform generator, and Cholesky and Jacobi eigen decompositions of an
// m x m matrix (m <= MAXM) held in LDS by one workgroup of NT threads.
#pragma once
#include "dev.h"

namespace msp {

__device__ __forceinline__ double hash_unit(unsigned long long a) {
  // splitmix64 finaliser -> uniform in [-1, 1)
  a += 0x9E3779B97F4A7C15ull;
  a = (a ^ (a >> 30)) * 0xBF58476D1CE4E5B9ull;
  a = (a ^ (a >> 27)) * 0x94D049BB133111EBull;
  a ^= a >> 31;
  return (double)(a >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

template <int NT>
__device__ void chol_small(double* G, int m, int* __restrict__ err) {
  const int tid = threadIdx.x;
  for (int p = 0; p < m; ++p) {
    __syncthreads();
    double d = G[p * m + p];
    if (!(d > 0.0) || !finite(d)) {
      if (tid == 0) atomicOr(err, ERR_EIG);
      d = 1e-300;
    }
    const double piv = sqrt(d);
    __syncthreads();
    for (int i = tid; i < m; i += NT) {
      if (i == p) G[p * m + p] = piv;
      else if (i > p) G[i * m + p] /= piv;
    }
    __syncthreads();
    for (int idx = tid; idx < m * m; idx += NT) {
      const int i = idx / m, j = idx - (idx / m) * m;
      if (i > p && j > p && j <= i) G[i * m + j] -= G[i * m + p] * G[j * m + p];
    }
  }
  __syncthreads();
}

// Jacobi eigenvalues of the symmetric m x m matrix A (LDS, stride m);
// V (LDS, stride m) receives the eigenvectors as columns.  Parallel
// round-robin ordering: m/2 disjoint rotations per round.
template <int NT>
__device__ void jacobi_small(double* A, double* V, int m, double* rc,
                             double* rs, int* rp, int* rq) {
  const int tid = threadIdx.x;
  const int me = (m + 1) & ~1;            // even number of players
  for (int idx = tid; idx < m * m; idx += NT) {
    const int i = idx / m, j = idx - (idx / m) * m;
    V[idx] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  __shared__ double jred[NT / 64 + 1];
  for (int sweep = 0; sweep < 30; ++sweep) {
    // convergence test: off-diagonal and diagonal squares, summed by the
    // whole workgroup (fixed order)
    double o = 0.0, d = 0.0;
    for (int idx = tid; idx < m * m; idx += NT) {
      const int i = idx / m, j = idx - (idx / m) * m;
      const double a = A[idx];
      if (i == j) d += a * a; else o += a * a;
    }
    const double offn = block_sum<NT>(o, jred);
    const double diagn = block_sum<NT>(d, jred);
    if (offn <= 1e-30 * diagn || offn == 0.0) break;
    for (int r = 0; r < me - 1; ++r) {
      if (tid < me / 2) {
        int p, q;
        if (tid == 0) {
          p = 0;
          q = 1 + (r % (me - 1));
        } else {
          p = 1 + (r + tid) % (me - 1);
          q = 1 + (r - tid + me - 1) % (me - 1);
        }
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, sn = 0.0;
        if (q < m) {
          const double apq = A[p * m + q];
          if (fabs(apq) > 1e-300) {
            const double th = (A[q * m + q] - A[p * m + p]) / (2.0 * apq);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            sn = t * c;
          }
        }
        rc[tid] = c;
        rs[tid] = sn;
        rp[tid] = p;
        rq[tid] = q;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int idx = tid; idx < (me / 2) * m; idx += NT) {
        const int pr = idx / m, col = idx - (idx / m) * m;
        const int p = rp[pr], q = rq[pr];
        if (q < m) {
          const double c = rc[pr], sn = rs[pr];
          const double ap = A[p * m + col], aq = A[q * m + col];
          A[p * m + col] = c * ap - sn * aq;
          A[q * m + col] = sn * ap + c * aq;
        }
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int idx = tid; idx < (me / 2) * m; idx += NT) {
        const int pr = idx / m, row = idx - (idx / m) * m;
        const int p = rp[pr], q = rq[pr];
        if (q < m) {
          const double c = rc[pr], sn = rs[pr];
          const double ap = A[row * m + p], aq = A[row * m + q];
          A[row * m + p] = c * ap - sn * aq;
          A[row * m + q] = sn * ap + c * aq;
          const double vp = V[row * m + p], vq = V[row * m + q];
          V[row * m + p] = c * vp - sn * vq;
          V[row * m + q] = sn * vp + c * vq;
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
}

}  // namespace msp
