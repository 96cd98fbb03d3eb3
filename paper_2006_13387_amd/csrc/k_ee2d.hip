// The M_EE coarse space of the 2D (Q1) preconditioner (Section 2.1): on
// every coarse neighbourhood omega_l the lowest eigenpairs of the local
// elasticity pencil -div sigma(psi) = lambda E psi (homogeneous Neumann on
// the boundary of omega_l, Dirichlet on its clamped part), times chi_l.
//
// The pencil K_l + sigma M_l is factored block-tridiagonally by node rows
// (a row of nx nodes holds 2 nx unknowns, u = 2 x + c, padded to the
// shared order ldp) exactly as the 3D heat pencils are by node planes: the
// row's Schur complement assembled from E, then its inverse by the batched
// Gauss-Jordan elimination.  The subspace iteration, its Gram matrices,
// Rayleigh-Ritz step, Ritz vectors and stopping test are the plane
// machinery of the 3D heat pencils (rows of unknowns instead of nodes).
//
// The coarse operator of M_EE is kept dense (a comparator for the paper's
// 100 x 100 examples, not the benchmark's path): Phi as an n x N_c column-
// major matrix, K Phi by the stiffness product, K_0 = Phi^T (K Phi), its
// generalised inverse by the Gauss-Jordan elimination of the 2D path; per
// PCG iteration c = Phi^T r, c0 = K_0^+ c and z += Phi c0.
#include "common.h"
#include "dev.h"
#include "small_dense.h"
#include "plane_eig.h"

namespace msp {

constexpr int E2_NT = 256;     // row kernels: a thread per unknown of a row
constexpr int E2_MAXP = 256;   // largest padded row order
constexpr int E2_SW = 512;     // sweep workgroup
constexpr int E2_CB = 16;      // columns of a Schur-complement workgroup
constexpr int E2_LB = 8;       // loads of a sweep product batch

// Coupling of unknown (X, Y, ca) with (X + dx, Y + dy, cb) in
// Ke + sigma (Me on each component) (unit-square element matrices: Ke 8 x 8
// with DOF 2 v + c, Ms 4 x 4, vertex v = sx + 2 sy), summed over the
// elements of omega's element box holding both nodes, weighted by E.
// With both set, the stiffness and mass couplings go to *k and *m.
__device__ __forceinline__ double e2_coef(const Geom& g, const Nbh3& w,
                                          const double* __restrict__ E,
                                          const double* Ke, const double* Ms,
                                          double sigma, int X, int Y, int dx, int dy,
                                          int ca, int cb, double* k, double* m) {
  double kk = 0.0, mm = 0.0;
#pragma unroll
  for (int sy = 0; sy < 2; ++sy) {
    const int oy = sy + dy, ey = Y - sy;
    if (oy < 0 || oy > 1 || ey < w.y0 || ey >= w.y0 + w.nbz - 1) continue;
#pragma unroll
    for (int sx = 0; sx < 2; ++sx) {
      const int ox = sx + dx, ex = X - sx;
      if (ox < 0 || ox > 1 || ex < w.x0 || ex >= w.x0 + w.nbx - 1) continue;
      const double kap = E[(long long)ey * g.nx + ex];
      const int va = sx + 2 * sy, vb = ox + 2 * oy;
      kk += kap * Ke[(2 * va + ca) * 8 + 2 * vb + cb];
      if (ca == cb) mm += kap * Ms[va * 4 + vb];
    }
  }
  if (k != nullptr) *k = kk;
  if (m != nullptr) *m = mm;
  return kk + sigma * mm;
}

__device__ __forceinline__ bool e2_fixed(const Geom& g, const uint8_t* __restrict__ mask,
                                         int X, int Y, int c) {
  return mask[2 * ((long long)Y * g.nnx + X) + c] != 0;
}

// Row k of every neighbourhood's block factorisation of K + sigma M:
// S_k = D_k - C_k^T G_{k-1} C_k into slot k (this workgroup's E2_CB columns
// as rows), identity on padding and on clamped DOFs; rows past the
// neighbourhood get the identity.  Grid (ldp / E2_CB, neighbourhoods).
__global__ void __launch_bounds__(E2_NT)
k2e_schur(Geom g, const Nbh3* __restrict__ nbs, int k, int ldp,
          const double* __restrict__ E, const uint8_t* __restrict__ mask,
          const double* __restrict__ Ke_g, const double* __restrict__ Ms_g,
          double sigma, double* __restrict__ G) {
  __shared__ double Ke[64], Ms[16];
  __shared__ double T[E2_MAXP * E2_CB];
  __shared__ double Cb[E2_CB * 6];
  __shared__ int Jb[E2_CB * 6];
  const Nbh3 w = nbs[blockIdx.y];
  const int tid = threadIdx.x;
  if (tid < 64) Ke[tid] = Ke_g[tid];
  if (tid < 16) Ms[tid] = Ms_g[tid];
  const long long ldp2 = (long long)ldp * ldp;
  double* Sk = G + w.goff + k * ldp2;
  const int b0 = blockIdx.x * E2_CB;
  if (k >= w.nbz) {
    for (int idx = tid; idx < E2_CB * ldp; idx += E2_NT) {
      const int t = idx / ldp, a = idx - t * ldp;
      Sk[(long long)(b0 + t) * ldp + a] = (a == b0 + t) ? 1.0 : 0.0;
    }
    return;
  }
  __syncthreads();
  const int np = w.np;
  const int Y = w.y0 + k;
  // couplings of column b (unknown of row k) with the 6 unknowns of the
  // three nodes below it in row k - 1
  if (k > 0 && tid < E2_CB * 6) {
    const int t = tid / 6, q = tid - 6 * (tid / 6);
    const int b = b0 + t;
    const int dx = q / 2 - 1, cj = q & 1;
    double c = 0.0;
    int j = -1;
    if (b < np) {
      const int bx = b >> 1, cb = b & 1;
      const int jx = bx + dx;
      if (jx >= 0 && jx < w.nbx) {
        j = 2 * jx + cj;
        const int X = w.x0 + bx;
        if (!e2_fixed(g, mask, X, Y, cb) && !e2_fixed(g, mask, X + dx, Y - 1, cj))
          c = e2_coef(g, w, E, Ke, Ms, sigma, X, Y, dx, -1, cb, cj, nullptr, nullptr);
      }
    }
    Cb[tid] = c;
    Jb[tid] = j;
  }
  __syncthreads();
  if (k > 0 && tid < ldp) {
    const double* Gp = Sk - ldp2;
    // every load of a column issued at once (an absent coupling reads row
    // 0 and weighs it by 0, which adds exactly nothing)
    for (int t = 0; t < E2_CB; ++t) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const int j = Jb[t * 6 + q];
        const double c = j >= 0 ? Cb[t * 6 + q] : 0.0;
        s = fma(Gp[(long long)max(j, 0) * ldp + tid], c, s);
      }
      T[tid * E2_CB + t] = s;
    }
  }
  __syncthreads();
  const int a = tid;
  if (a >= ldp) return;
  const bool arow = a < np;
  const int ax = a >> 1, ca = a & 1;
  bool rem = true;
  if (arow) rem = e2_fixed(g, mask, w.x0 + ax, Y, ca);
  double Din[6], Cdn[6];
  int Idn[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int dx = q / 2 - 1, cb = q & 1;
    Din[q] = 0.0;
    Cdn[q] = 0.0;
    Idn[q] = -1;
    if (arow && !rem) {
      const int nx_ = ax + dx;
      if (nx_ >= 0 && nx_ < w.nbx) {
        const int X = w.x0 + ax;
        if (!e2_fixed(g, mask, X + dx, Y, cb))
          Din[q] = e2_coef(g, w, E, Ke, Ms, sigma, X, Y, dx, 0, ca, cb, nullptr, nullptr);
        if (k > 0) {
          Idn[q] = 2 * nx_ + cb;
          if (!e2_fixed(g, mask, X + dx, Y - 1, cb))
            Cdn[q] = e2_coef(g, w, E, Ke, Ms, sigma, X, Y, dx, -1, ca, cb, nullptr, nullptr);
        }
      }
    }
  }
  for (int t = 0; t < E2_CB; ++t) {
    const int b = b0 + t;
    double v;
    if (!arow || rem || b >= np) {
      v = (a == b) ? 1.0 : 0.0;
    } else {
      const int dx = (b >> 1) - ax;
      v = (dx >= -1 && dx <= 1) ? Din[(dx + 1) * 2 + (b & 1)] : 0.0;
      if (k > 0) {
#pragma unroll
        for (int q = 0; q < 6; ++q)
          if (Idn[q] >= 0) v -= Cdn[q] * T[Idn[q] * E2_CB + t];
      }
    }
    Sk[(long long)b * ldp + a] = v;
  }
}

// X = a random start block (counter-based hash of neighbourhood, column and
// unknown), zero on clamped DOFs and padding.  Grid (rows,
// neighbourhoods), thread = unknown of the row.
__global__ void __launch_bounds__(E2_NT)
k2e_start(Geom g, const Nbh3* __restrict__ nbs, int ldp, int m,
          const uint8_t* __restrict__ mask, double* __restrict__ X) {
  const Nbh3 w = nbs[blockIdx.y];
  const int k = blockIdx.x, a = threadIdx.x;
  if (a >= ldp) return;
  double* row = X + w.xoff + ((long long)k * ldp + a) * m;
  bool live = k < w.nbz && a < w.np;
  if (live) live = !e2_fixed(g, mask, w.x0 + (a >> 1), w.y0 + k, a & 1);
  const unsigned long long u = (unsigned long long)k * w.np + a;
  for (int c = 0; c < m; ++c) {
    const unsigned long long key = ((unsigned long long)blockIdx.y << 40) ^
                                   ((unsigned long long)c << 24) ^ u;
    row[c] = live ? hash_unit(key) : 0.0;
  }
}

// Randomized start (Section 3 on the elasticity pencil, M_EE;Rand): columns
// 0..nsnap-1 uniform forcings in [-1, 1) (SplitMix64 output at the state
// key ^ (seed * gamma), key = l 2^40 + j 2^24 + u: l the neighbourhood, j
// the snapshot, u = 2 (box node, x fastest) + component the unknown's index
// in the box), zero on clamped DOFs, each made free of net force: per
// component c, f_j -= (w_c . f_j) / (w_c . 1_c) with w_c = M 1_c over the
// free DOFs; columns nsnap..nsnap+2 the rigid-body motions (the two
// translations, the rotation about the coarse node scaled by 1/H), zero on
// clamped DOFs; the remaining columns and the padding zero.  Also zeroes
// the Rayleigh-Ritz coefficients, so that the columns past the live ones
// stay zero.  T's first column holds w as scratch.  One workgroup per
// neighbourhood.
__global__ void __launch_bounds__(E2_NT)
k2e_rand_start(Geom g, const Nbh3* __restrict__ nbs, int pmax, int ldp, int m, int nsnap,
               unsigned int seed, double invH, const double* __restrict__ E,
               const uint8_t* __restrict__ mask, const double* __restrict__ Ke_g,
               const double* __restrict__ Ms_g, double* __restrict__ X,
               double* __restrict__ T, Eig3State* __restrict__ st) {
  __shared__ double Ke[64], Ms[16];
  __shared__ double red[2 * (E2_NT / 64)];
  const Nbh3 w = nbs[blockIdx.x];
  const int tid = threadIdx.x;
  if (tid < 64) Ke[tid] = Ke_g[tid];
  if (tid < 16) Ms[tid] = Ms_g[tid];
  Eig3State& es = st[blockIdx.x];
  for (int e = tid; e < MAXM * MAXM; e += E2_NT) es.V[e] = 0.0;
  for (int idx = tid; idx < pmax * ldp; idx += E2_NT) {
    const int k = idx / ldp, a = idx - (idx / ldp) * ldp;
    double* row = X + w.xoff + (long long)idx * m;
    if (k < w.nbz && a < w.np) {
      for (int c = nsnap + 3; c < m; ++c) row[c] = 0.0;
    } else {
      for (int c = 0; c < m; ++c) row[c] = 0.0;
    }
  }
  __syncthreads();
  const int nu = w.nbz * w.np;
  double w0 = 0.0, w1 = 0.0;
  for (int u = tid; u < nu; u += E2_NT) {
    const int k = u / w.np, a = u - (u / w.np) * w.np;
    const int ax = a >> 1, ca = a & 1;
    const int Xn = w.x0 + ax, Yn = w.y0 + k;
    const bool live = !e2_fixed(g, mask, Xn, Yn, ca);
    double wi = 0.0;
    if (live) {
      for (int dy = -1; dy <= 1; ++dy) {
        if (k + dy < 0 || k + dy >= w.nbz) continue;
        for (int dx = -1; dx <= 1; ++dx) {
          if (ax + dx < 0 || ax + dx >= w.nbx) continue;
          if (e2_fixed(g, mask, Xn + dx, Yn + dy, ca)) continue;
          double cK, cM;
          (void)e2_coef(g, w, E, Ke, Ms, 0.0, Xn, Yn, dx, dy, ca, ca, &cK, &cM);
          wi += cM;
        }
      }
    }
    double* row = X + w.xoff + ((long long)k * ldp + a) * m;
    T[w.xoff + ((long long)k * ldp + a) * m] = wi;
    if (ca) w1 += wi; else w0 += wi;
    const double rx = (double)(Xn - w.cx * g.sx) * g.h * invH;
    const double ry = (double)(Yn - w.cy * g.sy) * g.h * invH;
    row[nsnap] = (live && ca == 0) ? 1.0 : 0.0;
    row[nsnap + 1] = (live && ca == 1) ? 1.0 : 0.0;
    row[nsnap + 2] = live ? (ca == 0 ? -ry : rx) : 0.0;
  }
  const double2 W = block_sum2<E2_NT>(w0, w1, red);
  const unsigned long long sg = (unsigned long long)seed * 0x9E3779B97F4A7C15ull;
  for (int j = 0; j < nsnap; ++j) {
    double s0 = 0.0, s1 = 0.0;
    for (int u = tid; u < nu; u += E2_NT) {
      const int k = u / w.np, a = u - (u / w.np) * w.np;
      const int ca = a & 1;
      const long long o = w.xoff + ((long long)k * ldp + a) * m;
      double f = 0.0;
      if (!e2_fixed(g, mask, w.x0 + (a >> 1), w.y0 + k, ca)) {
        const unsigned long long key = ((unsigned long long)blockIdx.x << 40) |
                                       ((unsigned long long)j << 24) |
                                       (unsigned long long)u;
        f = hash_unit(key ^ sg);
      }
      X[o + j] = f;
      const double wf = T[o] * f;
      if (ca) s1 += wf; else s0 += wf;
    }
    const double2 S = block_sum2<E2_NT>(s0, s1, red);
    const double m0 = W.x > 0.0 ? S.x / W.x : 0.0;
    const double m1 = W.y > 0.0 ? S.y / W.y : 0.0;
    for (int u = tid; u < nu; u += E2_NT) {
      const int k = u / w.np, a = u - (u / w.np) * w.np;
      const int ca = a & 1;
      if (e2_fixed(g, mask, w.x0 + (a >> 1), w.y0 + k, ca)) continue;
      X[w.xoff + ((long long)k * ldp + a) * m + j] -= ca ? m1 : m0;
    }
  }
}

// Y's columns [c0, c1) := X's on every row of the box (rows past the
// neighbourhood included).  Grid (rows, neighbourhoods).
__global__ void __launch_bounds__(E2_NT)
k2e_copy_cols(const Nbh3* __restrict__ nbs, int ldp, int m, int c0, int c1,
              const double* __restrict__ X, double* __restrict__ Y) {
  const Nbh3 w = nbs[blockIdx.y];
  const int a = threadIdx.x;
  if (a >= ldp) return;
  const long long o = w.xoff + ((long long)blockIdx.x * ldp + a) * m;
  for (int c = c0; c < c1; ++c) Y[o + c] = X[o + c];
}

// OutM = M Y, and with BOTH also OutK = K Y, on row k of every unfinished
// neighbourhood (the 9 neighbouring nodes, both components; clamped DOFs:
// zero rows).
template <int M, bool BOTH>
__global__ void __launch_bounds__(E2_NT)
k2e_stencil(Geom g, const Nbh3* __restrict__ nbs, int ldp,
            const double* __restrict__ E, const uint8_t* __restrict__ mask,
            const double* __restrict__ Ke_g, const double* __restrict__ Ms_g,
            const double* __restrict__ Yw, double* __restrict__ OutK,
            double* __restrict__ OutM, const Eig3State* __restrict__ st) {
  __shared__ double Ke[64], Ms[16];
  if (st[blockIdx.y].done) return;
  const Nbh3 w = nbs[blockIdx.y];
  const int k = blockIdx.x, a = threadIdx.x;
  if (a < 64) Ke[a] = Ke_g[a];
  if (a < 16) Ms[a] = Ms_g[a];
  __syncthreads();
  if (k >= w.nbz || a >= ldp) return;
  const long long ro = w.xoff + ((long long)k * ldp + a) * M;
  double ok[M], om[M];
#pragma unroll
  for (int c = 0; c < M; ++c) {
    ok[c] = 0.0;
    om[c] = 0.0;
  }
  const int ax = a >> 1, ca = a & 1;
  bool live = a < w.np;
  if (live) live = !e2_fixed(g, mask, w.x0 + ax, w.y0 + k, ca);
  if (live) {
    const int X = w.x0 + ax, Y = w.y0 + k;
    for (int dy = -1; dy <= 1; ++dy) {
      if (k + dy < 0 || k + dy >= w.nbz) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        if (ax + dx < 0 || ax + dx >= w.nbx) continue;
        for (int cb = 0; cb < 2; ++cb) {
          if (e2_fixed(g, mask, X + dx, Y + dy, cb)) continue;
          double cK = 0.0, cM = 0.0;
          (void)e2_coef(g, w, E, Ke, Ms, 0.0, X, Y, dx, dy, ca, cb, &cK, &cM);
          const double* yr = Yw + w.xoff +
                             ((long long)(k + dy) * ldp + 2 * (ax + dx) + cb) * M;
#pragma unroll
          for (int c = 0; c < M; ++c) {
            const double y = yr[c];
            om[c] = fma(cM, y, om[c]);
            if (BOTH) ok[c] = fma(cK, y, ok[c]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < M; ++c) {
    OutM[ro + c] = om[c];
    if (BOTH) OutK[ro + c] = ok[c];
  }
}

// Y = (K + sigma M)^{-1} B by rows, forward and backward (the structure of
// the 3D heat sweep: y_k = G_k (b_k - C_k^T y_{k-1}), x_k = y_k - G_k
// C_{k+1} x_{k+1}).  One workgroup per unfinished neighbourhood; thread
// (i, h) forms row i of the row block's product over half h of the inner
// index.
template <int M>
__global__ void __launch_bounds__(E2_SW)
k2e_sweep(Geom g, const Nbh3* __restrict__ nbs, int ldp,
          const double* __restrict__ E, const uint8_t* __restrict__ mask,
          const double* __restrict__ Ke_g, const double* __restrict__ Ms_g,
          double sigma, const double* __restrict__ G, const double* __restrict__ B,
          double* __restrict__ Yw, const Eig3State* __restrict__ st) {
  __shared__ double Ke[64], Ms[16];
  __shared__ double R[E2_MAXP * M];
  __shared__ double P[E2_MAXP * M];
  if (st[blockIdx.x].done) return;
  const Nbh3 w = nbs[blockIdx.x];
  const int tid = threadIdx.x;
  const int i = tid & (E2_MAXP - 1), hh = tid / E2_MAXP;
  if (tid < 64) Ke[tid] = Ke_g[tid];
  if (tid < 16) Ms[tid] = Ms_g[tid];
  const long long ldp2 = (long long)ldp * ldp;
  const int np = w.np;
  // rows and inner indices past the row's unknowns are padding (identity
  // rows of G_k on zero right-hand sides): neither half reads them
  const int half = (np + 1) / 2, kk0 = hh * half, kk1 = min(np, kk0 + half);
  const int ax = tid >> 1, ca = tid & 1;
  __syncthreads();
  auto gemm = [&](int k, double (&acc)[M]) {
#pragma unroll
    for (int c = 0; c < M; ++c) acc[c] = 0.0;
    if (i >= np) return;
    const double* Gk = G + w.goff + k * ldp2 + i;
    // the column's loads in batches of E2_LB, all of a batch issued first
    for (int kb = kk0; kb < kk1; kb += E2_LB) {
      double gv[E2_LB];
#pragma unroll
      for (int u = 0; u < E2_LB; ++u) gv[u] = Gk[(long long)min(kb + u, kk1 - 1) * ldp];
#pragma unroll
      for (int u = 0; u < E2_LB; ++u) {
        if (kb + u < kk1) {
          const double* rr = R + (kb + u) * M;
#pragma unroll
          for (int c = 0; c < M; ++c) acc[c] = fma(gv[u], rr[c], acc[c]);
        }
      }
    }
  };
  // coupling of unknown tid (row k) with unknown q of the three nodes in
  // row k + dy
  auto couple = [&](int k, int dy, int q, int* nb_) -> double {
    const int dx = q / 2 - 1, cb = q & 1;
    const int jx = ax + dx;
    *nb_ = -1;
    if (jx < 0 || jx >= w.nbx) return 0.0;
    const int X = w.x0 + ax, Y = w.y0 + k;
    if (e2_fixed(g, mask, X, Y, ca) || e2_fixed(g, mask, X + dx, Y + dy, cb)) return 0.0;
    *nb_ = 2 * jx + cb;
    return e2_coef(g, w, E, Ke, Ms, sigma, X, Y, dx, dy, ca, cb, nullptr, nullptr);
  };
  double acc[M];
  for (int k = 0; k < w.nbz; ++k) {
    if (tid < ldp) {
      double r[M];
      const double* br = B + w.xoff + ((long long)k * ldp + tid) * M;
#pragma unroll
      for (int c = 0; c < M; ++c) r[c] = tid < np ? br[c] : 0.0;
      if (k > 0 && tid < np) {
        for (int q = 0; q < 6; ++q) {
          int j;
          const double cf = couple(k, -1, q, &j);
          if (j < 0 || cf == 0.0) continue;
#pragma unroll
          for (int c = 0; c < M; ++c) r[c] = fma(-cf, P[j * M + c], r[c]);
        }
      }
#pragma unroll
      for (int c = 0; c < M; ++c) R[tid * M + c] = r[c];
    }
    __syncthreads();
    gemm(k, acc);
    __syncthreads();
    if (hh == 1 && i < ldp) {
#pragma unroll
      for (int c = 0; c < M; ++c) R[i * M + c] = acc[c];
    }
    __syncthreads();
    if (hh == 0 && i < ldp) {
      double* yr = Yw + w.xoff + ((long long)k * ldp + i) * M;
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const double y = acc[c] + R[i * M + c];
        yr[c] = y;
        P[i * M + c] = y;
      }
    }
    __syncthreads();
  }
  for (int k = w.nbz - 2; k >= 0; --k) {
    if (tid < ldp) {
      double v[M];
#pragma unroll
      for (int c = 0; c < M; ++c) v[c] = 0.0;
      if (tid < np) {
        for (int q = 0; q < 6; ++q) {
          int j;
          const double cf = couple(k, 1, q, &j);
          if (j < 0 || cf == 0.0) continue;
#pragma unroll
          for (int c = 0; c < M; ++c) v[c] = fma(cf, P[j * M + c], v[c]);
        }
      }
#pragma unroll
      for (int c = 0; c < M; ++c) R[tid * M + c] = v[c];
    }
    __syncthreads();
    gemm(k, acc);
    __syncthreads();
    if (hh == 1 && i < ldp) {
#pragma unroll
      for (int c = 0; c < M; ++c) R[i * M + c] = acc[c];
    }
    __syncthreads();
    if (hh == 0 && i < ldp) {
      double* yr = Yw + w.xoff + ((long long)k * ldp + i) * M;
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const double x = yr[c] - (acc[c] + R[i * M + c]);
        yr[c] = x;
        P[i * M + c] = x;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------
// Dense coarse operator

// Phi (column-major, n rows): column col of coarse node l = chi_l times
// mode j (psi compact: unknown u = k np + a of the box, nmodes values each),
// zero outside the box and at clamped DOFs.  Grid (node blocks, columns).
__global__ void __launch_bounds__(256)
k2e_basis(Geom g, const Nbh3* __restrict__ nbs, const int* __restrict__ col_node,
          const uint8_t* __restrict__ mask, const double* __restrict__ psi,
          double* __restrict__ Phi) {
  const long long nn = (long long)g.nnx * g.nny;
  const long long node = (long long)blockIdx.x * 256 + threadIdx.x;
  if (node >= nn) return;
  const int col = blockIdx.y;
  const Nbh3 w = nbs[col_node[col]];
  const int j = col - w.col0;
  const int X = (int)(node % g.nnx), Y = (int)(node / g.nnx);
  double v0 = 0.0, v1 = 0.0;
  if (X >= w.x0 && X < w.x0 + w.nbx && Y >= w.y0 && Y < w.y0 + w.nbz) {
    const int dx = X - w.cx * g.sx, dy = Y - w.cy * g.sy;
    const double chi = (1.0 - fabs((double)dx) / g.sx) * (1.0 - fabs((double)dy) / g.sy);
    if (chi > 0.0) {
      const long long u = (long long)(Y - w.y0) * w.np + 2 * (X - w.x0);
      v0 = mask[2 * node] ? 0.0 : chi * psi[w.psi_off + u * w.nmodes + j];
      v1 = mask[2 * node + 1] ? 0.0 : chi * psi[w.psi_off + (u + 1) * w.nmodes + j];
    }
  }
  double* o = Phi + (long long)col * 2 * nn + 2 * node;
  o[0] = v0;
  o[1] = v1;
}

// K_0 = Phi^T W (W = K Phi), 16 x 16 tiles: the tile's 16 + 16 columns
// staged in LDS 64 rows at a time; thread (i, j) sums its entry in row
// order.  Grid (tiles in b, tiles in a).
__global__ void __launch_bounds__(256)
k2e_k0(const double* __restrict__ Phi, const double* __restrict__ W, long long n, int nc,
       double* __restrict__ K0, int ldk) {
  __shared__ double A[16][65], Bt[16][65];
  const int a0 = blockIdx.y * 16, b0 = blockIdx.x * 16;
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  double acc = 0.0;
  for (long long r0 = 0; r0 < n; r0 += 64) {
    for (int idx = tid; idx < 16 * 64; idx += 256) {
      const int c = idx >> 6, r = idx & 63;
      const long long row = r0 + r;
      A[c][r] = (a0 + c < nc && row < n) ? Phi[(long long)(a0 + c) * n + row] : 0.0;
      Bt[c][r] = (b0 + c < nc && row < n) ? W[(long long)(b0 + c) * n + row] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int r = 0; r < 64; ++r) acc = fma(A[ti][r], Bt[tj][r], acc);
    __syncthreads();
  }
  if (a0 + ti < nc && b0 + tj < nc) K0[(long long)(a0 + ti) * ldk + b0 + tj] = acc;
}

// c = Phi^T r into band 0 of the restriction's partials: one workgroup per
// column, fixed-order sums.
__global__ void __launch_bounds__(256)
k2e_restrict(const double* __restrict__ Phi, long long n, const double* __restrict__ r,
             double* __restrict__ c, const CGScalars* __restrict__ sc) {
  __shared__ double red[256 / 64 + 1];
  __shared__ int shd;
  if (sc != nullptr && block_read_done(sc, &shd)) return;
  const double* ph = Phi + (long long)blockIdx.x * n;
  double s = 0.0;
  for (long long i = threadIdx.x; i < n; i += 256) s = fma(ph[i], r[i], s);
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) c[blockIdx.x] = s;
}

// z = Phi c0 (thread per DOF; columns in order).
__global__ void __launch_bounds__(256)
k2e_prolong(const double* __restrict__ Phi, long long n, int nc,
            const double* __restrict__ c0, double* __restrict__ z,
            const CGScalars* __restrict__ sc) {
  __shared__ int shd;
  if (sc != nullptr && block_read_done(sc, &shd)) return;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < nc; ++j) s = fma(Phi[(long long)j * n + i], c0[j], s);
  z[i] = s;
}

// ---------------------------------------------------------------- launchers

void launch_local_inverse3_strided(double*, int, int, long long, double*, double*,
                                   double*, double*, int*, float*, hipStream_t);

int ee2_max_row() { return E2_MAXP; }

void launch_ee2_factor(const Geom& g, const Nbh3* nbs, int nnb, int pmax, int ldp,
                       const double* E, const uint8_t* mask, const double* Ke,
                       const double* Ms, double sigma, double* G, double* sdiag,
                       double* LD, double* Lp, double* Rp, int* dropped, hipStream_t s) {
  const long long ldp2 = (long long)ldp * ldp;
  for (int k = 0; k < pmax; ++k) {
    hipLaunchKernelGGL(k2e_schur, dim3(ldp / E2_CB, nnb), dim3(E2_NT), 0, s, g, nbs, k,
                       ldp, E, mask, Ke, Ms, sigma, G);
    launch_local_inverse3_strided(G + k * ldp2, ldp, nnb, pmax * ldp2, sdiag, LD, Lp, Rp,
                                  dropped, nullptr, s);
  }
}

void launch_ee2_start(const Geom& g, const Nbh3* nbs, int nnb, int pmax, int ldp, int m,
                      const uint8_t* mask, double* X, hipStream_t s) {
  hipLaunchKernelGGL(k2e_start, dim3(pmax, nnb), dim3(E2_NT), 0, s, g, nbs, ldp, m, mask, X);
}

// The products of one sweep of the subspace iteration: T = M X, Y = (K +
// sigma M)^{-1} T, then T = K Y and U = M Y for the Rayleigh-Ritz step.
template <int M>
static void ee2_products_m(const Geom& g, const Nbh3* nbs, int nnb, int pmax, int ldp,
                           const double* E, const uint8_t* mask, const double* Ke,
                           const double* Ms, double sigma, const double* G,
                           const double* X, double* Y, double* T, double* U,
                           const Eig3State* st, hipStream_t s) {
  hipLaunchKernelGGL((k2e_stencil<M, false>), dim3(pmax, nnb), dim3(E2_NT), 0, s, g, nbs,
                     ldp, E, mask, Ke, Ms, X, (double*)nullptr, T, st);
  hipLaunchKernelGGL((k2e_sweep<M>), dim3(nnb), dim3(E2_SW), 0, s, g, nbs, ldp, E, mask,
                     Ke, Ms, sigma, G, T, Y, st);
  hipLaunchKernelGGL((k2e_stencil<M, true>), dim3(pmax, nnb), dim3(E2_NT), 0, s, g, nbs,
                     ldp, E, mask, Ke, Ms, Y, T, U, st);
}

void launch_ee2_products(int m, const Geom& g, const Nbh3* nbs, int nnb, int pmax,
                         int ldp, const double* E, const uint8_t* mask, const double* Ke,
                         const double* Ms, double sigma, const double* G, const double* X,
                         double* Y, double* T, double* U, const void* st, hipStream_t s) {
  const Eig3State* es = (const Eig3State*)st;
  switch (m) {
    case 8: ee2_products_m<8>(g, nbs, nnb, pmax, ldp, E, mask, Ke, Ms, sigma, G, X, Y, T, U, es, s); break;
    case 16: ee2_products_m<16>(g, nbs, nnb, pmax, ldp, E, mask, Ke, Ms, sigma, G, X, Y, T, U, es, s); break;
    case 24: ee2_products_m<24>(g, nbs, nnb, pmax, ldp, E, mask, Ke, Ms, sigma, G, X, Y, T, U, es, s); break;
    default: ee2_products_m<32>(g, nbs, nnb, pmax, ldp, E, mask, Ke, Ms, sigma, G, X, Y, T, U, es, s); break;
  }
}

// The randomized setup's products: the start block (forcings made free of
// net force, the rigid-body motions), T = M X, Y = (K + sigma M)^{-1} T on
// every column, the motions copied back over their solved columns (W =
// span{u_j} + span{rigid-body motions}), then T = K Y and U = M Y for the
// Rayleigh-Ritz step on the nsnap + 3 live columns.
template <int M>
static void ee2_rand_m(const Geom& g, const Nbh3* nbs, int nnb, int pmax, int ldp,
                       int nsnap, unsigned int seed, double invH, const double* E,
                       const uint8_t* mask, const double* Ke, const double* Ms,
                       double sigma, const double* G, double* X, double* Y, double* T,
                       double* U, Eig3State* st, hipStream_t s) {
  hipLaunchKernelGGL(k2e_rand_start, dim3(nnb), dim3(E2_NT), 0, s, g, nbs, pmax, ldp, M,
                     nsnap, seed, invH, E, mask, Ke, Ms, X, T, st);
  hipLaunchKernelGGL((k2e_stencil<M, false>), dim3(pmax, nnb), dim3(E2_NT), 0, s, g, nbs,
                     ldp, E, mask, Ke, Ms, X, (double*)nullptr, T, st);
  hipLaunchKernelGGL((k2e_sweep<M>), dim3(nnb), dim3(E2_SW), 0, s, g, nbs, ldp, E, mask,
                     Ke, Ms, sigma, G, T, Y, st);
  hipLaunchKernelGGL(k2e_copy_cols, dim3(pmax, nnb), dim3(E2_NT), 0, s, nbs, ldp, M,
                     nsnap, nsnap + 3, X, Y);
  hipLaunchKernelGGL((k2e_stencil<M, true>), dim3(pmax, nnb), dim3(E2_NT), 0, s, g, nbs,
                     ldp, E, mask, Ke, Ms, Y, T, U, st);
}

void launch_ee2_rand(int m, int nsnap, unsigned int seed, double invH, const Geom& g,
                     const Nbh3* nbs, int nnb, int pmax, int ldp, const double* E,
                     const uint8_t* mask, const double* Ke, const double* Ms, double sigma,
                     const double* G, double* X, double* Y, double* T, double* U, void* st,
                     hipStream_t s) {
  Eig3State* es = (Eig3State*)st;
  switch (m) {
    case 8: ee2_rand_m<8>(g, nbs, nnb, pmax, ldp, nsnap, seed, invH, E, mask, Ke, Ms, sigma, G, X, Y, T, U, es, s); break;
    case 16: ee2_rand_m<16>(g, nbs, nnb, pmax, ldp, nsnap, seed, invH, E, mask, Ke, Ms, sigma, G, X, Y, T, U, es, s); break;
    case 24: ee2_rand_m<24>(g, nbs, nnb, pmax, ldp, nsnap, seed, invH, E, mask, Ke, Ms, sigma, G, X, Y, T, U, es, s); break;
    default: ee2_rand_m<32>(g, nbs, nnb, pmax, ldp, nsnap, seed, invH, E, mask, Ke, Ms, sigma, G, X, Y, T, U, es, s); break;
  }
}

void launch_ee2_basis(const Geom& g, const Nbh3* nbs, const int* col_node, int nc,
                      const uint8_t* mask, const double* psi, double* Phi, hipStream_t s) {
  if (nc <= 0) return;
  const long long nn = (long long)g.nnx * g.nny;
  hipLaunchKernelGGL(k2e_basis, dim3((unsigned)((nn + 255) / 256), nc), dim3(256), 0, s,
                     g, nbs, col_node, mask, psi, Phi);
}

void launch_ee2_k0(const double* Phi, const double* W, long long n, int nc, double* K0,
                   int ldk, hipStream_t s) {
  if (nc <= 0) return;
  const int nt = (nc + 15) / 16;
  hipLaunchKernelGGL(k2e_k0, dim3(nt, nt), dim3(256), 0, s, Phi, W, n, nc, K0, ldk);
}

void launch_ee2_restrict(const double* Phi, long long n, int nc, const double* r,
                         double* c, const CGScalars* sc, hipStream_t s) {
  if (nc <= 0) return;
  hipLaunchKernelGGL(k2e_restrict, dim3(nc), dim3(256), 0, s, Phi, n, r, c, sc);
}

void launch_ee2_prolong(const double* Phi, long long n, int nc, const double* c0,
                        double* z, const CGScalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(k2e_prolong, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Phi,
                     n, nc, c0, z, sc);
}

}  // namespace msp
