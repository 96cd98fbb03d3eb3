// Local systems on node boxes: block-tridiagonal LDL^T factorisation with
// explicit inverse Schur blocks, the first-level apply of the additive
// Schwarz preconditioner, and the heat eigenproblems of the coarse space.
//
// A box of nxb x nyb nodes ordered row by row gives a block-tridiagonal
// matrix with nyb diagonal blocks D_k (one node row, bs = ndof*nxb DOFs)
// and couplings B_k between rows k+1 and k.  With S_0 = D_0 and
// S_{k+1} = D_{k+1} - B_k S_k^{-1} B_k^T, a solve is
//   forward  t_k = S_k^{-1} (r_k - B_{k-1} t_{k-1})
//   backward x_k = t_k - S_k^{-1} B_k^T x_{k+1}.
// Only the blocks S_k^{-1} are stored; B_k is rebuilt from the element
// moduli on the fly, so one solve reads 2 * nyb * bs^2 stored values.
// Clamped (Dirichlet) DOFs become identity rows with zero couplings, which
// keeps the principal submatrix of the free DOFs exact.
#include "common.h"
#include "dev.h"

namespace msp {

constexpr int FT_NT = 256;    // factorisation workgroup
constexpr int AP_NT = 512;    // first-level apply workgroup
constexpr int EG_NT = 512;    // eigen workgroup
constexpr int LDSTR = MAXBS + 1;   // LDS row stride of a dense block

// K entry between DOF (xa,ya,ca) and DOF (xb,yb,cb): sum over the elements
// of the system's element box that contain both nodes.
template <int NDOF>
__device__ __forceinline__ double coupling(const Geom& g, const SysDesc& s,
                                           const double* __restrict__ E,
                                           const double* __restrict__ Kel,
                                           int xa, int ya, int ca, int xb,
                                           int yb, int cb) {
  const int exlo = max(max(xa, xb) - 1, s.ex0);
  const int exhi = min(min(xa, xb), s.ex1 - 1);
  const int eylo = max(max(ya, yb) - 1, s.ey0);
  const int eyhi = min(min(ya, yb), s.ey1 - 1);
  double v = 0.0;
  for (int ey = eylo; ey <= eyhi; ++ey)
    for (int ex = exlo; ex <= exhi; ++ex) {
      const int va = (xa - ex) + 2 * (ya - ey);
      const int vb = (xb - ex) + 2 * (yb - ey);
      v += E[(long long)ey * g.nx + ex] *
           Kel[(NDOF * va + ca) * (4 * NDOF) + NDOF * vb + cb];
    }
  return v;
}

template <int NDOF>
__device__ __forceinline__ bool is_fixed(const Geom& g,
                                         const uint8_t* __restrict__ flag,
                                         int x, int y, int c) {
  const long long node = (long long)y * g.nnx + x;
  return flag[NDOF * node + c] != 0;
}

// In-place Gauss-Jordan inversion of an SPD block in LDS (no pivoting is
// needed for SPD matrices).  rowv/colv: scratch vectors of MAXBS.
template <int NT>
__device__ void gj_invert(double* S, int bs, double* rowv, double* colv,
                          int* __restrict__ err) {
  const int tid = threadIdx.x;
  for (int p = 0; p < bs; ++p) {
    for (int i = tid; i < bs; i += NT) {
      colv[i] = S[i * LDSTR + p];
      rowv[i] = S[p * LDSTR + i];
    }
    __syncthreads();
    double piv = colv[p];
    if (!(piv > 0.0) || !finite(piv)) {
      if (tid == 0) atomicOr(err, ERR_NOT_SPD);
      piv = 1.0;
    }
    const double ip = 1.0 / piv;
    for (int idx = tid; idx < bs * bs; idx += NT) {
      const int i = idx / bs, j = idx - (idx / bs) * bs;
      double v;
      if (i == p) v = (j == p) ? ip : rowv[j] * ip;
      else if (j == p) v = -colv[i] * ip;
      else v = S[i * LDSTR + j] - colv[i] * rowv[j] * ip;
      S[i * LDSTR + j] = v;
    }
    __syncthreads();
  }
}

// Factorise every system: one workgroup per system.  TOUT is double (FP64
// local solves) or float (inverse blocks rounded for the FP32 path).
template <int NDOF, typename TOUT>
__global__ void __launch_bounds__(FT_NT)
k_factor(Geom g, const SysDesc* __restrict__ systems,
         const double* __restrict__ E, const uint8_t* __restrict__ flag,
         const double* __restrict__ Kel, TOUT* __restrict__ out,
         int* __restrict__ err) {
  __shared__ double buf[3][MAXBS * LDSTR];
  __shared__ double Bv[MAXBS * 3 * NDOF];
  __shared__ double rowv[MAXBS], colv[MAXBS];
  const SysDesc s = systems[blockIdx.x];
  const int tid = threadIdx.x;
  const int bs = NDOF * s.nxb;
  int cur = 0, prev = 1, wb = 2;
  for (int k = 0; k < s.nyb; ++k) {
    const int y = s.y0 + k;
    double* S = buf[cur];
    // D_k
    for (int idx = tid; idx < bs * bs; idx += FT_NT) {
      const int a = idx / bs, b = idx - (idx / bs) * bs;
      const int ia = a / NDOF, ca = a - ia * NDOF;
      const int ib = b / NDOF, cb = b - ib * NDOF;
      double v = 0.0;
      const bool fa = is_fixed<NDOF>(g, flag, s.x0 + ia, y, ca);
      const bool fb = is_fixed<NDOF>(g, flag, s.x0 + ib, y, cb);
      if (fa || fb) {
        v = (a == b) ? 1.0 : 0.0;
      } else if (abs(ia - ib) <= 1) {
        v = coupling<NDOF>(g, s, E, Kel, s.x0 + ia, y, ca, s.x0 + ib, y, cb);
      }
      S[a * LDSTR + b] = v;
    }
    if (k > 0) {
      // B_{k-1}: rows a in node row y, columns in node row y-1, banded
      for (int idx = tid; idx < bs * 3 * NDOF; idx += FT_NT) {
        const int a = idx / (3 * NDOF), t = idx - a * (3 * NDOF);
        const int ia = a / NDOF, ca = a - ia * NDOF;
        const int di = t / NDOF - 1, cb = t - (t / NDOF) * NDOF;
        const int ib = ia + di;
        double v = 0.0;
        if (ib >= 0 && ib < s.nxb &&
            !is_fixed<NDOF>(g, flag, s.x0 + ia, y, ca) &&
            !is_fixed<NDOF>(g, flag, s.x0 + ib, y - 1, cb))
          v = coupling<NDOF>(g, s, E, Kel, s.x0 + ia, y, ca, s.x0 + ib, y - 1, cb);
        Bv[idx] = v;
      }
      __syncthreads();
      // W = S_{k-1}^{-1} B_{k-1}^T : W[b][a]
      const double* P = buf[prev];
      double* W = buf[wb];
      for (int idx = tid; idx < bs * bs; idx += FT_NT) {
        const int b = idx / bs, a = idx - (idx / bs) * bs;
        const int ia = a / NDOF;
        double v = 0.0;
#pragma unroll
        for (int t = 0; t < 3 * NDOF; ++t) {
          const int col = NDOF * (ia + t / NDOF - 1) + (t % NDOF);
          if (col >= 0 && col < bs) v += P[b * LDSTR + col] * Bv[a * 3 * NDOF + t];
        }
        W[b * LDSTR + a] = v;
      }
      __syncthreads();
      // S -= B W
      for (int idx = tid; idx < bs * bs; idx += FT_NT) {
        const int a = idx / bs, a2 = idx - (idx / bs) * bs;
        const int ia = a / NDOF;
        double v = 0.0;
#pragma unroll
        for (int t = 0; t < 3 * NDOF; ++t) {
          const int row = NDOF * (ia + t / NDOF - 1) + (t % NDOF);
          if (row >= 0 && row < bs) v += Bv[a * 3 * NDOF + t] * W[row * LDSTR + a2];
        }
        S[a * LDSTR + a2] -= v;
      }
    }
    __syncthreads();
    gj_invert<FT_NT>(S, bs, rowv, colv, err);
    TOUT* o = out + s.foff + (long long)k * bs * bs;
    for (int idx = tid; idx < bs * bs; idx += FT_NT) {
      const int j = idx / bs, i = idx - (idx / bs) * bs;
      o[idx] = (TOUT)S[i * LDSTR + j];      // column j contiguous
    }
    __syncthreads();
    const int t = prev;
    prev = cur;
    cur = t;
  }
}

// ---------------------------------------------------------------------
// First level: z_i = K_i^{-1} R_i r for every subdomain (2D elasticity).
// One workgroup per subdomain; the local vector stays in LDS.  Threads are
// grouped NG = AP_NT / bs ways over the columns of each inverse block; a
// group's lanes read consecutive entries of a column (coalesced).
template <typename T>
__global__ void __launch_bounds__(AP_NT)
k_level1(Geom g, const SysDesc* __restrict__ systems,
         const double* __restrict__ E, const uint8_t* __restrict__ mask,
         const double* __restrict__ Kel, const T* __restrict__ Sinv,
         const double* __restrict__ r, T* __restrict__ lsol,
         const CGScalars* __restrict__ sc) {
  __shared__ T v[MAXBS * 40];          // whole local vector (nyb*bs <= 2880)
  __shared__ T tmp[MAXBS];
  __shared__ T part[AP_NT];
  __shared__ double Bc[MAXBS * 6];     // coupling coefficients of one row
  if (sc != nullptr && sc->done) return;
  const SysDesc s = systems[blockIdx.x];
  const int tid = threadIdx.x;
  const int bs = 2 * s.nxb;
  const int nb = s.nyb;
  const int NG = AP_NT / bs;
  const int grp = tid / bs, li = tid - (tid / bs) * bs;

  for (int idx = tid; idx < nb * bs; idx += AP_NT) {
    const int k = idx / bs, a = idx - (idx / bs) * bs;
    const int x = s.x0 + a / 2, y = s.y0 + k, c = a & 1;
    const long long d = 2 * ((long long)y * g.nnx + x) + c;
    v[idx] = mask[d] ? (T)0 : (T)r[d];
  }
  __syncthreads();

  // forward sweep
  for (int k = 0; k < nb; ++k) {
    const int y = s.y0 + k;
    if (k > 0) {
      // coupling of row y (a) with row y-1 (i + di)
      for (int idx = tid; idx < bs * 6; idx += AP_NT) {
        const int a = idx / 6, t = idx - a * 6;
        const int ia = a >> 1, ca = a & 1;
        const int ib = ia + t / 2 - 1, cb = t & 1;
        double cv = 0.0;
        if (ib >= 0 && ib < s.nxb && !mask[2 * ((long long)y * g.nnx + s.x0 + ia) + ca] &&
            !mask[2 * ((long long)(y - 1) * g.nnx + s.x0 + ib) + cb])
          cv = coupling<2>(g, s, E, Kel, s.x0 + ia, y, ca, s.x0 + ib, y - 1, cb);
        Bc[idx] = cv;
      }
      __syncthreads();
      for (int a = tid; a < bs; a += AP_NT) {
        const int ia = a >> 1;
        T acc = v[k * bs + a];
#pragma unroll
        for (int t = 0; t < 6; ++t) {
          const int col = 2 * (ia + t / 2 - 1) + (t & 1);
          if (col >= 0 && col < bs) acc -= (T)Bc[a * 6 + t] * v[(k - 1) * bs + col];
        }
        tmp[a] = acc;
      }
    } else {
      for (int a = tid; a < bs; a += AP_NT) tmp[a] = v[a];
    }
    __syncthreads();
    const T* Sk = Sinv + s.foff + (long long)k * bs * bs;
    if (grp < NG) {
      T acc = 0;
      for (int j = grp; j < bs; j += NG) acc += Sk[(long long)j * bs + li] * tmp[j];
      part[grp * bs + li] = acc;
    }
    __syncthreads();
    for (int a = tid; a < bs; a += AP_NT) {
      T acc = 0;
      for (int q = 0; q < NG; ++q) acc += part[q * bs + a];
      v[k * bs + a] = acc;
    }
    __syncthreads();
  }
  // backward sweep
  for (int k = nb - 2; k >= 0; --k) {
    const int y = s.y0 + k;
    // (B_k^T x_{k+1})[b], b in row y, neighbours (i+di) in row y+1
    for (int idx = tid; idx < bs * 6; idx += AP_NT) {
      const int b = idx / 6, t = idx - b * 6;
      const int ib = b >> 1, cb = b & 1;
      const int ia = ib + t / 2 - 1, ca = t & 1;
      double cv = 0.0;
      if (ia >= 0 && ia < s.nxb && !mask[2 * ((long long)y * g.nnx + s.x0 + ib) + cb] &&
          !mask[2 * ((long long)(y + 1) * g.nnx + s.x0 + ia) + ca])
        cv = coupling<2>(g, s, E, Kel, s.x0 + ib, y, cb, s.x0 + ia, y + 1, ca);
      Bc[idx] = cv;
    }
    __syncthreads();
    for (int b = tid; b < bs; b += AP_NT) {
      const int ib = b >> 1;
      T acc = 0;
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const int col = 2 * (ib + t / 2 - 1) + (t & 1);
        if (col >= 0 && col < bs) acc += (T)Bc[b * 6 + t] * v[(k + 1) * bs + col];
      }
      tmp[b] = acc;
    }
    __syncthreads();
    const T* Sk = Sinv + s.foff + (long long)k * bs * bs;
    if (grp < NG) {
      T acc = 0;
      for (int j = grp; j < bs; j += NG) acc += Sk[(long long)j * bs + li] * tmp[j];
      part[grp * bs + li] = acc;
    }
    __syncthreads();
    for (int a = tid; a < bs; a += AP_NT) {
      T acc = 0;
      for (int q = 0; q < NG; ++q) acc += part[q * bs + a];
      v[k * bs + a] -= acc;
    }
    __syncthreads();
  }
  T* o = lsol + s.voff;
  for (int idx = tid; idx < nb * bs; idx += AP_NT) o[idx] = v[idx];
}

// ---------------------------------------------------------------------
// Heat eigenproblems (paper Section 4.1): on each coarse neighbourhood
// omega_l, the smallest eigenpairs of A psi = lambda M psi with
// A = sum_e E_e int grad N grad N, M = sum_e E_e int N N over the elements
// of omega_l (Neumann boundary, clamped nodes removed).  Shift-invert
// block subspace iteration with C = A + sigma M (block-tridiagonal inverse
// blocks from k_factor<1>), M-orthonormalisation by Cholesky QR applied
// twice, and Rayleigh-Ritz with a parallel (round-robin) Jacobi solver for
// the small projected matrix.  One workgroup per neighbourhood.

struct EigParams {
  int m;             // subspace block size
  int kmax;          // cap on selected modes
  int maxit;         // subspace iterations
  int rr_every;      // Rayleigh-Ritz period
  double lim;        // select lambda < lim (= tau / H^2)
  double tol;        // relative convergence of the Ritz values
};

__device__ __forceinline__ double hash_unit(unsigned long long a) {
  // splitmix64 finaliser -> uniform in [-1, 1)
  a += 0x9E3779B97F4A7C15ull;
  a = (a ^ (a >> 30)) * 0xBF58476D1CE4E5B9ull;
  a = (a ^ (a >> 27)) * 0x94D049BB133111EBull;
  a ^= a >> 31;
  return (double)(a >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// out[j][node] = sum_e kappa_e (Kel in)[node] over omega's elements for the
// first m columns; Dirichlet rows are 0.
__device__ void omega_stencil(const Geom& g, const SysDesc& s,
                              const double* __restrict__ E,
                              const uint8_t* __restrict__ dflag,
                              const double* __restrict__ Kel4,
                              const double* in, double* out, int n, int m) {
  for (int idx = threadIdx.x; idx < n * m; idx += EG_NT) {
    const int j = idx / n, node = idx - (idx / n) * n;
    const int i = node % s.nxb, k = node / s.nxb;
    const int x = s.x0 + i, y = s.y0 + k;
    double acc = 0.0;
    if (!dflag[(long long)y * g.nnx + x]) {
      for (int ey = max(y - 1, s.ey0); ey <= min(y, s.ey1 - 1); ++ey)
        for (int ex = max(x - 1, s.ex0); ex <= min(x, s.ex1 - 1); ++ex) {
          const int va = (x - ex) + 2 * (y - ey);
          double t = 0.0;
#pragma unroll
          for (int vb = 0; vb < 4; ++vb) {
            const int xb = ex + (vb & 1), yb = ey + (vb >> 1);
            t += Kel4[va * 4 + vb] * in[(long long)j * n + (yb - s.y0) * s.nxb + (xb - s.x0)];
          }
          acc += E[(long long)ey * g.nx + ex] * t;
        }
    }
    out[(long long)j * n + node] = acc;
  }
}

// G = Y^T Z (m x m) into LDS G[MAXM*MAXM]; stage is LDS scratch of
// 2*MAXM*64 doubles.
__device__ void gram(const double* Y, const double* Z, int n, int m,
                     double* G, double* stage) {
  const int tid = threadIdx.x;
  double acc0 = 0.0, acc1 = 0.0;
  const int e0 = tid, e1 = tid + EG_NT;
  for (int c0 = 0; c0 < n; c0 += 64) {
    const int cn = min(64, n - c0);
    for (int idx = tid; idx < m * 64; idx += EG_NT) {
      const int j = idx / 64, t = idx - j * 64;
      stage[j * 64 + t] = (t < cn) ? Y[(long long)j * n + c0 + t] : 0.0;
      stage[MAXM * 64 + j * 64 + t] = (t < cn) ? Z[(long long)j * n + c0 + t] : 0.0;
    }
    __syncthreads();
    if (e0 < m * m) {
      const int a = e0 / m, b = e0 - (e0 / m) * m;
      for (int t = 0; t < 64; ++t) acc0 += stage[a * 64 + t] * stage[MAXM * 64 + b * 64 + t];
    }
    if (e1 < m * m) {
      const int a = e1 / m, b = e1 - (e1 / m) * m;
      for (int t = 0; t < 64; ++t) acc1 += stage[a * 64 + t] * stage[MAXM * 64 + b * 64 + t];
    }
    __syncthreads();
  }
  if (e0 < m * m) G[e0] = acc0;
  if (e1 < m * m) G[e1] = acc1;
  __syncthreads();
  // symmetrise
  if (e0 < m * m) {
    const int a = e0 / m, b = e0 - (e0 / m) * m;
    if (a < b) {
      const double v = 0.5 * (G[a * m + b] + G[b * m + a]);
      G[a * m + b] = v;
      G[b * m + a] = v;
    }
  }
  if (e1 < m * m) {
    const int a = e1 / m, b = e1 - (e1 / m) * m;
    if (a < b) {
      const double v = 0.5 * (G[a * m + b] + G[b * m + a]);
      G[a * m + b] = v;
      G[b * m + a] = v;
    }
  }
  __syncthreads();
}

// In-place lower Cholesky of the m x m matrix G (row-major, stride m).
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
    for (int i = tid; i < m; i += EG_NT) {
      if (i == p) G[p * m + p] = piv;
      else if (i > p) G[i * m + p] /= piv;
    }
    __syncthreads();
    for (int idx = tid; idx < m * m; idx += EG_NT) {
      const int i = idx / m, j = idx - (idx / m) * m;
      if (i > p && j > p && j <= i) G[i * m + j] -= G[i * m + p] * G[j * m + p];
    }
  }
  __syncthreads();
}

// Y <- Y L^{-T} (each node's row of m values solved with L).
__device__ void apply_linvT(double* Y, int n, int m, const double* L) {
  for (int node = threadIdx.x; node < n; node += EG_NT) {
    double yv[MAXM];
#pragma unroll
    for (int j = 0; j < MAXM; ++j)
      if (j < m) yv[j] = Y[(long long)j * n + node];
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      if (i < m) {
        double t = yv[i];
#pragma unroll
        for (int k = 0; k < MAXM; ++k)
          if (k < i) t -= L[i * m + k] * yv[k];
        yv[i] = t / L[i * m + i];
      }
    }
#pragma unroll
    for (int j = 0; j < MAXM; ++j)
      if (j < m) Y[(long long)j * n + node] = yv[j];
  }
  __syncthreads();
}

// Jacobi eigenvalues of the symmetric m x m matrix A (LDS, stride m);
// V (LDS, stride m) receives the eigenvectors as columns.  Parallel
// round-robin ordering: m/2 disjoint rotations per round.
__device__ void jacobi_small(double* A, double* V, int m, double* rc,
                             double* rs, int* rp, int* rq) {
  const int tid = threadIdx.x;
  const int me = (m + 1) & ~1;            // even number of players
  for (int idx = tid; idx < m * m; idx += EG_NT) {
    const int i = idx / m, j = idx - (idx / m) * m;
    V[idx] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 30; ++sweep) {
    // convergence test
    __shared__ double offn, diagn;
    if (tid == 0) {
      double o = 0.0, d = 0.0;
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
          const double a = A[i * m + j];
          if (i == j) d += a * a; else o += a * a;
        }
      offn = o;
      diagn = d;
    }
    __syncthreads();
    if (offn <= 1e-30 * diagn || offn == 0.0) break;
    __syncthreads();
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
      for (int idx = tid; idx < (me / 2) * m; idx += EG_NT) {
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
      for (int idx = tid; idx < (me / 2) * m; idx += EG_NT) {
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

__global__ void __launch_bounds__(EG_NT)
k_heat_eigen(Geom g, const SysDesc* __restrict__ systems,
             const double* __restrict__ E, const uint8_t* __restrict__ dflag,
             const double* __restrict__ Ae, const double* __restrict__ Me,
             const double* __restrict__ Cel, const double* __restrict__ Sinv,
             double* __restrict__ Xw, double* __restrict__ Yw,
             double* __restrict__ Zw, EigParams prm,
             double* __restrict__ psi_out, double* __restrict__ lam_out,
             int* __restrict__ nsel_out, int* __restrict__ cap_out,
             int* __restrict__ err) {
  __shared__ double lbuf[3 * MAXBS * MAXM];   // solve rows / gram staging
  __shared__ double G[MAXM * MAXM];
  __shared__ double V[MAXM * MAXM];
  __shared__ double theta[MAXM], theta_old[MAXM];
  __shared__ double rc[MAXM], rs[MAXM];
  __shared__ int rp[MAXM], rq[MAXM], order[MAXM];
  __shared__ int converged;
  const SysDesc s = systems[blockIdx.x];
  const int tid = threadIdx.x;
  const int n = s.nxb * s.nyb;
  const int bs = s.nxb, nb = s.nyb;
  const int m = prm.m;
  const long long wo = s.voff * (long long)m;
  double* X = Xw + wo;
  double* Y = Yw + wo;
  double* Z = Zw + wo;

  for (int idx = tid; idx < n * m; idx += EG_NT) {
    const int j = idx / n, node = idx - (idx / n) * n;
    const int x = s.x0 + node % s.nxb, y = s.y0 + node / s.nxb;
    const bool d = dflag[(long long)y * g.nnx + x] != 0;
    const unsigned long long key =
        ((unsigned long long)blockIdx.x << 40) ^ ((unsigned long long)j << 24) ^ (unsigned long long)node;
    X[idx] = d ? 0.0 : hash_unit(key);
  }
  if (tid < MAXM) theta_old[tid] = 0.0;
  if (tid == 0) converged = 0;
  __syncthreads();

  double* Wl = lbuf;                    // bs x m
  double* Tp = lbuf + MAXBS * MAXM;     // previous row result
  double* Tc = lbuf + 2 * MAXBS * MAXM; // current row result

  for (int it = 0; it < prm.maxit; ++it) {
    // Z = M X
    omega_stencil(g, s, E, dflag, Me, X, Z, n, m);
    __syncthreads();
    // Y = C^{-1} Z : forward
    for (int k = 0; k < nb; ++k) {
      const int y = s.y0 + k;
      for (int idx = tid; idx < bs * m; idx += EG_NT) {
        const int a = idx / m, j = idx - (idx / m) * m;
        const int x = s.x0 + a;
        double w = Z[(long long)j * n + k * bs + a];
        if (k > 0 && !dflag[(long long)y * g.nnx + x]) {
          for (int di = -1; di <= 1; ++di) {
            const int b = a + di;
            if (b < 0 || b >= bs) continue;
            if (dflag[(long long)(y - 1) * g.nnx + s.x0 + b]) continue;
            const double cv = coupling<1>(g, s, E, Cel, x, y, 0, s.x0 + b, y - 1, 0);
            w -= cv * Tp[b * MAXM + j];
          }
        }
        Wl[a * MAXM + j] = w;
      }
      __syncthreads();
      const double* Sk = Sinv + s.foff + (long long)k * bs * bs;
      for (int idx = tid; idx < bs * m; idx += EG_NT) {
        const int i = idx % bs, j = idx / bs;
        double acc = 0.0;
        for (int b = 0; b < bs; ++b) acc += Sk[(long long)b * bs + i] * Wl[b * MAXM + j];
        Tc[i * MAXM + j] = acc;
        Y[(long long)j * n + k * bs + i] = acc;
      }
      __syncthreads();
      double* t = Tp; Tp = Tc; Tc = t;
    }
    // backward: Tp holds row nb-1 (final)
    for (int k = nb - 2; k >= 0; --k) {
      const int y = s.y0 + k;
      for (int idx = tid; idx < bs * m; idx += EG_NT) {
        const int b = idx / m, j = idx - (idx / m) * m;
        const int x = s.x0 + b;
        double w = 0.0;
        if (!dflag[(long long)y * g.nnx + x]) {
          for (int di = -1; di <= 1; ++di) {
            const int a = b + di;
            if (a < 0 || a >= bs) continue;
            if (dflag[(long long)(y + 1) * g.nnx + s.x0 + a]) continue;
            const double cv = coupling<1>(g, s, E, Cel, x, y, 0, s.x0 + a, y + 1, 0);
            w += cv * Tp[a * MAXM + j];
          }
        }
        Wl[b * MAXM + j] = w;
      }
      __syncthreads();
      const double* Sk = Sinv + s.foff + (long long)k * bs * bs;
      for (int idx = tid; idx < bs * m; idx += EG_NT) {
        const int i = idx % bs, j = idx / bs;
        double acc = 0.0;
        for (int b = 0; b < bs; ++b) acc += Sk[(long long)b * bs + i] * Wl[b * MAXM + j];
        const double val = Y[(long long)j * n + k * bs + i] - acc;
        Tc[i * MAXM + j] = val;
        Y[(long long)j * n + k * bs + i] = val;
      }
      __syncthreads();
      double* t = Tp; Tp = Tc; Tc = t;
    }
    // M-orthonormalise Y twice (Cholesky QR)
    for (int pass = 0; pass < 2; ++pass) {
      omega_stencil(g, s, E, dflag, Me, Y, Z, n, m);
      __syncthreads();
      gram(Y, Z, n, m, G, lbuf);
      chol_small(G, m, err);
      apply_linvT(Y, n, m, G);
    }
    const bool do_rr = ((it + 1) % prm.rr_every == 0) || (it + 1 == prm.maxit);
    if (do_rr) {
      omega_stencil(g, s, E, dflag, Ae, Y, Z, n, m);
      __syncthreads();
      gram(Y, Z, n, m, G, lbuf);
      jacobi_small(G, V, m, rc, rs, rp, rq);
      if (tid == 0) {
        for (int i = 0; i < m; ++i) order[i] = i;
        for (int i = 1; i < m; ++i) {       // insertion sort by eigenvalue
          const int oi = order[i];
          const double key = G[oi * m + oi];
          int j = i - 1;
          while (j >= 0 && G[order[j] * m + order[j]] > key) {
            order[j + 1] = order[j];
            --j;
          }
          order[j + 1] = oi;
        }
        double dmax = 0.0;
        const int nchk = min(m, prm.kmax + 1);
        for (int i = 0; i < nchk; ++i) {
          const double th = G[order[i] * m + order[i]];
          const double rel = fabs(th - theta_old[i]) / (fabs(th) + prm.lim);
          dmax = fmax(dmax, rel);
          theta[i] = th;
          theta_old[i] = th;
        }
        for (int i = nchk; i < m; ++i) theta[i] = G[order[i] * m + order[i]];
        converged = (it > 0 && dmax < prm.tol) ? 1 : 0;
      }
      __syncthreads();
      // X = Y V (columns sorted ascending)
      for (int node = tid; node < n; node += EG_NT) {
        double yv[MAXM];
#pragma unroll
        for (int j = 0; j < MAXM; ++j)
          if (j < m) yv[j] = Y[(long long)j * n + node];
        for (int c = 0; c < m; ++c) {
          const int oc = order[c];
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < MAXM; ++j)
            if (j < m) acc += yv[j] * V[j * m + oc];
          X[(long long)c * n + node] = acc;
        }
      }
      __syncthreads();
      if (converged) break;
    } else {
      double* t = X; X = Y; Y = t;
    }
  }
  // X holds the Ritz vectors (ascending).  Select lambda < lim, <= kmax.
  __shared__ int nsel;
  if (tid == 0) {
    int cnt = 0;
    for (int i = 0; i < m; ++i)
      if (theta[i] < prm.lim) ++cnt;
    nsel = min(cnt, prm.kmax);
    nsel_out[blockIdx.x] = nsel;
    cap_out[blockIdx.x] = (cnt > prm.kmax) ? 1 : 0;
    for (int i = 0; i < prm.kmax; ++i)
      lam_out[(long long)blockIdx.x * prm.kmax + i] = (i < nsel) ? theta[i] : __builtin_nan("");
  }
  __syncthreads();
  double* po = psi_out + s.voff * (long long)prm.kmax;
  for (int idx = tid; idx < nsel * n; idx += EG_NT) po[idx] = X[idx];
}

// ---------------------------------------------------------------- launchers

void launch_factor_elastic(const Geom& g, const SysDesc* sys, int nsys,
                           const double* E, const uint8_t* mask,
                           const double* Ke, void* out, bool fp32, int* err,
                           hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL((k_factor<2, float>), dim3(nsys), dim3(FT_NT), 0, s, g,
                       sys, E, mask, Ke, (float*)out, err);
  else
    hipLaunchKernelGGL((k_factor<2, double>), dim3(nsys), dim3(FT_NT), 0, s, g,
                       sys, E, mask, Ke, (double*)out, err);
}

void launch_factor_heat(const Geom& g, const SysDesc* sys, int nsys,
                        const double* E, const uint8_t* dflag,
                        const double* Cel, double* out, int* err,
                        hipStream_t s) {
  hipLaunchKernelGGL((k_factor<1, double>), dim3(nsys), dim3(FT_NT), 0, s, g,
                     sys, E, dflag, Cel, out, err);
}

void launch_level1(const Geom& g, const SysDesc* sys, int nsys,
                   const double* E, const uint8_t* mask, const double* Ke,
                   const void* Sinv, const double* r, void* lsol, bool fp32,
                   const CGScalars* sc, hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_level1<float>, dim3(nsys), dim3(AP_NT), 0, s, g, sys,
                       E, mask, Ke, (const float*)Sinv, r, (float*)lsol, sc);
  else
    hipLaunchKernelGGL(k_level1<double>, dim3(nsys), dim3(AP_NT), 0, s, g, sys,
                       E, mask, Ke, (const double*)Sinv, r, (double*)lsol, sc);
}

void launch_heat_eigen(const Geom& g, const SysDesc* sys, int nsys,
                       const double* E, const uint8_t* dflag, const double* Ae,
                       const double* Me, const double* Cel, const double* Sinv,
                       double* X, double* Y, double* Z, int m, int kmax,
                       int maxit, int rr_every, double lim, double tol,
                       double* psi, double* lam, int* nsel, int* cap, int* err,
                       hipStream_t s) {
  EigParams p{m, kmax, maxit, rr_every, lim, tol};
  hipLaunchKernelGGL(k_heat_eigen, dim3(nsys), dim3(EG_NT), 0, s, g, sys, E,
                     dflag, Ae, Me, Cel, Sinv, X, Y, Z, p, psi, lam, nsel, cap,
                     err);
}

}  // namespace msp
