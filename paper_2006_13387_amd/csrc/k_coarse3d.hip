// The coarse space of the 3D (H8) two-level preconditioner, M_EH+Rot
// (Section 4.1: heat eigenproblems on the coarse neighbourhoods with the
// eigenvalue threshold; Section 4.2: three rotations per coarse node in 3D;
// Section 2: the coarse term R_0^T K_0^{-1} R_0 of the additive operator),
// on the trilinear brick of Section 1.1.
//
// Heat pencils.  On omega_l (up to 13^3 nodes for S = 6) the pencil
// A psi = lambda M psi (kappa = E, clamped nodes removed) is solved for its
// lowest eigenpairs by shift-invert block subspace iteration with a
// Rayleigh-Ritz step every sweep.  A + sigma M is factored block-
// tridiagonally by node planes of constant z: the inverse Schur block of
// every plane is formed explicitly (the plane's Schur complement assembled
// from E by one kernel, then inverted by the batched Gauss-Jordan
// elimination on the FP64 matrix cores, all neighbourhoods at once, one
// plane after the other).  A sweep applies (A + sigma M)^{-1} to the m
// vectors of a neighbourhood as one workgroup walking its planes forward
// and back, each step a dense product with the plane's inverse block.
// Clamped nodes stay in the plane blocks as decoupled identity rows with
// zero mass, so the iterates are zero there.
//
// Coarse operator.  Columns per coarse node: chi_l psi_j e_c for each
// component c, then chi_l r_k (k = 1..3) when a mode was selected.  K Phi is
// formed column by column on the column's box, K_0 = Phi^T (K Phi) by pairs
// of neighbouring coarse nodes (fixed summation order), and K_0's
// generalised inverse by the blocked Gauss-Jordan elimination of the 2D
// path.  In the PCG the restriction runs one workgroup per coarse node and
// the prolongation is added node by node inside the first level's summation
// kernel.
#include "common.h"
#include "dev.h"
#include "small_dense.h"
#include "plane_eig.h"

namespace msp {

constexpr int C3_NT = 256;     // plane kernels: a thread per in-plane node
constexpr int C3_MAXP = 256;   // largest padded plane order
constexpr int HS_NT = 512;     // sweep, Gram and Rayleigh-Ritz workgroups
constexpr int SC_CB = 16;      // columns of a Schur-complement workgroup
constexpr int C3_MAXCOL = 3 * 24 + 3;   // columns of one coarse node (kmax <= 24)

size_t eig3_state_bytes() { return sizeof(Eig3State); }

__device__ __forceinline__ long long node_id(const Geom& g, int X, int Y, int Z) {
  return ((long long)Z * g.nny + Y) * g.nnx + X;
}

// Coupling of node (X,Y,Z) with node (X+dx, Y+dy, Z+dz) in the pencil
// matrices el (8 x 8 unit-brick element matrices, vertex v = sx + 2 sy + 4
// sz), summed over the elements of omega's element box holding both.  With
// el2 non-null the second matrix's coupling goes to *v2.
__device__ __forceinline__ double pair_coef(const Geom& g, const Nbh3& w,
                                            const double* __restrict__ E,
                                            const double* el, const double* el2,
                                            double* v2, int X, int Y, int Z,
                                            int dx, int dy, int dz) {
  double v = 0.0, u = 0.0;
#pragma unroll
  for (int sz = 0; sz < 2; ++sz) {
    const int oz = sz + dz, ez = Z - sz;
    if (oz < 0 || oz > 1 || ez < w.z0 || ez >= w.z0 + w.nbz - 1) continue;
#pragma unroll
    for (int sy = 0; sy < 2; ++sy) {
      const int oy = sy + dy, ey = Y - sy;
      if (oy < 0 || oy > 1 || ey < w.y0 || ey >= w.y0 + w.nby - 1) continue;
#pragma unroll
      for (int sx = 0; sx < 2; ++sx) {
        const int ox = sx + dx, ex = X - sx;
        if (ox < 0 || ox > 1 || ex < w.x0 || ex >= w.x0 + w.nbx - 1) continue;
        const double k = E[((long long)ez * g.ny + ey) * g.nx + ex];
        const int e = (sx + 2 * sy + 4 * sz) * 8 + ox + 2 * oy + 4 * oz;
        v += k * el[e];
        if (el2 != nullptr) u += k * el2[e];
      }
    }
  }
  if (v2 != nullptr) *v2 = u;
  return v;
}

// ---------------------------------------------------------------------
// Plane factorisation

// Plane k of every neighbourhood's block factorisation of A + sigma M:
// S_k = D_k - C_k^T G_{k-1} C_k (D_k the plane's own block, C_k the coupling
// of plane k-1 with plane k, G_{k-1} the inverse already formed in slot
// k-1), written over slot k: this workgroup's SC_CB columns b as rows (S is
// symmetric), identity on padding and on clamped nodes; the slots of
// neighbourhoods with fewer planes get the identity.  Grid (ldp / SC_CB,
// neighbourhoods); thread a forms row a.
__global__ void __launch_bounds__(C3_NT)
k3h_schur(Geom g, const Nbh3* __restrict__ nbs, int k, int ldp,
          const double* __restrict__ E, const uint8_t* __restrict__ nmask,
          const double* __restrict__ hel, double sigma, double* __restrict__ G) {
  __shared__ double el[64];
  __shared__ double T[C3_MAXP * SC_CB];
  __shared__ double Cb[SC_CB * 9];
  __shared__ int Jb[SC_CB * 9];
  const Nbh3 w = nbs[blockIdx.y];
  const int tid = threadIdx.x;
  if (tid < 64) el[tid] = hel[tid] + sigma * hel[64 + tid];
  const long long ldp2 = (long long)ldp * ldp;
  double* Sk = G + w.goff + k * ldp2;
  const int b0 = blockIdx.x * SC_CB;
  if (k >= w.nbz) {
    for (int idx = tid; idx < SC_CB * ldp; idx += C3_NT) {
      const int t = idx / ldp, a = idx - t * ldp;
      Sk[(long long)(b0 + t) * ldp + a] = (a == b0 + t) ? 1.0 : 0.0;
    }
    return;
  }
  __syncthreads();
  const int np = w.np;
  const int Z = w.z0 + k;
  if (k > 0 && tid < SC_CB * 9) {
    const int t = tid / 9, q = tid - 9 * (tid / 9);
    const int b = b0 + t;
    const int dx = q % 3 - 1, dy = q / 3 - 1;
    double c = 0.0;
    int j = -1;
    if (b < np) {
      const int bx = b % w.nbx, by = b / w.nbx;
      const int jx = bx + dx, jy = by + dy;
      if (jx >= 0 && jx < w.nbx && jy >= 0 && jy < w.nby) {
        j = jy * w.nbx + jx;
        const int X = w.x0 + bx, Y = w.y0 + by;
        if (!nmask[node_id(g, X, Y, Z)] && !nmask[node_id(g, X + dx, Y + dy, Z - 1)])
          c = pair_coef(g, w, E, el, nullptr, nullptr, X, Y, Z, dx, dy, -1);
      }
    }
    Cb[tid] = c;
    Jb[tid] = j;
  }
  __syncthreads();
  // T(i, t) = sum_q G_{k-1}(i, j_q) C(j_q, b_t)  (G symmetric: row j_q at i)
  if (k > 0 && tid < ldp) {
    const double* Gp = Sk - ldp2;
    // every load of a column issued at once (an absent coupling reads row
    // 0 and weighs it by 0, which adds exactly nothing)
    for (int t = 0; t < SC_CB; ++t) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const int j = Jb[t * 9 + q];
        const double c = j >= 0 ? Cb[t * 9 + q] : 0.0;
        s = fma(Gp[(long long)max(j, 0) * ldp + tid], c, s);
      }
      T[tid * SC_CB + t] = s;
    }
  }
  __syncthreads();
  const int a = tid;
  if (a >= ldp) return;
  const bool arow = a < np;
  int ax = 0, ay = 0;
  bool rem = true;
  if (arow) {
    ax = a % w.nbx;
    ay = a / w.nbx;
    rem = nmask[node_id(g, w.x0 + ax, w.y0 + ay, Z)] != 0;
  }
  double Din[9], Cdn[9];
  int Idn[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int dx = q % 3 - 1, dy = q / 3 - 1;
    Din[q] = 0.0;
    Cdn[q] = 0.0;
    Idn[q] = -1;
    if (arow && !rem) {
      const int nx_ = ax + dx, ny_ = ay + dy;
      if (nx_ >= 0 && nx_ < w.nbx && ny_ >= 0 && ny_ < w.nby) {
        const int X = w.x0 + ax, Y = w.y0 + ay;
        if (!nmask[node_id(g, X + dx, Y + dy, Z)])
          Din[q] = pair_coef(g, w, E, el, nullptr, nullptr, X, Y, Z, dx, dy, 0);
        if (k > 0) {
          Idn[q] = ny_ * w.nbx + nx_;
          if (!nmask[node_id(g, X + dx, Y + dy, Z - 1)])
            Cdn[q] = pair_coef(g, w, E, el, nullptr, nullptr, X, Y, Z, dx, dy, -1);
        }
      }
    }
  }
  for (int t = 0; t < SC_CB; ++t) {
    const int b = b0 + t;
    double v;
    if (!arow || rem || b >= np) {
      v = (a == b) ? 1.0 : 0.0;
    } else {
      const int dx = b % w.nbx - ax, dy = b / w.nbx - ay;
      v = (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) ? Din[(dy + 1) * 3 + dx + 1] : 0.0;
      if (k > 0) {
#pragma unroll
        for (int q = 0; q < 9; ++q)
          if (Idn[q] >= 0) v -= Cdn[q] * T[Idn[q] * SC_CB + t];
      }
    }
    Sk[(long long)b * ldp + a] = v;
  }
}

// ---------------------------------------------------------------------
// Subspace iteration

// X = a random start block (a counter-based hash of neighbourhood, column
// and box node: the same on every run), zero on clamped nodes and padding;
// state reset.  Grid (planes, neighbourhoods), thread = in-plane node.
__global__ void __launch_bounds__(C3_NT)
k3h_start(Geom g, const Nbh3* __restrict__ nbs, int ldp, int m,
          const uint8_t* __restrict__ nmask, double* __restrict__ X,
          Eig3State* __restrict__ st) {
  const Nbh3 w = nbs[blockIdx.y];
  const int k = blockIdx.x, a = threadIdx.x;
  if (k == 0 && a == 0) {
    st[blockIdx.y].done = 0;
    st[blockIdx.y].conv = 0;
  }
  if (k == 0 && a < MAXM) st[blockIdx.y].theta_old[a] = 0.0;
  if (a >= ldp) return;
  double* row = X + w.xoff + ((long long)k * ldp + a) * m;
  bool live = k < w.nbz && a < w.np;
  if (live) live = !nmask[node_id(g, w.x0 + a % w.nbx, w.y0 + a / w.nbx, w.z0 + k)];
  const unsigned long long bnode = (unsigned long long)k * w.np + a;
  for (int c = 0; c < m; ++c) {
    const unsigned long long key = ((unsigned long long)blockIdx.y << 40) ^
                                   ((unsigned long long)c << 24) ^ bnode;
    row[c] = live ? hash_unit(key) : 0.0;
  }
}

// OutM = M Y, and with BOTH also OutA = A Y, on plane k of every unfinished
// neighbourhood: row a sums the 27 neighbouring rows of Y weighted by the
// element couplings (clamped nodes: zero rows).  Grid (planes,
// neighbourhoods), thread = in-plane node.
template <int M, bool BOTH>
__global__ void __launch_bounds__(C3_NT)
k3h_stencil(Geom g, const Nbh3* __restrict__ nbs, int ldp,
            const double* __restrict__ E, const uint8_t* __restrict__ nmask,
            const double* __restrict__ hel, const double* __restrict__ Yw,
            double* __restrict__ OutA, double* __restrict__ OutM,
            const Eig3State* __restrict__ st) {
  __shared__ double el[128];
  if (st[blockIdx.y].done) return;
  const Nbh3 w = nbs[blockIdx.y];
  const int k = blockIdx.x, a = threadIdx.x;
  if (a < 128) el[a] = hel[a];
  __syncthreads();
  if (k >= w.nbz || a >= ldp) return;
  const long long ro = w.xoff + ((long long)k * ldp + a) * M;
  double oa[M], om[M];
#pragma unroll
  for (int c = 0; c < M; ++c) {
    oa[c] = 0.0;
    om[c] = 0.0;
  }
  bool live = a < w.np;
  int ax = 0, ay = 0;
  if (live) {
    ax = a % w.nbx;
    ay = a / w.nbx;
    live = !nmask[node_id(g, w.x0 + ax, w.y0 + ay, w.z0 + k)];
  }
  if (live) {
    // the vectors are zero at clamped nodes (so a clamped neighbour adds
    // exactly nothing and is not tested)
    const int X = w.x0 + ax, Y = w.y0 + ay, Z = w.z0 + k;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
      if (k + dz < 0 || k + dz >= w.nbz) continue;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        if (ay + dy < 0 || ay + dy >= w.nby) continue;
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          if (ax + dx < 0 || ax + dx >= w.nbx) continue;
          // the mass coupling, and the stiffness one into cA
          double cA = 0.0;
          const double cM = pair_coef(g, w, E, el + 64, BOTH ? el : nullptr,
                                      BOTH ? &cA : nullptr, X, Y, Z, dx, dy, dz);
          const double* yr = Yw + w.xoff +
                             ((long long)(k + dz) * ldp + (ay + dy) * w.nbx + ax + dx) * M;
#pragma unroll
          for (int c = 0; c < M; ++c) {
            const double y = yr[c];
            om[c] = fma(cM, y, om[c]);
            if (BOTH) oa[c] = fma(cA, y, oa[c]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < M; ++c) {
    OutM[ro + c] = om[c];
    if (BOTH) OutA[ro + c] = oa[c];
  }
}

// Y = (A + sigma M)^{-1} B on the m = M columns of every unfinished
// neighbourhood, forward and backward over its planes:
//   forward   y_k = G_k (b_k - C_k^T y_{k-1})
//   backward  x_k = y_k - G_k C_{k+1} x_{k+1}
// (C_k: the coupling of plane k-1 with plane k).  One workgroup per
// neighbourhood.  Thread (i, h) forms row i of the product of G_k with the
// right-hand side held in LDS over half h of the inner index; G_k is
// symmetric, so its row kk is read along i and a wave's loads are
// contiguous.  The halves are added through LDS.  The two row blocks R
// and P (ldp x M each) are dynamic LDS sized by the plane order, so that
// two workgroups fit a CU at ldp = 192, M = 24.
constexpr int SW_LB = 8;       // loads of a sweep product batch
template <int M>
__global__ void __launch_bounds__(HS_NT)
k3h_sweep(Geom g, const Nbh3* __restrict__ nbs, int ldp,
          const double* __restrict__ E, const uint8_t* __restrict__ nmask,
          const double* __restrict__ hel, double sigma,
          const double* __restrict__ G, const double* __restrict__ B,
          double* __restrict__ Yw, const Eig3State* __restrict__ st) {
  __shared__ double el[64];
  extern __shared__ double sweep_lds[];
  double* R = sweep_lds;
  double* P = sweep_lds + ldp * M;
  if (st[blockIdx.x].done) return;
  const Nbh3 w = nbs[blockIdx.x];
  const int tid = threadIdx.x;
  const int i = tid & (C3_MAXP - 1), hh = tid / C3_MAXP;
  if (tid < 64) el[tid] = hel[tid] + sigma * hel[64 + tid];
  const long long ldp2 = (long long)ldp * ldp;
  const int np = w.np;
  // rows and inner indices past the plane's nodes are padding (identity
  // rows of G_k on zero right-hand sides): neither half reads them
  const int half = (np + 1) / 2, kk0 = hh * half, kk1 = min(np, kk0 + half);
  int ax = 0, ay = 0;
  if (tid < np) {
    ax = tid % w.nbx;
    ay = tid / w.nbx;
  }
  __syncthreads();
  auto gemm = [&](int k, double (&acc)[M]) {
#pragma unroll
    for (int c = 0; c < M; ++c) acc[c] = 0.0;
    if (i >= np) return;
    const double* Gk = G + w.goff + k * ldp2 + i;
    // the column's loads in batches of SW_LB, all of a batch issued before
    // any is used (a plain loop waits for each few in turn)
    for (int kb = kk0; kb < kk1; kb += SW_LB) {
      double gv[SW_LB];
#pragma unroll
      for (int u = 0; u < SW_LB; ++u) gv[u] = Gk[(long long)min(kb + u, kk1 - 1) * ldp];
#pragma unroll
      for (int u = 0; u < SW_LB; ++u) {
        if (kb + u < kk1) {
          const double* rr = R + (kb + u) * M;
#pragma unroll
          for (int c = 0; c < M; ++c) acc[c] = fma(gv[u], rr[c], acc[c]);
        }
      }
    }
  };
  // the coupling of row tid (not clamped) with its 9 neighbours in plane
  // k + dz.  The right-hand sides are zero at clamped nodes and G_k's rows
  // and columns there are the identity's, so the vectors stay zero there:
  // a clamped neighbour adds exactly nothing and is not tested.
  auto couple = [&](int k, int dz, int q, int* nb_) -> double {
    const int dx = q % 3 - 1, dy = q / 3 - 1;
    const int jx = ax + dx, jy = ay + dy;
    *nb_ = -1;
    if (jx < 0 || jx >= w.nbx || jy < 0 || jy >= w.nby) return 0.0;
    const int X = w.x0 + ax, Y = w.y0 + ay, Z = w.z0 + k;
    *nb_ = jy * w.nbx + jx;
    return pair_coef(g, w, E, el, nullptr, nullptr, X, Y, Z, dx, dy, dz);
  };
  auto clamped = [&](int k) -> bool {
    return nmask[node_id(g, w.x0 + ax, w.y0 + ay, w.z0 + k)] != 0;
  };
  double acc[M];
  for (int k = 0; k < w.nbz; ++k) {
    if (tid < ldp) {
      double r[M];
      const double* br = B + w.xoff + ((long long)k * ldp + tid) * M;
#pragma unroll
      for (int c = 0; c < M; ++c) r[c] = tid < np ? br[c] : 0.0;
      if (k > 0 && tid < np && !clamped(k)) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
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
      if (tid < np && !clamped(k)) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
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

// GA = Y^T (A Y), GM = Y^T (M Y) over the neighbourhood's node rows, on the
// FP64 matrix cores.  Wave w forms 16 x 16 tile (w/2 % 2, w % 2) of GA
// (w < 4) or of GM; rows are staged in LDS 64 at a time (columns padded
// to 32).  Per MFMA 16x16x4 lane l supplies Y(4K + l/16, 16 ti + l%16) and
// Z(4K + l/16, 16 tj + l%16) and holds the tile entry (l/16 + 4r, l%16) in
// register r.  One workgroup per unfinished neighbourhood.
typedef double c3_d4 __attribute__((ext_vector_type(4)));
constexpr int GR_LD = 32 + 2;
template <int M>
__global__ void __launch_bounds__(HS_NT)
k3h_gram(const Nbh3* __restrict__ nbs, int ldp, const double* __restrict__ Yw,
         const double* __restrict__ AYw, const double* __restrict__ MYw,
         Eig3State* __restrict__ st) {
  __shared__ double Ys[64 * GR_LD], As[64 * GR_LD], Ms[64 * GR_LD];
  Eig3State& es = st[blockIdx.x];
  if (es.done) return;
  const Nbh3 w = nbs[blockIdx.x];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int mat = wave >> 2, ti = (wave >> 1) & 1, tj = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  const int nrows = w.nbz * w.np;
  c3_d4 acc = {0.0, 0.0, 0.0, 0.0};
  const double* Z = mat ? Ms : As;
  for (int base = 0; base < nrows; base += 64) {
    for (int idx = tid; idx < 64 * 32; idx += HS_NT) {
      const int r = idx >> 5, c = idx & 31;
      const int kr = base + r;
      double y = 0.0, ay = 0.0, my = 0.0;
      if (kr < nrows && c < M) {
        const long long o = w.xoff + ((long long)(kr / w.np) * ldp + kr % w.np) * M + c;
        y = Yw[o];
        ay = AYw[o];
        my = MYw[o];
      }
      Ys[r * GR_LD + c] = y;
      As[r * GR_LD + c] = ay;
      Ms[r * GR_LD + c] = my;
    }
    __syncthreads();
#pragma unroll
    for (int K = 0; K < 16; ++K) {
      const double av = Ys[(4 * K + lk) * GR_LD + 16 * ti + li];
      const double bv = Z[(4 * K + lk) * GR_LD + 16 * tj + li];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  double* out = mat ? es.GM : es.GA;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ii = 16 * ti + lk + 4 * r, jj = 16 * tj + li;
    if (ii < M && jj < M) out[ii * MAXM + jj] = acc[r];
  }
}

// Rayleigh-Ritz on the span of Y: with GM = L L^T, the eigenpairs (theta, Q)
// of C = L^{-1} GA L^{-T} give the Ritz values and the coefficients
// V = L^{-T} Q (columns in ascending order, M-orthonormal Ritz vectors
// Y V).  Convergence test as in the 2D iteration: the Ritz values below
// the threshold lim (at most kmax) and the next one change by less than
// tol relative to |theta| + scale (scale = lim for the heat pencils)
// since the previous step; conv counts the consecutive steps that passed
// it.  One workgroup per neighbourhood.
__global__ void __launch_bounds__(HS_NT)
k3h_rr(int m, int kmax, double lim, double scale, double tol, int first,
       Eig3State* __restrict__ st, int* __restrict__ err) {
  __shared__ double GA[MAXM * MAXM], L[MAXM * MAXM], W[MAXM * MAXM], Q[MAXM * MAXM];
  __shared__ double rc[MAXM], rs[MAXM];
  __shared__ int rp[MAXM], rq[MAXM], order[MAXM];
  Eig3State& es = st[blockIdx.x];
  if (es.done) return;
  const int tid = threadIdx.x;
  for (int e = tid; e < m * m; e += HS_NT) {
    const int a = e / m, c = e - (e / m) * m;
    GA[e] = 0.5 * (es.GA[a * MAXM + c] + es.GA[c * MAXM + a]);
    L[e] = 0.5 * (es.GM[a * MAXM + c] + es.GM[c * MAXM + a]);
  }
  __syncthreads();
  chol_small<HS_NT>(L, m, err);
  // W = L^{-1} GA (column c by thread c), then C = L^{-1} W^T into GA
  if (tid < m) {
    const int c = tid;
    for (int i = 0; i < m; ++i) {
      double t = GA[i * m + c];
      for (int k = 0; k < i; ++k) t -= L[i * m + k] * W[k * m + c];
      W[i * m + c] = t / L[i * m + i];
    }
  }
  __syncthreads();
  if (tid < m) {
    const int c = tid;
    for (int i = 0; i < m; ++i) {
      double t = W[c * m + i];
      for (int k = 0; k < i; ++k) t -= L[i * m + k] * Q[k * m + c];
      Q[i * m + c] = t / L[i * m + i];
    }
  }
  __syncthreads();
  for (int e = tid; e < m * m; e += HS_NT) {
    const int a = e / m, c = e - (e / m) * m;
    GA[e] = 0.5 * (Q[a * m + c] + Q[c * m + a]);
  }
  __syncthreads();
  jacobi_small<HS_NT>(GA, Q, m, rc, rs, rp, rq);
  // V = L^{-T} Q (back substitution, column c by thread c) into W
  if (tid < m) {
    const int c = tid;
    for (int i = m - 1; i >= 0; --i) {
      double t = Q[i * m + c];
      for (int k = i + 1; k < m; ++k) t -= L[k * m + i] * W[k * m + c];
      W[i * m + c] = t / L[i * m + i];
    }
  }
  if (tid == 0) {
    for (int i = 0; i < m; ++i) order[i] = i;
    for (int i = 1; i < m; ++i) {
      const int oi = order[i];
      const double key = GA[oi * m + oi];
      int j = i - 1;
      while (j >= 0 && GA[order[j] * m + order[j]] > key) {
        order[j + 1] = order[j];
        --j;
      }
      order[j + 1] = oi;
    }
    int nbelow = 0;
    for (int i = 0; i < m; ++i) {
      es.theta[i] = GA[order[i] * m + order[i]];
      if (es.theta[i] < lim) ++nbelow;
    }
    const int nchk = min(m - 1, min(nbelow, kmax) + 1);
    double dmax = 0.0;
    for (int i = 0; i < nchk; ++i)
      dmax = fmax(dmax, fabs(es.theta[i] - es.theta_old[i]) / (fabs(es.theta[i]) + scale));
    for (int i = 0; i < m; ++i) es.theta_old[i] = es.theta[i];
    es.conv = (!first && dmax < tol) ? es.conv + 1 : 0;
  }
  __syncthreads();
  for (int e = tid; e < m * m; e += HS_NT) {
    const int j = e / m, c = e - (e / m) * m;
    es.V[j * MAXM + c] = W[j * m + order[c]];
  }
}

// X = Y V (the Ritz vectors, ascending) on plane k; grid (planes,
// neighbourhoods), thread = in-plane row (padding rows included).
template <int M>
__global__ void __launch_bounds__(C3_NT)
k3h_ritz(const Nbh3* __restrict__ nbs, int ldp, const double* __restrict__ Yw,
         double* __restrict__ X, const Eig3State* __restrict__ st) {
  __shared__ double V[MAXM * M];
  const Eig3State& es = st[blockIdx.y];
  if (es.done) return;
  const Nbh3 w = nbs[blockIdx.y];
  for (int e = threadIdx.x; e < M * M; e += C3_NT) {
    const int j = e / M, c = e - (e / M) * M;
    V[j * M + c] = es.V[j * MAXM + c];
  }
  __syncthreads();
  const int k = blockIdx.x, a = threadIdx.x;
  if (k >= w.nbz || a >= ldp) return;
  const long long o = w.xoff + ((long long)k * ldp + a) * M;
  double y[M];
#pragma unroll
  for (int j = 0; j < M; ++j) y[j] = Yw[o + j];
#pragma unroll
  for (int c = 0; c < M; ++c) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) s = fma(y[j], V[j * M + c], s);
    X[o + c] = s;
  }
}

// A neighbourhood stops once `need` consecutive Rayleigh-Ritz steps passed
// the test: the Ritz values converge with the square of the subspace's
// angle to the eigenspace, so the steps after the first pass (each
// shrinking that angle by about (lambda_k + sigma) / (lambda_{m+1} +
// sigma)) bring the vectors to the accuracy of the values.  The number
// still iterating goes to *count (one workgroup).
__global__ void __launch_bounds__(256)
k3h_count(Eig3State* __restrict__ st, int n, int need, int* __restrict__ count) {
  __shared__ int c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  int mine = 0;
  for (int i = threadIdx.x; i < n; i += 256) {
    if (!st[i].done && st[i].conv >= need) st[i].done = 1;
    mine += st[i].done ? 0 : 1;
  }
  if (mine) atomicAdd(&c, mine);
  __syncthreads();
  if (threadIdx.x == 0) *count = c;
}

// The threshold: lambda < lim in ascending order, at most kmax; the count,
// the cap flag and the selected eigenvalues (NaN past the count).
__global__ void k3h_select(const Eig3State* __restrict__ st, int n, int m,
                           int kmax, double lim, int* __restrict__ nsel,
                           int* __restrict__ cap, double* __restrict__ lam) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n) return;
  const Eig3State& es = st[l];
  int cnt = 0;
  for (int i = 0; i < m; ++i)
    if (es.theta[i] < lim) ++cnt;
  const int ns = min(cnt, kmax);
  nsel[l] = ns;
  cap[l] = cnt > kmax ? 1 : 0;
  for (int i = 0; i < kmax; ++i)
    lam[(long long)l * kmax + i] = i < ns ? es.theta[i] : __builtin_nan("");
}

// psi of the selected modes, compact: box node b = k np + a, b nmodes + j.
template <int M>
__global__ void __launch_bounds__(C3_NT)
k3h_psi(const Nbh3* __restrict__ nbs, int ldp, const double* __restrict__ X,
        double* __restrict__ psi) {
  const Nbh3 w = nbs[blockIdx.y];
  const int k = blockIdx.x, a = threadIdx.x;
  if (k >= w.nbz || a >= w.np || w.nmodes == 0) return;
  const double* xr = X + w.xoff + ((long long)k * ldp + a) * M;
  double* pr = psi + w.psi_off + ((long long)k * w.np + a) * w.nmodes;
  for (int j = 0; j < w.nmodes; ++j) pr[j] = xr[j];
}

// ---------------------------------------------------------------------
// Coarse basis and K_0

// Value of column q of coarse node w at node (X, Y, Z) of its box: mode j
// of component c is chi_l psi_j e_c, rotation k is chi_l r_k with
// r_1 = (0, -z, y), r_2 = (z, 0, -x), r_3 = (-y, x, 0) in coordinates
// relative to the coarse node scaled by 1/H; zero at clamped DOFs.
__device__ __forceinline__ double3 phi3(const Geom& g, const Nbh3& w, int q,
                                        int X, int Y, int Z, int S0, int S1, int S2,
                                        double invH, const double* __restrict__ psi,
                                        const uint8_t* __restrict__ nmask) {
  double3 v = make_double3(0.0, 0.0, 0.0);
  const int rx_ = X - w.cx * S0, ry_ = Y - w.cy * S1, rz_ = Z - w.cz * S2;
  const double chi = (1.0 - fabs((double)rx_) / S0) * (1.0 - fabs((double)ry_) / S1) *
                     (1.0 - fabs((double)rz_) / S2);
  if (!(chi > 0.0)) return v;
  const int mb = nmask[node_id(g, X, Y, Z)];
  const int nm = w.nmodes;
  if (q < 3 * nm) {
    const int c = q / nm, j = q - c * nm;
    const long long b = ((long long)(Z - w.z0) * w.nby + (Y - w.y0)) * w.nbx + (X - w.x0);
    const double p = chi * psi[w.psi_off + b * nm + j];
    if (!(mb & (1 << c))) {
      if (c == 0) v.x = p;
      else if (c == 1) v.y = p;
      else v.z = p;
    }
  } else {
    const int k = q - 3 * nm;
    const double x = rx_ * g.h * invH, y = ry_ * g.h * invH, z = rz_ * g.h * invH;
    if (k == 0) v = make_double3(0.0, -z, y);
    else if (k == 1) v = make_double3(z, 0.0, -x);
    else v = make_double3(-y, x, 0.0);
    v.x = (mb & 1) ? 0.0 : chi * v.x;
    v.y = (mb & 2) ? 0.0 : chi * v.y;
    v.z = (mb & 4) ? 0.0 : chi * v.z;
  }
  return v;
}

// W_q = K phi_q on the box of column q's coarse node (3 values a box node,
// zero at clamped DOFs): every element of the box adds E_e K^_e phi_e at
// its vertices.  Grid (planes, columns), thread = in-plane node.
__global__ void __launch_bounds__(C3_NT)
k3c_kphi(Geom g, const Nbh3* __restrict__ nbs, const int* __restrict__ col_node,
         int S0, int S1, int S2, double invH, const double* __restrict__ Ke,
         const double* __restrict__ E, const uint8_t* __restrict__ nmask,
         const double* __restrict__ psi, double* __restrict__ Wk) {
  __shared__ double K[576];
  for (int e = threadIdx.x; e < 576; e += C3_NT) K[e] = Ke[e];
  __syncthreads();
  const int col = blockIdx.y;
  const Nbh3 w = nbs[col_node[col]];
  const int q = col - w.col0;
  const int k = blockIdx.x, a = threadIdx.x;
  if (k >= w.nbz || a >= w.np) return;
  const int ax = a % w.nbx, ay = a / w.nbx;
  const int X = w.x0 + ax, Y = w.y0 + ay, Z = w.z0 + k;
  double o0 = 0.0, o1 = 0.0, o2 = 0.0;
  for (int v = 0; v < 8; ++v) {
    const int sx = v & 1, sy = (v >> 1) & 1, sz = v >> 2;
    const int ex = X - sx, ey = Y - sy, ez = Z - sz;
    if (ex < w.x0 || ex >= w.x0 + w.nbx - 1 || ey < w.y0 || ey >= w.y0 + w.nby - 1 ||
        ez < w.z0 || ez >= w.z0 + w.nbz - 1)
      continue;
    const double Ee = E[((long long)ez * g.ny + ey) * g.nx + ex];
    for (int vb = 0; vb < 8; ++vb) {
      const double3 ph = phi3(g, w, q, ex + (vb & 1), ey + ((vb >> 1) & 1), ez + (vb >> 2),
                              S0, S1, S2, invH, psi, nmask);
      if (ph.x == 0.0 && ph.y == 0.0 && ph.z == 0.0) continue;
      const double* k0 = K + (3 * v) * 24 + 3 * vb;
      o0 += Ee * (k0[0] * ph.x + k0[1] * ph.y + k0[2] * ph.z);
      o1 += Ee * (k0[24] * ph.x + k0[25] * ph.y + k0[26] * ph.z);
      o2 += Ee * (k0[48] * ph.x + k0[49] * ph.y + k0[50] * ph.z);
    }
  }
  const int mb = nmask[node_id(g, X, Y, Z)];
  const long long nbox = (long long)w.nbz * w.np;
  double* out = Wk + w.woff + (long long)q * nbox * 3 + ((long long)k * w.np + a) * 3;
  out[0] = (mb & 1) ? 0.0 : o0;
  out[1] = (mb & 2) ? 0.0 : o1;
  out[2] = (mb & 4) ? 0.0 : o2;
}

// K_0 block of the coarse-node pair (A, B): K_0(a, b) = sum over the
// overlap of the two boxes of phi_a . W_b, the overlap's nodes taken in
// chunks of K0C staged in LDS, written in K_0's slab column order (compact
// = 1: the plain column numbering col0).  One workgroup per pair.
constexpr int K0C = 16;
constexpr int K0_ACC = (C3_MAXCOL * C3_MAXCOL + C3_NT - 1) / C3_NT;
__global__ void __launch_bounds__(C3_NT)
k3c_k0(Geom g, const Nbh3* __restrict__ nbs, const int2* __restrict__ pairs,
       int S0, int S1, int S2, double invH, const uint8_t* __restrict__ nmask,
       const double* __restrict__ psi, const double* __restrict__ Wk,
       double* __restrict__ K0, int ldk, int compact) {
  __shared__ double PA[C3_MAXCOL * 3 * K0C], WB[C3_MAXCOL * 3 * K0C];
  const int2 pr = pairs[blockIdx.x];
  const Nbh3 A = nbs[pr.x], B = nbs[pr.y];
  const int na = 3 * A.nmodes + A.nrot, nb = 3 * B.nmodes + B.nrot;
  if (na == 0 || nb == 0) return;
  const int ox0 = max(A.x0, B.x0), ox1 = min(A.x0 + A.nbx, B.x0 + B.nbx);
  const int oy0 = max(A.y0, B.y0), oy1 = min(A.y0 + A.nby, B.y0 + B.nby);
  const int oz0 = max(A.z0, B.z0), oz1 = min(A.z0 + A.nbz, B.z0 + B.nbz);
  if (ox1 <= ox0 || oy1 <= oy0 || oz1 <= oz0) return;
  const int onx = ox1 - ox0, ony = oy1 - oy0;
  const int nov = onx * ony * (oz1 - oz0);
  const long long bbox = (long long)B.nbz * B.np;
  const int tid = threadIdx.x;
  double acc[K0_ACC];
#pragma unroll
  for (int u = 0; u < K0_ACC; ++u) acc[u] = 0.0;
  const int nent = na * nb;
  for (int base = 0; base < nov; base += K0C) {
    for (int idx = tid; idx < na * K0C; idx += C3_NT) {
      const int qa = idx / K0C, t = idx - qa * K0C;
      const int o = base + t;
      double3 ph = make_double3(0.0, 0.0, 0.0);
      if (o < nov) {
        const int X = ox0 + o % onx, Y = oy0 + (o / onx) % ony, Z = oz0 + o / (onx * ony);
        ph = phi3(g, A, qa, X, Y, Z, S0, S1, S2, invH, psi, nmask);
      }
      double* d = PA + qa * 3 * K0C + 3 * t;
      d[0] = ph.x;
      d[1] = ph.y;
      d[2] = ph.z;
    }
    for (int idx = tid; idx < nb * K0C; idx += C3_NT) {
      const int qb = idx / K0C, t = idx - qb * K0C;
      const int o = base + t;
      double* d = WB + qb * 3 * K0C + 3 * t;
      if (o < nov) {
        const int X = ox0 + o % onx, Y = oy0 + (o / onx) % ony, Z = oz0 + o / (onx * ony);
        const long long bn = ((long long)(Z - B.z0) * B.nby + (Y - B.y0)) * B.nbx + (X - B.x0);
        const double* s = Wk + B.woff + (long long)qb * bbox * 3 + bn * 3;
        d[0] = s[0];
        d[1] = s[1];
        d[2] = s[2];
      } else {
        d[0] = d[1] = d[2] = 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < K0_ACC; ++u) {
      const int e = tid + u * C3_NT;
      if (e < nent) {
        const int qa = e / nb, qb = e - qa * nb;
        const double* pa = PA + qa * 3 * K0C;
        const double* wb = WB + qb * 3 * K0C;
        double s = acc[u];
        for (int t = 0; t < 3 * K0C; ++t) s = fma(pa[t], wb[t], s);
        acc[u] = s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < K0_ACC; ++u) {
    const int e = tid + u * C3_NT;
    if (e < nent) {
      const int qa = e / nb, qb = e - qa * nb;
      const int ra = compact ? A.col0 : A.kcol0, rb = compact ? B.col0 : B.kcol0;
      K0[(long long)(ra + qa) * ldk + rb + qb] = acc[u];
    }
  }
}

// Dense export of the basis (column-major n x N_c) for checks on small
// meshes: grid (node blocks, columns).
__global__ void __launch_bounds__(C3_NT)
k3c_export(Geom g, const Nbh3* __restrict__ nbs, const int* __restrict__ col_node,
           int S0, int S1, int S2, double invH, const uint8_t* __restrict__ nmask,
           const double* __restrict__ psi, double* __restrict__ out) {
  const long long nn = (long long)g.nnx * g.nny * g.nnz;
  const long long node = (long long)blockIdx.x * C3_NT + threadIdx.x;
  if (node >= nn) return;
  const int col = blockIdx.y;
  const Nbh3 w = nbs[col_node[col]];
  const int X = (int)(node % g.nnx), Y = (int)((node / g.nnx) % g.nny), Z = (int)(node / ((long long)g.nnx * g.nny));
  double3 v = make_double3(0.0, 0.0, 0.0);
  if (X >= w.x0 && X < w.x0 + w.nbx && Y >= w.y0 && Y < w.y0 + w.nby && Z >= w.z0 &&
      Z < w.z0 + w.nbz)
    v = phi3(g, w, col - w.col0, X, Y, Z, S0, S1, S2, invH, psi, nmask);
  double* o = out + (long long)col * 3 * nn + 3 * node;
  o[0] = v.x;
  o[1] = v.y;
  o[2] = v.z;
}

// ---------------------------------------------------------------------
// Coarse apply

// c = R_0 r (in K_0's slab column order): one workgroup per coarse node,
// its columns' sums over the box (per-thread partials over a fixed node
// stride, then the workgroup sum in fixed order); up to 16 modes a pass.
__global__ void __launch_bounds__(C3_NT)
k3c_restrict(Geom g, const Nbh3* __restrict__ nbs, int S0, int S1, int S2,
             double invH, const uint8_t* __restrict__ nmask,
             const double* __restrict__ psi, const double* __restrict__ r,
             double* __restrict__ c, const CGScalars* __restrict__ sc) {
  __shared__ double red[C3_NT / 64][3 * 16 + 3];
  __shared__ int shd;
  if (sc != nullptr && block_read_done(sc, &shd)) return;
  const Nbh3 w = nbs[blockIdx.x];
  const int nm = w.nmodes;
  if (3 * nm + w.nrot == 0) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nbox = w.nbz * w.np;
  for (int j0 = 0; j0 < max(nm, 1); j0 += 16) {
    const int nj = min(16, nm - j0);
    const bool rot = j0 == 0 && w.nrot > 0;
    double acc[3 * 16 + 3];
#pragma unroll
    for (int u = 0; u < 3 * 16 + 3; ++u) acc[u] = 0.0;
    for (int b = tid; b < nbox; b += C3_NT) {
      const int k = b / w.np, a = b - k * w.np;
      const int rx_ = a % w.nbx + w.x0 - w.cx * S0, ry_ = a / w.nbx + w.y0 - w.cy * S1,
                rz_ = k + w.z0 - w.cz * S2;
      const double chi = (1.0 - fabs((double)rx_) / S0) * (1.0 - fabs((double)ry_) / S1) *
                         (1.0 - fabs((double)rz_) / S2);
      if (!(chi > 0.0)) continue;
      const long long node = node_id(g, w.x0 + a % w.nbx, w.y0 + a / w.nbx, w.z0 + k);
      // the mask, r and the modes are loaded together (no load waits for
      // the mask), the clamped components dropped afterwards
      const int mb = nmask[node];
      const double rv0 = r[3 * node], rv1 = r[3 * node + 1], rv2 = r[3 * node + 2];
      const double r0 = (mb & 1) ? 0.0 : chi * rv0;
      const double r1 = (mb & 2) ? 0.0 : chi * rv1;
      const double r2 = (mb & 4) ? 0.0 : chi * rv2;
      const double* ps = psi + w.psi_off + (long long)b * nm + j0;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        if (j < nj) {
          const double p = ps[j];
          acc[j] = fma(p, r0, acc[j]);
          acc[16 + j] = fma(p, r1, acc[16 + j]);
          acc[32 + j] = fma(p, r2, acc[32 + j]);
        }
      }
      if (rot) {
        const double x = rx_ * g.h * invH, y = ry_ * g.h * invH, z = rz_ * g.h * invH;
        acc[48] += -z * r1 + y * r2;
        acc[49] += z * r0 - x * r2;
        acc[50] += -y * r0 + x * r1;
      }
    }
#pragma unroll
    for (int u = 0; u < 3 * 16 + 3; ++u) {
      const double s = wave_sum(acc[u]);
      if (lane == 0) red[wave][u] = s;
    }
    __syncthreads();
    if (tid < 3 * 16 + 3) {
      double s = 0.0;
#pragma unroll
      for (int v = 0; v < C3_NT / 64; ++v) s += red[v][tid];
      const int u = tid;
      if (u < 48) {
        const int comp = u / 16, j = u - 16 * comp;
        if (j < nj) c[w.kcol0 + comp * nm + j0 + j] = s;
      } else if (rot) {
        c[w.kcol0 + 3 * nm + (u - 48)] = s;
      }
    }
    __syncthreads();
  }
}

// One step of the slab solve with K_0's block LDL^T (the windowed
// Gauss-Jordan factors of the scaled K_0 = S K S, S = diag(sd)):
//   out_i = sd_i bias_i + sum_{j in [a0, a1)} F_ij xa_j - sum_{j in [b0, b1)} F_ij xb_j
// for the rows i of one slab, and outs_i = sd_i out_i when outs is set.
// Forward, slab k: bias = c, a = slab k-1 with xa = w (F = -C^T G there),
// out = w.  Backward: a = slab k with xa = w (F = G_k), b = slab k+1 with
// xb = y (F = G_k C_k), out = y, outs = c0 = S y.  Each wave takes one row
// with 16-byte loads, unrolled so that a lane's loads of the row (about
// nine of each range) are in flight together: a step costs about one
// memory latency, and four rows a workgroup put about 270 workgroups on the
// chip for a slab of 1,088 rows.
constexpr int SLAB_ROWS = 4;
__global__ void __launch_bounds__(256)
k3c_slab_step(const double* __restrict__ F, int ldk, int r0, int r1,
              const double* __restrict__ bias, const double* __restrict__ sd,
              int a0, int a1, const double* __restrict__ xa, int b0, int b1,
              const double* __restrict__ xb, double* __restrict__ out,
              double* __restrict__ outs, const CGScalars* __restrict__ sc) {
  __shared__ int shd;
  if (sc != nullptr && block_read_done(sc, &shd)) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = r0 + blockIdx.x * SLAB_ROWS + wave;
  if (i >= r1) return;
  const double* f = F + (long long)i * ldk;
  double s = 0.0, t = 0.0;
  // column ranges are whole 64-column blocks: 16-byte loads stay aligned
#pragma unroll 8
  for (int j = a0 + 2 * lane; j < a1; j += 128) {
    const double2 x = *reinterpret_cast<const double2*>(xa + j);
    const double2 p = *reinterpret_cast<const double2*>(f + j);
    s = fma(p.x, x.x, fma(p.y, x.y, s));
  }
#pragma unroll 8
  for (int j = b0 + 2 * lane; j < b1; j += 128) {
    const double2 x = *reinterpret_cast<const double2*>(xb + j);
    const double2 p = *reinterpret_cast<const double2*>(f + j);
    t = fma(p.x, x.x, fma(p.y, x.y, t));
  }
  const double u = wave_sum(s) - wave_sum(t);
  if (lane == 0) {
    double v = u;
    if (bias != nullptr) v += sd[i] * bias[i];
    out[i] = v;
    if (outs != nullptr) outs[i] = sd[i] * v;
  }
}

// ---------------------------------------------------------------- launchers

void launch_local_inverse3_strided(double*, int, int, long long, double*, double*,
                                   double*, double*, int*, float*, hipStream_t);

int eig3_block(int kmax) {
  const int m = ((kmax + 8 + 7) / 8) * 8;
  return m > MAXM ? MAXM : m;
}

int coarse3_max_plane() { return C3_MAXP; }
int coarse3_max_cols() { return C3_MAXCOL; }

// Block factorisation of every neighbourhood's A + sigma M, plane by plane:
// Schur complement, then its inverse in place (scaled batched Gauss-Jordan).
void launch_heat3_factor(const Geom& g, const Nbh3* nbs, int nnb, int pmax, int ldp,
                         const double* E, const uint8_t* nmask, const double* hel,
                         double sigma, double* G, double* sdiag, double* LD,
                         double* Lp, double* Rp, int* dropped, hipStream_t s) {
  const long long ldp2 = (long long)ldp * ldp;
  for (int k = 0; k < pmax; ++k) {
    hipLaunchKernelGGL(k3h_schur, dim3(ldp / SC_CB, nnb), dim3(C3_NT), 0, s, g, nbs,
                       k, ldp, E, nmask, hel, sigma, G);
    launch_local_inverse3_strided(G + k * ldp2, ldp, nnb, pmax * ldp2, sdiag, LD, Lp,
                                  Rp, dropped, nullptr, s);
  }
}

void launch_heat3_start(const Geom& g, const Nbh3* nbs, int nnb, int pmax, int ldp,
                        int m, const uint8_t* nmask, double* X, void* st,
                        hipStream_t s) {
  hipLaunchKernelGGL(k3h_start, dim3(pmax, nnb), dim3(C3_NT), 0, s, g, nbs, ldp, m,
                     nmask, X, (Eig3State*)st);
}

template <int M>
static void heat3_step_m(const Geom& g, const Nbh3* nbs, int nnb, int pmax, int ldp,
                         const double* E, const uint8_t* nmask, const double* hel,
                         double sigma, const double* G, double* X, double* Y,
                         double* T, double* U, Eig3State* st, int kmax, double lim,
                         double tol, int first, int* err, hipStream_t s) {
  // T = M X; Y = (A + sigma M)^{-1} T; T = A Y, U = M Y; Gram; RR; X = Y V
  hipLaunchKernelGGL((k3h_stencil<M, false>), dim3(pmax, nnb), dim3(C3_NT), 0, s, g,
                     nbs, ldp, E, nmask, hel, X, nullptr, T, st);
  const size_t lds = 2ull * ldp * M * sizeof(double);
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k3h_sweep<M>),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(2ull * C3_MAXP * M * sizeof(double)));
    attr_set = true;
  }
  hipLaunchKernelGGL((k3h_sweep<M>), dim3(nnb), dim3(HS_NT), lds, s, g, nbs, ldp, E,
                     nmask, hel, sigma, G, T, Y, st);
  hipLaunchKernelGGL((k3h_stencil<M, true>), dim3(pmax, nnb), dim3(C3_NT), 0, s, g,
                     nbs, ldp, E, nmask, hel, Y, T, U, st);
  hipLaunchKernelGGL((k3h_gram<M>), dim3(nnb), dim3(HS_NT), 0, s, nbs, ldp, Y, T, U, st);
  hipLaunchKernelGGL(k3h_rr, dim3(nnb), dim3(HS_NT), 0, s, M, kmax, lim, lim, tol,
                     first, st, err);
  hipLaunchKernelGGL((k3h_ritz<M>), dim3(pmax, nnb), dim3(C3_NT), 0, s, nbs, ldp, Y,
                     X, st);
}

void launch_heat3_step(int m, const Geom& g, const Nbh3* nbs, int nnb, int pmax,
                       int ldp, const double* E, const uint8_t* nmask,
                       const double* hel, double sigma, const double* G, double* X,
                       double* Y, double* T, double* U, void* st, int kmax,
                       double lim, double tol, int first, int* err, hipStream_t s) {
  Eig3State* es = (Eig3State*)st;
  switch (m) {
    case 8: heat3_step_m<8>(g, nbs, nnb, pmax, ldp, E, nmask, hel, sigma, G, X, Y, T, U, es, kmax, lim, tol, first, err, s); break;
    case 16: heat3_step_m<16>(g, nbs, nnb, pmax, ldp, E, nmask, hel, sigma, G, X, Y, T, U, es, kmax, lim, tol, first, err, s); break;
    case 24: heat3_step_m<24>(g, nbs, nnb, pmax, ldp, E, nmask, hel, sigma, G, X, Y, T, U, es, kmax, lim, tol, first, err, s); break;
    default: heat3_step_m<32>(g, nbs, nnb, pmax, ldp, E, nmask, hel, sigma, G, X, Y, T, U, es, kmax, lim, tol, first, err, s); break;
  }
}

// The Rayleigh-Ritz part of a sweep on row-blocked pencils of any kind:
// Gram matrices of Y with A Y (in T) and M Y (in U), the small
// eigenproblem, X = Y V.
// The first mrr columns take part in the small eigenproblem (mrr < M: the
// rest are zero and their coefficients must be zero too).
template <int M>
static void plane_rr_m(const Nbh3* nbs, int nnb, int pmax, int ldp, const double* Y,
                       const double* T, const double* U, double* X, Eig3State* st,
                       int kmax, double lim, double scale, double tol, int first,
                       int* err, hipStream_t s, int mrr = M) {
  hipLaunchKernelGGL((k3h_gram<M>), dim3(nnb), dim3(HS_NT), 0, s, nbs, ldp, Y, T, U, st);
  hipLaunchKernelGGL(k3h_rr, dim3(nnb), dim3(HS_NT), 0, s, mrr, kmax, lim, scale, tol,
                     first, st, err);
  hipLaunchKernelGGL((k3h_ritz<M>), dim3(pmax, nnb), dim3(C3_NT), 0, s, nbs, ldp, Y,
                     X, st);
}

void launch_plane_rr(int m, const Nbh3* nbs, int nnb, int pmax, int ldp, const double* Y,
                     const double* T, const double* U, double* X, void* st, int kmax,
                     double lim, double scale, double tol, int first, int* err,
                     hipStream_t s) {
  Eig3State* es = (Eig3State*)st;
  switch (m) {
    case 8: plane_rr_m<8>(nbs, nnb, pmax, ldp, Y, T, U, X, es, kmax, lim, scale, tol, first, err, s); break;
    case 16: plane_rr_m<16>(nbs, nnb, pmax, ldp, Y, T, U, X, es, kmax, lim, scale, tol, first, err, s); break;
    case 24: plane_rr_m<24>(nbs, nnb, pmax, ldp, Y, T, U, X, es, kmax, lim, scale, tol, first, err, s); break;
    default: plane_rr_m<32>(nbs, nnb, pmax, ldp, Y, T, U, X, es, kmax, lim, scale, tol, first, err, s); break;
  }
}

// One Rayleigh-Ritz step on the first mrr of m stored columns (the
// randomized setup: snapshots and rigid-body motions, zero columns after
// them, zero coefficients there from the start kernel).
void launch_plane_rr_live(int m, int mrr, const Nbh3* nbs, int nnb, int pmax, int ldp,
                          const double* Y, const double* T, const double* U, double* X,
                          void* st, int kmax, double lim, double scale, int* err,
                          hipStream_t s) {
  Eig3State* es = (Eig3State*)st;
  switch (m) {
    case 8: plane_rr_m<8>(nbs, nnb, pmax, ldp, Y, T, U, X, es, kmax, lim, scale, 0.0, 1, err, s, mrr); break;
    case 16: plane_rr_m<16>(nbs, nnb, pmax, ldp, Y, T, U, X, es, kmax, lim, scale, 0.0, 1, err, s, mrr); break;
    case 24: plane_rr_m<24>(nbs, nnb, pmax, ldp, Y, T, U, X, es, kmax, lim, scale, 0.0, 1, err, s, mrr); break;
    default: plane_rr_m<32>(nbs, nnb, pmax, ldp, Y, T, U, X, es, kmax, lim, scale, 0.0, 1, err, s, mrr); break;
  }
}

// State reset for a new subspace iteration (the start block is the
// caller's).
__global__ void k3h_reset(Eig3State* __restrict__ st, int n) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n) return;
  st[l].done = 0;
  st[l].conv = 0;
  for (int i = 0; i < MAXM; ++i) st[l].theta_old[i] = 0.0;
}

void launch_plane_reset(void* st, int nnb, hipStream_t s) {
  hipLaunchKernelGGL(k3h_reset, dim3((nnb + 127) / 128), dim3(128), 0, s,
                     (Eig3State*)st, nnb);
}

// Selection by count: want[l] lowest Ritz values (at most m), their
// values into lam (kmax_out per neighbourhood, NaN past the count).
__global__ void k3h_select_count(const Eig3State* __restrict__ st, int n, int m,
                                 const int* __restrict__ want, int kmax_out,
                                 int* __restrict__ nsel, double* __restrict__ lam) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n) return;
  const int ns = min(want[l], m);
  nsel[l] = ns;
  for (int i = 0; i < kmax_out; ++i)
    lam[(long long)l * kmax_out + i] = i < ns ? st[l].theta[i] : __builtin_nan("");
}

void launch_plane_select_count(const void* st, int nnb, int m, const int* want,
                               int kmax_out, int* nsel, double* lam, hipStream_t s) {
  hipLaunchKernelGGL(k3h_select_count, dim3((nnb + 127) / 128), dim3(128), 0, s,
                     (const Eig3State*)st, nnb, m, want, kmax_out, nsel, lam);
}

void launch_heat3_count(void* st, int nnb, int need, int* count, hipStream_t s) {
  hipLaunchKernelGGL(k3h_count, dim3(1), dim3(256), 0, s, (Eig3State*)st, nnb, need,
                     count);
}

void launch_heat3_select(const void* st, int nnb, int m, int kmax, double lim,
                         int* nsel, int* cap, double* lam, hipStream_t s) {
  hipLaunchKernelGGL(k3h_select, dim3((nnb + 127) / 128), dim3(128), 0, s,
                     (const Eig3State*)st, nnb, m, kmax, lim, nsel, cap, lam);
}

void launch_heat3_psi(int m, const Nbh3* nbs, int nnb, int pmax, int ldp,
                      const double* X, double* psi, hipStream_t s) {
  const dim3 gr(pmax, nnb);
  switch (m) {
    case 8: hipLaunchKernelGGL(k3h_psi<8>, gr, dim3(C3_NT), 0, s, nbs, ldp, X, psi); break;
    case 16: hipLaunchKernelGGL(k3h_psi<16>, gr, dim3(C3_NT), 0, s, nbs, ldp, X, psi); break;
    case 24: hipLaunchKernelGGL(k3h_psi<24>, gr, dim3(C3_NT), 0, s, nbs, ldp, X, psi); break;
    default: hipLaunchKernelGGL(k3h_psi<32>, gr, dim3(C3_NT), 0, s, nbs, ldp, X, psi); break;
  }
}

void launch_coarse3_kphi(const Geom& g, const Nbh3* nbs, const int* col_node, int ncols,
                         int pmax, int S0, int S1, int S2, double invH,
                         const double* Ke, const double* E, const uint8_t* nmask,
                         const double* psi, double* W, hipStream_t s) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k3c_kphi, dim3(pmax, ncols), dim3(C3_NT), 0, s, g, nbs, col_node,
                     S0, S1, S2, invH, Ke, E, nmask, psi, W);
}

void launch_coarse3_k0(const Geom& g, const Nbh3* nbs, const int2* pairs, int npairs,
                       int S0, int S1, int S2, double invH, const uint8_t* nmask,
                       const double* psi, const double* W, double* K0, int ldk,
                       int compact, hipStream_t s) {
  if (npairs <= 0) return;
  hipLaunchKernelGGL(k3c_k0, dim3(npairs), dim3(C3_NT), 0, s, g, nbs, pairs, S0, S1,
                     S2, invH, nmask, psi, W, K0, ldk, compact);
}

void launch_coarse3_export(const Geom& g, const Nbh3* nbs, const int* col_node,
                           int ncols, int S0, int S1, int S2, double invH,
                           const uint8_t* nmask, const double* psi, double* out,
                           hipStream_t s) {
  if (ncols <= 0) return;
  const long long nn = (long long)g.nnx * g.nny * g.nnz;
  hipLaunchKernelGGL(k3c_export, dim3((unsigned)((nn + C3_NT - 1) / C3_NT), ncols),
                     dim3(C3_NT), 0, s, g, nbs, col_node, S0, S1, S2, invH, nmask,
                     psi, out);
}

void launch_coarse3_restrict(const Geom& g, const Nbh3* nbs, int nnb, int S0, int S1,
                             int S2, double invH, const uint8_t* nmask,
                             const double* psi, const double* r, double* c,
                             const CGScalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(k3c_restrict, dim3(nnb), dim3(C3_NT), 0, s, g, nbs, S0, S1, S2,
                     invH, nmask, psi, r, c, sc);
}

// c0 = K_0^+ c by the slab factors (sb: slab k spans the 64-column blocks
// [sb[k], sb[k+1])): forward over the slabs into w, backward into y and
// c0 = S y.
void launch_coarse3_solve(const double* F, int ldk, const int* sb, int nslab,
                          const double* sd, const double* c, double* w, double* y,
                          double* c0, const CGScalars* sc, hipStream_t s) {
  for (int k = 0; k < nslab; ++k) {
    const int r0 = 64 * sb[k], r1 = 64 * sb[k + 1];
    const int a0 = k > 0 ? 64 * sb[k - 1] : r0, a1 = k > 0 ? r0 : r0;
    hipLaunchKernelGGL(k3c_slab_step, dim3((r1 - r0 + SLAB_ROWS - 1) / SLAB_ROWS), dim3(256),
                       0, s, F, ldk, r0, r1, c, sd, a0, a1, w, 0, 0, (const double*)nullptr, w,
                       (double*)nullptr, sc);
  }
  for (int k = nslab - 1; k >= 0; --k) {
    const int r0 = 64 * sb[k], r1 = 64 * sb[k + 1];
    const int b0 = r1, b1 = k + 1 < nslab ? 64 * sb[k + 2] : r1;
    hipLaunchKernelGGL(k3c_slab_step, dim3((r1 - r0 + SLAB_ROWS - 1) / SLAB_ROWS), dim3(256),
                       0, s, F, ldk, r0, r1, (const double*)nullptr, sd, r0, r1, w, b0, b1, y,
                       y, c0, sc);
  }
}

}  // namespace msp
