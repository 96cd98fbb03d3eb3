// Coarse level of M_EH+Rot (paper Sections 2, 4.1-4.3) and the kernel that
// assembles z = M^{-1} r.
//
// Coarse basis (implicit): for coarse node l with heat modes psi_j on its
// neighbourhood omega_l, columns chi_l psi_j e_c (c = 0, 1) and, when at
// least one mode was selected, chi_l r_l with r_l the rotation about the
// coarse node scaled by 1/H.  chi_l is the coarse bilinear hat, evaluated
// analytically; only psi is stored.  Entries at clamped DOFs are zero.
//
// K_0 = R_0 K R_0^T is assembled from W = K Phi per column and the
// products Phi_a^T W_b over overlapping neighbourhoods, scaled to unit
// diagonal and inverted by blocked Gauss-Jordan with zero-pivot dropping
// (each block step: the pivot block by pivot-by-pivot Gauss-Jordan, the
// block row and column by substitution with its L D L^T factors, the rest
// by a rank-64 update on the FP64 matrix cores).
// Dropping a (numerically) dependent direction gives a generalized inverse
// G of K_0, and R_0^T G R_0 does not depend on which one: it is the
// K-orthogonal projection onto the coarse space composed with K^{-1}.
#include <algorithm>
#include "common.h"
#include "dev.h"

namespace msp {

constexpr int CK_NT = 256;
constexpr int GJB = 64;           // Gauss-Jordan block

__device__ __forceinline__ double chi_at(const Geom& g, int cx, int cy, int x,
                                         int y) {
  const double ax = 1.0 - fabs((double)(x - cx * g.sx)) / g.sx;
  const double ay = 1.0 - fabs((double)(y - cy * g.sy)) / g.sy;
  return (ax > 0.0 && ay > 0.0) ? ax * ay : 0.0;
}

// Value of coarse column lc of coarse node cn at node (x, y) (2 comps).
__device__ __forceinline__ double2 phi_at(const Geom& g, const CoarseNode& cn,
                                          const double* __restrict__ psi,
                                          const uint8_t* __restrict__ mask,
                                          int lc, int x, int y, double invH) {
  if (x < cn.x0 || x >= cn.x0 + cn.nxw || y < cn.y0 || y >= cn.y0 + cn.nyw)
    return make_double2(0.0, 0.0);
  const double chi = chi_at(g, cn.cx, cn.cy, x, y);
  if (chi == 0.0) return make_double2(0.0, 0.0);
  const long long node = (long long)y * g.nnx + x;
  const uchar2 m = reinterpret_cast<const uchar2*>(mask)[node];
  const int nw = cn.nxw * cn.nyw;
  const int loc = (y - cn.y0) * cn.nxw + (x - cn.x0);
  double vx = 0.0, vy = 0.0;
  if (lc < 2 * cn.nmodes) {
    const int comp = lc / cn.nmodes, j = lc - comp * cn.nmodes;
    const double v = chi * psi[cn.psi_off + (long long)j * nw + loc];
    if (comp == 0) vx = v; else vy = v;
  } else {
    const double rx = (x - cn.cx * g.sx) * g.h * invH;
    const double ry = (y - cn.cy * g.sy) * g.h * invH;
    vx = -chi * ry;
    vy = chi * rx;
  }
  return make_double2(m.x ? 0.0 : vx, m.y ? 0.0 : vy);
}

// W_col = K Phi_col on the closed box of omega_l (zero at clamped DOFs).
__global__ void __launch_bounds__(CK_NT)
k_coarse_kphi(Geom g, const CoarseNode* __restrict__ cnodes,
              const int* __restrict__ col_node, const double* __restrict__ Ke,
              const double* __restrict__ E, const uint8_t* __restrict__ mask,
              const double* __restrict__ psi, double* __restrict__ W,
              double invH) {
  __shared__ double ks[64];
  const int col = blockIdx.x;
  const int l = col_node[col];
  const CoarseNode cn = cnodes[l];
  const int lc = col - cn.col0;
  if (threadIdx.x < 64) ks[threadIdx.x] = Ke[threadIdx.x];
  __syncthreads();
  const int nw = cn.nxw * cn.nyw;
  double* out = W + cn.w_off + (long long)lc * 2 * nw;
  for (int loc = threadIdx.x; loc < nw; loc += CK_NT) {
    const int x = cn.x0 + loc % cn.nxw, y = cn.y0 + loc / cn.nxw;
    double y0 = 0.0, y1 = 0.0;
    for (int ey = max(y - 1, 0); ey <= min(y, g.ny - 1); ++ey)
      for (int ex = max(x - 1, 0); ex <= min(x, g.nx - 1); ++ex) {
        const int a = (x - ex) + 2 * (y - ey);
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const double2 u = phi_at(g, cn, psi, mask, lc, ex + (b & 1), ey + (b >> 1), invH);
          s0 += ks[(2 * a) * 8 + 2 * b] * u.x + ks[(2 * a) * 8 + 2 * b + 1] * u.y;
          s1 += ks[(2 * a + 1) * 8 + 2 * b] * u.x + ks[(2 * a + 1) * 8 + 2 * b + 1] * u.y;
        }
        const double ee = E[(long long)ey * g.nx + ex];
        y0 += ee * s0;
        y1 += ee * s1;
      }
    const uchar2 m = reinterpret_cast<const uchar2*>(mask)[(long long)y * g.nnx + x];
    out[2 * loc] = m.x ? 0.0 : y0;
    out[2 * loc + 1] = m.y ? 0.0 : y1;
  }
}

// K_0 block of coarse nodes (l, l2): K0[a][b] = Phi_a^T W_b over the
// intersection of omega_l and omega_l2.  One workgroup per ordered pair.
// Chunks of K0_CH nodes (2 K0_CH DOFs) of the pair's columns are staged in
// LDS (rows of K0_LD doubles), and the block accumulates on the FP64 matrix
// cores: wave w owns the 16 x 16 tiles w, w + 4, ... of the (up to 4 x 4)
// tile grid; per MFMA 16x16x4, lane l supplies Phi_a(16R + l%16, k) and
// W_b(k, 16C + l%16) for the chunk DOF k = 4K + l/16 and receives
// (16R + l/16 + 4r, 16C + l%16) in register r.  Staged rows past na / nbc
// hold stale values that reach only dropped rows and columns.
constexpr int K0_CH = 32;      // nodes per LDS chunk
constexpr int K0_LD = 2 * K0_CH + 2;   // LDS row stride (banks)
constexpr int MAXCOL = 2 * 24 + 1;
constexpr int K0_TR = (MAXCOL + 15) / 16;   // tile rows (and columns)
typedef double k0_d4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(CK_NT)
k_coarse_k0(Geom g, const CoarseNode* __restrict__ cnodes,
            const int2* __restrict__ pairs, const uint8_t* __restrict__ mask,
            const double* __restrict__ psi, const double* __restrict__ W,
            double* __restrict__ K0, int ldk, double invH) {
  static_assert(CK_NT == 256, "four waves share the tiles");
  __shared__ double pa[16 * K0_TR * K0_LD];
  __shared__ double wb[16 * K0_TR * K0_LD];
  const int2 pr = pairs[blockIdx.x];
  const CoarseNode A = cnodes[pr.x];
  const CoarseNode B = cnodes[pr.y];
  const int na = 2 * A.nmodes + A.nrot;
  const int nbc = 2 * B.nmodes + B.nrot;
  if (na == 0 || nbc == 0) return;
  const int xlo = max(A.x0, B.x0), xhi = min(A.x0 + A.nxw, B.x0 + B.nxw);
  const int ylo = max(A.y0, B.y0), yhi = min(A.y0 + A.nyw, B.y0 + B.nyw);
  const int nxi = max(0, xhi - xlo), nyi = max(0, yhi - ylo);
  const int ni = nxi * nyi;
  const int nwB = B.nxw * B.nyw;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int tra = (na + 15) >> 4, trb = (nbc + 15) >> 4;
  k0_d4 acc[K0_TR];
#pragma unroll
  for (int u = 0; u < K0_TR; ++u) acc[u] = {0.0, 0.0, 0.0, 0.0};
  for (int c0 = 0; c0 < ni; c0 += K0_CH) {
    const int cn = min(K0_CH, ni - c0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < na * K0_CH; idx += CK_NT) {
      const int a = idx / K0_CH, t = idx - a * K0_CH;
      double2 v = make_double2(0.0, 0.0);
      if (t < cn) {
        const int q = c0 + t;
        const int x = xlo + q % nxi, y = ylo + q / nxi;
        v = phi_at(g, A, psi, mask, a, x, y, invH);
      }
      pa[a * K0_LD + 2 * t] = v.x;
      pa[a * K0_LD + 2 * t + 1] = v.y;
    }
    for (int idx = threadIdx.x; idx < nbc * K0_CH; idx += CK_NT) {
      const int b = idx / K0_CH, t = idx - b * K0_CH;
      double vx = 0.0, vy = 0.0;
      if (t < cn) {
        const int q = c0 + t;
        const int x = xlo + q % nxi, y = ylo + q / nxi;
        const int loc = (y - B.y0) * B.nxw + (x - B.x0);
        const double* wcol = W + B.w_off + (long long)b * 2 * nwB;
        vx = wcol[2 * loc];
        vy = wcol[2 * loc + 1];
      }
      wb[b * K0_LD + 2 * t] = vx;
      wb[b * K0_LD + 2 * t + 1] = vy;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < K0_TR; ++u) {
      const int tl = wave + 4 * u;
      const int R = tl / K0_TR, C = tl - (tl / K0_TR) * K0_TR;
      if (R < tra && C < trb) {
        const double* ap = pa + (16 * R + li) * K0_LD + lk;
        const double* bp = wb + (16 * C + li) * K0_LD + lk;
#pragma unroll
        for (int K = 0; K < 2 * K0_CH / 4; ++K)
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[4 * K], bp[4 * K], acc[u], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < K0_TR; ++u) {
    const int tl = wave + 4 * u;
    const int R = tl / K0_TR, C = tl - (tl / K0_TR) * K0_TR;
    if (R < tra && C < trb) {
      const int b = 16 * C + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 16 * R + lk + 4 * r;
        if (a < na && b < nbc) K0[(long long)(A.col0 + a) * ldk + (B.col0 + b)] = acc[u][r];
      }
    }
  }
}

// Symmetrise, scale to unit diagonal (s_j = 1/sqrt(K0_jj), 0 for empty
// columns, padding, the ndep dependent columns from dep_col and the columns
// flagged in drop (when given), so that their pivots are dropped).  One
// thread per entry.
__global__ void k_k0_scale_factors(const double* __restrict__ K0, int ldk,
                                   int nc, int dep_col, int ndep,
                                   const uint8_t* __restrict__ drop,
                                   double* __restrict__ sdiag) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ldk) return;
  double s = 0.0;
  if (j < nc && (j < dep_col || j >= dep_col + ndep) && !(drop != nullptr && drop[j])) {
    const double d = K0[(long long)j * ldk + j];
    if (d > 0.0 && finite(d)) s = 1.0 / sqrt(d);
  }
  sdiag[j] = s;
}

// K0 <- S ((K0 + K0^T) / 2) S, S = diag(sdiag), in place: one workgroup per
// pair of mirror tiles (K0T_T x K0T_T, the upper triangle's tiles in row
// order), both staged in LDS and written row-wise; entry (i, j) is
// 0.5 (K0_lo,hi + K0_hi,lo) s_lo s_hi (lo = min(i, j)), so the two halves
// get the same bits.  Used for the scaling and for undoing it.
constexpr int K0T_T = 32;
__global__ void __launch_bounds__(256)
k_k0_scale(double* __restrict__ K0, int ldk, const double* __restrict__ sdiag) {
  __shared__ double t1[K0T_T][K0T_T + 1], t2[K0T_T][K0T_T + 1];
  const int nt = ldk / K0T_T;
  long long p = blockIdx.x;
  int I = 0;
  while (p >= nt - I) {
    p -= nt - I;
    ++I;
  }
  const int J = I + (int)p;
  const int tx = threadIdx.x & (K0T_T - 1), ty = threadIdx.x / K0T_T;
  for (int r = ty; r < K0T_T; r += 256 / K0T_T) {
    t1[r][tx] = K0[(long long)(I * K0T_T + r) * ldk + J * K0T_T + tx];
    t2[r][tx] = K0[(long long)(J * K0T_T + r) * ldk + I * K0T_T + tx];
  }
  __syncthreads();
  auto put = [&](int i, int j, double a_lohi, double a_hilo) {
    const int lo = min(i, j), hi = max(i, j);
    K0[(long long)i * ldk + j] = 0.5 * (a_lohi + a_hilo) * sdiag[lo] * sdiag[hi];
  };
  for (int r = ty; r < K0T_T; r += 256 / K0T_T) {
    const int i = I * K0T_T + r, j = J * K0T_T + tx;
    if (i <= j) put(i, j, t1[r][tx], t2[tx][r]);
    else put(i, j, t2[tx][r], t1[r][tx]);
    if (I != J) put(J * K0T_T + r, I * K0T_T + tx, t1[tx][r], t2[r][tx]);
  }
}

static unsigned k0_scale_grid(int ldk) {
  const long long nt = ldk / K0T_T;
  return (unsigned)(nt * (nt + 1) / 2);
}

// Blocked Gauss-Jordan on the scaled K_0, block k: invert the 64 x 64
// diagonal block in LDS, dropping pivots <= tol (row and column zeroed).
// One pivot p = 16 PU + pt of the 64 x 64 diagonal block held as 4 x 4
// register tiles by 16 x 16 threads (rows ti + 16u, columns tj + 16w); PU is
// a compile-time constant, so the pivot's tile row and column are static.
// A pivot at or below tol (scaled matrix) is dropped: its row and column
// become zero, the rest is unchanged (a generalised inverse).  The owner
// of the next pivot forms its reciprocal during the current update and
// publishes it with the pivot row (0 for a dropped pivot), off the
// barrier-to-barrier path.  On entry nv / inv hold (on the pivot's owner,
// ti = tj = pt) the pivot and its reciprocal; on exit those of pivot p+1.
template <int PU>
__device__ __forceinline__ void gjp_pivot(double (&a)[4][4], int pt, int ti,
                                          int tj, double tol, double* pv,
                                          double& nv, double& inv,
                                          int* __restrict__ dropped,
                                          double* __restrict__ Lg,
                                          double* __restrict__ Dg) {
  const int p = 16 * PU + pt;
  double* rowv = pv + (p & 1) * 2 * GJB;
  double* colv = rowv + GJB;
  double* ipv = pv + 4 * GJB + (p & 1);
  const bool prow = ti == pt, pcol = tj == pt;
  if (prow) {
#pragma unroll
    for (int w = 0; w < 4; ++w) rowv[tj + 16 * w] = a[PU][w];
    if (pcol) {
      const bool dr = !(nv > tol) || !finite(nv);
      if (dr) atomicAdd(dropped, 1);
      *ipv = dr ? 0.0 : inv;
    }
  }
  if (pcol) {
#pragma unroll
    for (int u = 0; u < 4; ++u) colv[ti + 16 * u] = a[u][PU];
  }
  __syncthreads();
  const double ip = *ipv;
  const bool drop = ip == 0.0;
  double cv[4], rv[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) cv[u] = colv[ti + 16 * u];
#pragma unroll
  for (int w = 0; w < 4; ++w) rv[w] = rowv[tj + 16 * w] * ip;
  // the block's L D L^T, kept for the panels: column p of the unit lower L
  // is the pivot column below the pivot over the pivot (zero if dropped)
  if (pcol) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int row = ti + 16 * u;
      Lg[row * GJB + p] = row > p ? cv[u] * ip : 0.0;
    }
    if (prow) Dg[p] = ip;
  }
  // the entry of pivot p + 1 first: (PU, PU), or (PU + 1, PU + 1) after the
  // last pivot of this tile row
  constexpr int PN = PU + 1 < 4 ? PU + 1 : PU;
  const double e_pp = a[PU][PU] - cv[PU] * rv[PU];
  const double e_nn = a[PN][PN] - cv[PN] * rv[PN];
  nv = pt == 15 ? e_nn : e_pp;
  inv = 1.0 / nv;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const double upd = a[u][w] - cv[u] * rv[w];   // drop: rv = 0, unchanged
      if (u == PU && w == PU)
        a[u][w] = prow ? (pcol ? ip : (drop ? 0.0 : rv[w]))
                       : (pcol ? (drop ? 0.0 : -cv[u] * ip) : upd);
      else if (u == PU)
        a[u][w] = prow ? (drop ? 0.0 : rv[w]) : upd;
      else if (w == PU)
        a[u][w] = pcol ? (drop ? 0.0 : -cv[u] * ip) : upd;
      else
        a[u][w] = upd;
    }
}

template <int PU>
__device__ __forceinline__ void gjp_tile(double (&a)[4][4], int ti, int tj,
                                         double tol, double* pv, double& nv,
                                         double& inv, int* __restrict__ dropped,
                                         double* __restrict__ Lg,
                                         double* __restrict__ Dg) {
  for (int pt = 0; pt < 16; ++pt)
    gjp_pivot<PU>(a, pt, ti, tj, tol, pv, nv, inv, dropped, Lg, Dg);
}

// Block step kb, first part: P = GJ inverse (generalised) of the diagonal
// block, written over it, and the block's factors L D L^T (unit lower L
// row-major in LD[0 .. 4095], 1/D in LD[4096 .. 4159], 0 for a dropped
// pivot) for the panels.
__global__ void __launch_bounds__(CK_NT)
k_gj_pivot(double* __restrict__ A, int ld, int kb, double* __restrict__ LD,
           double tol, int* __restrict__ dropped, GjStride bs) {
  static_assert(GJB == 64 && CK_NT == 256, "pivot tiling: 16 x 16 threads, 4 x 4 tiles");
  __shared__ double pv[4 * GJB + 2];
  A += blockIdx.z * bs.a;
  LD += blockIdx.z * bs.ld;
  const int tid = threadIdx.x;
  const int tj = tid & 15, ti = tid >> 4;
  const long long base = (long long)kb * GJB;
  double* Lg = LD;
  double* Dg = LD + GJB * GJB;
  double a[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int w = 0; w < 4; ++w)
      a[u][w] = A[(base + ti + 16 * u) * ld + base + tj + 16 * w];
  double nv = a[0][0], inv = 1.0 / nv;
  gjp_tile<0>(a, ti, tj, tol, pv, nv, inv, dropped, Lg, Dg);
  gjp_tile<1>(a, ti, tj, tol, pv, nv, inv, dropped, Lg, Dg);
  gjp_tile<2>(a, ti, tj, tol, pv, nv, inv, dropped, Lg, Dg);
  gjp_tile<3>(a, ti, tj, tol, pv, nv, inv, dropped, Lg, Dg);
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int w = 0; w < 4; ++w)
      A[(base + ti + 16 * u) * ld + base + tj + 16 * w] = a[u][w];
}

// Block step kb, second part, for every other block index ib: the block
// column A_ik and the block row A_ki are transformed by substitution with
// the pivot block's factors instead of by products with its explicit
// inverse P = L^-T D^-1 L^-1.  Multiplying by an explicit P amplifies the
// rounding of its entries by cond(A_kk), which reaches 1e8 in the soft
// region of a high-contrast K_0; substitution repeats the arithmetic of
// pivot-by-pivot Gauss-Jordan.  Lane v of wave 0 takes row v of A_ik, lane
// v of wave 1 column v of A_ki (a 64-vector a, in registers):
//   w = a L^-T (forward substitution), y = w D^-1, x = y L^-1 (backward);
// then A_ik <- -x (rows), A_ki <- x^T (columns), and for the update
// Lp_i = y (rows) and Rp_i = w^T (columns), so that
// A_ij - A_ik P A_kj = A_ij - Lp_i Rp_j.
constexpr int GJP_NT = 128;
__global__ void __launch_bounds__(GJP_NT)
k_gj_panel(double* __restrict__ A, int ld, int kb, int b0,
           const double* __restrict__ LD, double* __restrict__ Lp,
           double* __restrict__ Rp, GjStride bs) {
  __shared__ double Ls[GJB * GJB];
  __shared__ double Di[GJB];
  const int ib = b0 + blockIdx.x;
  if (ib == kb) return;
  A += blockIdx.z * bs.a;
  LD += blockIdx.z * bs.ld;
  Lp += blockIdx.z * bs.p;
  Rp += blockIdx.z * bs.p;
  const int tid = threadIdx.x;
  for (int q = tid; q < GJB * GJB; q += GJP_NT) Ls[q] = LD[q];
  if (tid < GJB) Di[tid] = LD[GJB * GJB + tid];
  const long long kbase = (long long)kb * GJB, ibase = (long long)ib * GJB;
  const bool colv = tid < GJB;               // wave 0: rows of A_ik
  const int v = tid & (GJB - 1);
  double a[GJB];
  if (colv) {
    const double2* src = reinterpret_cast<const double2*>(A + (ibase + v) * ld + kbase);
#pragma unroll
    for (int t = 0; t < GJB / 2; ++t) {
      const double2 q = src[t];
      a[2 * t] = q.x;
      a[2 * t + 1] = q.y;
    }
  } else {
#pragma unroll
    for (int t = 0; t < GJB; ++t) a[t] = A[(kbase + t) * ld + ibase + v];
  }
  __syncthreads();
  // w = a L^-T: w_t = a_t - sum_{s<t} w_s L_ts, in pivot order
#pragma unroll
  for (int t = 1; t < GJB; ++t) {
    double acc = a[t];
#pragma unroll
    for (int s = 0; s + 1 < t; s += 2) {
      const double2 l = *reinterpret_cast<const double2*>(Ls + t * GJB + s);
      acc = fma(-a[s], l.x, acc);
      acc = fma(-a[s + 1], l.y, acc);
    }
    if (t & 1) acc = fma(-a[t - 1], Ls[t * GJB + t - 1], acc);
    a[t] = acc;
  }
  if (!colv) {
#pragma unroll
    for (int t = 0; t < GJB; ++t) Rp[(long long)t * ld + ibase + v] = a[t];
  }
#pragma unroll
  for (int t = 0; t < GJB; ++t) a[t] *= Di[t];
  if (colv) {
    double2* dst = reinterpret_cast<double2*>(Lp + (ibase + v) * GJB);
#pragma unroll
    for (int t = 0; t < GJB / 2; ++t) dst[t] = make_double2(a[2 * t], a[2 * t + 1]);
  }
  // x = y L^-1: x_s = y_s - sum_{t>s} x_t L_ts, right-looking from the last
#pragma unroll
  for (int t = GJB - 1; t > 0; --t) {
    const double xt = a[t];
#pragma unroll
    for (int s = 0; s + 1 < t; s += 2) {
      const double2 l = *reinterpret_cast<const double2*>(Ls + t * GJB + s);
      a[s] = fma(-xt, l.x, a[s]);
      a[s + 1] = fma(-xt, l.y, a[s + 1]);
    }
    if (t & 1) a[t - 1] = fma(-xt, Ls[t * GJB + t - 1], a[t - 1]);
  }
  if (colv) {
    double2* dst = reinterpret_cast<double2*>(A + (ibase + v) * ld + kbase);
#pragma unroll
    for (int t = 0; t < GJB / 2; ++t) dst[t] = make_double2(-a[2 * t], -a[2 * t + 1]);
  } else {
#pragma unroll
    for (int t = 0; t < GJB; ++t) A[(kbase + t) * ld + ibase + v] = a[t];
  }
}

// Block step kb, last part: A_ij -= Lp_i Rp_j for the tiles outside block
// row and column kb (those were written by the first two parts).  Grid
// (nblk, nblk) of 64 x 64 tiles from block b0 (0: the whole matrix).
__global__ void __launch_bounds__(CK_NT)
k_gj_update(double* __restrict__ A, int ld, int kb, int b0,
            const double* __restrict__ Lp, const double* __restrict__ Rp,
            GjStride bs) {
  __shared__ double Ls[GJB * (GJB + 1)];
  __shared__ double Rs[GJB * (GJB + 1)];
  const int ib = b0 + blockIdx.y, jb = b0 + blockIdx.x;
  if (ib == kb || jb == kb) return;
  A += blockIdx.z * bs.a;
  Lp += blockIdx.z * bs.p;
  Rp += blockIdx.z * bs.p;
  const int tid = threadIdx.x;
  const long long ibase = (long long)ib * GJB, jbase = (long long)jb * GJB;
  // The product on FP64 matrix cores: wave w takes rows 16w..16w+15 of the
  // tile and all four 16-column tiles; per MFMA 16x16x4, lane l supplies
  // Ls(16w + l%16, 4K + l/16) and Rs(4K + l/16, 16C + l%16) and holds
  // C(16w + l/16 + 4r, 16C + l%16) in register r.  The accumulators start
  // from this lane's entries of A_ij and Ls holds -Lp_i, so the 64 pivots'
  // terms are subtracted from A_ij in pivot order, four at a time (as the
  // pivot-by-pivot elimination does) rather than summed first.
  const int wave = tid >> 6, li = tid & 15, lk = (tid & 63) >> 4;
  k0_d4 acc[4];
#pragma unroll
  for (int C = 0; C < 4; ++C)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      acc[C][r] = A[(ibase + 16 * wave + lk + 4 * r) * ld + jbase + 16 * C + li];
  for (int idx = tid; idx < GJB * GJB; idx += CK_NT) {
    const int i = idx / GJB, j = idx - i * GJB;
    Ls[i * (GJB + 1) + j] = -Lp[(ibase + i) * GJB + j];
    Rs[i * (GJB + 1) + j] = Rp[(long long)i * ld + jbase + j];
  }
  __syncthreads();
  static_assert(GJB == 64 && CK_NT == 256, "four waves of 16-row strips");
  const double* la = Ls + (16 * wave + li) * (GJB + 1) + lk;
  const double* rb = Rs + lk * (GJB + 1) + li;
#pragma unroll 4
  for (int K = 0; K < GJB / 4; ++K) {
    const double av = la[4 * K];
#pragma unroll
    for (int C = 0; C < 4; ++C)
      acc[C] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, rb[4 * K * (GJB + 1) + 16 * C], acc[C], 0, 0, 0);
  }
#pragma unroll
  for (int C = 0; C < 4; ++C)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      A[(ibase + 16 * wave + lk + 4 * r) * ld + jbase + 16 * C + li] = acc[C][r];
}


// ---------------------------------------------------------------------
// Restriction c = R_0 r: RS_CH workgroups per coarse node, each over a
// band of rows of the neighbourhood.  A thread reads r, the mask and chi
// once per node and accumulates every column of the node in registers
// (coalesced psi reads); column sums are a wavefront butterfly and a
// fixed-order sum over the waves, written per band to cpart[band][col].
// The psi loads of RS_JC modes at all of a thread's nodes are issued
// together (indices clamped into the valid range, extra modes dropped), and
// the first chunk together with the loads of r, so that a workgroup waits
// for HBM about once per chunk rather than once per mode.
constexpr int RS_NT = 256;
constexpr int RS_CH = 4;       // bands of neighbourhood rows per coarse node
constexpr int RS_NPT = 6;      // band nodes per thread (band <= RS_NT*RS_NPT)
constexpr int RS_JC = 8;       // modes per load chunk
constexpr int KMAXD = 24;

struct RsLds {
  double red[(2 * KMAXD + 1) * (RS_NT / 64)];
  double redc[RS_NT / 64 + 1];
  int shi;
};

// the heat modes in the element type T: FP64, or the FP32 copy of the
// FP32-local path (the same rounded values)
template <typename T> __device__ __forceinline__ const T* psi_of(const double* p, const float* p32);
template <> __device__ __forceinline__ const double* psi_of<double>(const double* p, const float*) { return p; }
template <> __device__ __forceinline__ const float* psi_of<float>(const double*, const float* p32) { return p32; }

// Workgroup bid = (coarse node, band): partial restriction of r.
template <typename T>
__device__ __forceinline__ void restrict_body(const RestrictArgs& a, int bid,
                                              RsLds& L) {
  const Geom& g = a.g;
  const uint8_t* __restrict__ mask = a.mask;
  const double* __restrict__ r = a.r;
  const double invH = a.invH;
  double* red = L.red;
  // the coarse node's descriptor is read alongside the stop test
  const CoarseNode cn = a.cn[bid / RS_CH];
  if (a.sc != nullptr) {
    if (a.check) {
      if (cg_check_done<RS_NT>(a.sc, a.part_upd, a.nb_upd, L.redc, &L.shi, bid == 0)) return;
    } else if (block_read_done(a.sc, &L.shi)) {
      return;
    }
  }
  const int band = bid % RS_CH;
  const int nm = cn.nmodes;
  const int ncol = 2 * nm + cn.nrot;
  if (ncol == 0) return;
  const int nw = cn.nxw * cn.nyw;
  const int r0w = (band * cn.nyw) / RS_CH, r1w = ((band + 1) * cn.nyw) / RS_CH;
  const int lo = r0w * cn.nxw, hi = r1w * cn.nxw;
  const T* ps = psi_of<T>(a.psi, a.psi32) + cn.psi_off;
  // this thread's nodes of the band (past the band's end: its first node,
  // weighted 0)
  int locs[RS_NPT];
  bool okp[RS_NPT];
#pragma unroll
  for (int p = 0; p < RS_NPT; ++p) {
    const int loc = lo + threadIdx.x + p * RS_NT;
    okp[p] = loc < hi;
    locs[p] = okp[p] ? loc : lo;
  }
  constexpr int JC = RS_JC;
  T pv[JC][RS_NPT];       // in the element type: FP32 halves the registers
  auto load_chunk = [&](int j0) {
#pragma unroll
    for (int u = 0; u < JC; ++u) {
      const long long j = min(j0 + u, nm - 1);
#pragma unroll
      for (int p = 0; p < RS_NPT; ++p) pv[u][p] = ps[j * nw + locs[p]];
    }
  };
  load_chunk(0);
  // masked chi*r at the nodes, and the rotation column's partial sum
  double r0[RS_NPT], r1[RS_NPT];
  double ar = 0.0;
#pragma unroll
  for (int p = 0; p < RS_NPT; ++p) {
    const int x = cn.x0 + locs[p] % cn.nxw, y = cn.y0 + locs[p] / cn.nxw;
    const double chi = chi_at(g, cn.cx, cn.cy, x, y);
    const long long node = (long long)y * g.nnx + x;
    const double2 rv = reinterpret_cast<const double2*>(r)[node];
    const uchar2 m = reinterpret_cast<const uchar2*>(mask)[node];
    r0[p] = (!okp[p] || m.x) ? 0.0 : chi * rv.x;
    r1[p] = (!okp[p] || m.y) ? 0.0 : chi * rv.y;
    const double rx = (x - cn.cx * g.sx) * g.h * invH;
    const double ry = (y - cn.cy * g.sy) * g.h * invH;
    ar += -ry * r0[p] + rx * r1[p];
  }
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < (KMAXD + JC - 1) / JC; ++c) {
    const int j0 = c * JC;
    if (j0 >= nm) break;
    if (c > 0) load_chunk(j0);
#pragma unroll
    for (int u = 0; u < JC; ++u) {
      const int j = j0 + u;
      if (j < nm) {
        double ax = 0.0, ay = 0.0;
#pragma unroll
        for (int p = 0; p < RS_NPT; ++p) {
          ax += (double)pv[u][p] * r0[p];
          ay += (double)pv[u][p] * r1[p];
        }
        const double sx = wave_sum(ax);
        const double sy = wave_sum(ay);
        if ((threadIdx.x & 63) == 0) {
          red[j * (RS_NT / 64) + w] = sx;
          red[(nm + j) * (RS_NT / 64) + w] = sy;
        }
      }
    }
  }
  if (cn.nrot) {
    const double sr = wave_sum(ar);
    if ((threadIdx.x & 63) == 0) red[(2 * nm) * (RS_NT / 64) + w] = sr;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < ncol; j += RS_NT) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < RS_NT / 64; ++q) t += red[j * (RS_NT / 64) + q];
    a.cpart[(long long)band * a.ldc + cn.col0 + j] = t;
  }
}

// one kernel per element type, so that the FP32 one keeps few enough
// registers for three workgroups per CU
template <typename T>
__global__ void __launch_bounds__(RS_NT, sizeof(T) == 4 ? 3 : 2) k_restrict(RestrictArgs a) {
  __shared__ RsLds L;
  restrict_body<T>(a, blockIdx.x, L);
}

__global__ void __launch_bounds__(RS_NT)
k_restrict_batch(const RestrictArgs* __restrict__ tab, const int* __restrict__ start,
                 int nent) {
  __shared__ RsLds L;
  const int e = batch_entry(start, nent, blockIdx.x);
  if (tab[e].psi32 != nullptr)
    restrict_body<float>(tab[e], blockIdx.x - start[e], L);
  else
    restrict_body<double>(tab[e], blockIdx.x - start[e], L);
}

// c0 = K_0^+ c with c the sum of the restriction's band partials.  Rows of
// K_0^+ are split over many small workgroups so that every CU streams a few
// rows; each workgroup first sums the bands into LDS (fixed order).  One
// wave per GV_RPW rows, four independent accumulators per lane.
constexpr int GV_NT = 256;
constexpr int GV_RPW = 2;                               // rows per wave
constexpr int GV_ROWS = (GV_NT / 64) * GV_RPW;          // rows per workgroup
constexpr int GV_MAXC = 12288;
constexpr int GV_U = 32;                                // row columns a lane loads at once

struct GvLds {
  double cl[GV_MAXC];
  int shi;
};

__device__ __forceinline__ void gemv_body(const GemvArgs& a, int bid, GvLds& L) {
  const double* __restrict__ K0 = a.K0;
  const int ldk = a.ldk, nc = a.nc, ldc = a.ldc;
  const double* __restrict__ cpart = a.cpart;
  double* cl = L.cl;
  static_assert(GV_RPW == 2, "the row loop pairs two rows");
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r0 = bid * GV_ROWS + wave * GV_RPW, r1 = r0 + 1;
  const bool has0 = r0 < nc, has1 = r1 < nc;
  const double* k0 = K0 + (long long)(has0 ? r0 : 0) * ldk;
  const double* k1 = K0 + (long long)(has1 ? r1 : (has0 ? r0 : 0)) * ldk;
  // The wave's two rows (GV_U columns a lane at a time), the band partials
  // of c and the done word all go out before the first use, so that for
  // nc <= 64 GV_U the kernel waits for memory once.
  double kv0[GV_U], kv1[GV_U];
  auto load_rows = [&](int jb) {
#pragma unroll
    for (int u = 0; u < GV_U; ++u) {
      const int j = jb + lane + 64 * u;
      const bool ok = j < nc;
      kv0[u] = ok ? k0[j] : 0.0;
      kv1[u] = ok ? k1[j] : 0.0;
    }
  };
  // c = sum of the band partials (fixed order) into LDS, GV_CC columns per
  // thread at a time with all their loads issued together
  constexpr int GV_CC = 8;
  double v[GV_CC][RS_CH];
  auto load_c = [&](int j0) {
#pragma unroll
    for (int u = 0; u < GV_CC; ++u) {
      const int j = min(j0 + (int)threadIdx.x + u * GV_NT, nc - 1);
#pragma unroll
      for (int b = 0; b < RS_CH; ++b) v[u][b] = cpart[(long long)b * ldc + j];
    }
  };
  load_rows(0);
  load_c(0);
  if (a.sc != nullptr && block_read_done(a.sc, &L.shi)) return;
  for (int j0 = 0; j0 < nc; j0 += GV_CC * GV_NT) {
    if (j0 > 0) load_c(j0);
#pragma unroll
    for (int u = 0; u < GV_CC; ++u) {
      const int j = j0 + threadIdx.x + u * GV_NT;
      double t = 0.0;
#pragma unroll
      for (int b = 0; b < RS_CH; ++b) t += v[u][b];
      if (j < nc) cl[j] = t;
    }
  }
  __syncthreads();
  if (!has0) return;
  // column j = jb + lane + 64 u into accumulator u % 4
  double s[4] = {0.0, 0.0, 0.0, 0.0}, t[4] = {0.0, 0.0, 0.0, 0.0};
  for (int jb = 0; jb < nc; jb += 64 * GV_U) {
    if (jb > 0) load_rows(jb);
#pragma unroll
    for (int u = 0; u < GV_U; ++u) {
      const int j = jb + lane + 64 * u;
      const double c = j < nc ? cl[j] : 0.0;
      s[u & 3] += kv0[u] * c;
      t[u & 3] += kv1[u] * c;
    }
  }
  const double sa = wave_sum((s[0] + s[1]) + (s[2] + s[3]));
  const double sb = wave_sum((t[0] + t[1]) + (t[2] + t[3]));
  if (lane == 0) {
    a.c0[r0] = sa;
    if (has1) a.c0[r1] = sb;
  }
}

__global__ void __launch_bounds__(GV_NT) k_coarse_gemv(GemvArgs a) {
  __shared__ GvLds L;
  gemv_body(a, blockIdx.x, L);
}

__global__ void __launch_bounds__(GV_NT)
k_coarse_gemv_batch(const GemvArgs* __restrict__ tab, const int* __restrict__ start,
                    int nent) {
  __shared__ GvLds L;
  const int e = batch_entry(start, nent, blockIdx.x);
  gemv_body(tab[e], blockIdx.x - start[e], L);
}

// MODE 0: plain apply.  MODE 1 (CG iteration) and 2 (CG start): also the
// partial sums of r.z and, flexible, z.q per workgroup, read by the next
// iteration's stiffness and update kernels; in MODE 1 workgroup 0 advances
// the iteration counter.
// Combination z = (first-level part + coarse part) on free DOFs, with the
// CG partials.  One workgroup per (coarse cell, band of the cell's node
// rows): cell (cx, cy) owns the nodes x in [cx S, cx S + S) (the last cell
// column also x = nx), likewise in y.  Everything that can touch those
// nodes is the same for the whole workgroup and is staged in LDS first: the
// subdomains of the 3 x 3 block of subdomain-grid cells around the cell
// (a node lies in at most 4 of them) and the cell's four corner coarse
// nodes with their coefficients c0.  The per-node loads (local solutions,
// psi of every corner's modes, r, q) then go out together.
constexpr int CB_NT = 256;
constexpr int CB_JC = 8;                      // modes per load chunk
constexpr int CB_NCOL = 2 * KMAXD + 1;        // columns of one coarse node

struct CbLds {
  double red[CB_NT / 64 + 1];
  double c0[4][CB_NCOL];
  long long svoff[9];
  long long cpsi[4];
  int sx0[9], sy0[9], snx[9], sny[9];
  int cx0[4], cy0[4], cnxw[4], cnw[4], cnm[4], crot[4], ccol[4];
  int shi;
};

// rows of a cell per workgroup, and bands per cell
__host__ __device__ inline int cb_rows(const Geom& g) { return CB_NT / (g.sx + 1); }
__host__ __device__ inline int cb_bands(const Geom& g) {
  return (g.sy + 1 + cb_rows(g) - 1) / cb_rows(g);
}

template <int MODE, typename T>
__device__ __forceinline__ void combine_body(const CombineCall& a, int bid,
                                             int nblk, CbLds& L) {
  const Geom& g = a.g;
  const CombineArgs& ca = a.ca;
  const uint8_t* __restrict__ mask = a.mask;
  CGScalars* sc = a.sc;
  const int tid = threadIdx.x;
  const int ncellx = g.nx / g.sx, ncelly = g.ny / g.sy;
  const int nbands = cb_bands(g), rpb = cb_rows(g);
  const int cell = bid / nbands, band = bid - (bid / nbands) * nbands;
  const int cx = cell % ncellx, cy = cell / ncellx;
  const int wx = g.sx + (cx == ncellx - 1 ? 1 : 0);
  const int wy = g.sy + (cy == ncelly - 1 ? 1 : 0);
  const int ty = band * rpb + tid / wx, tx = tid - (tid / wx) * wx;
  const bool act = tid < rpb * wx && ty < wy;
  // idle threads stand on the cell's first node (valid addresses, no output)
  const int x = cx * g.sx + (act ? tx : 0), y = cy * g.sy + (act ? ty : 0);
  const long long node = (long long)y * g.nnx + x;
  // Every read that needs no staged value goes out at once: the done word,
  // the candidates (empty boxes / no modes where there are none) and the
  // node's mask, r and (flexible) q.
  int dn = DONE_RUNNING;
  if (MODE != 0 && tid == 0)
    dn = __hip_atomic_load(&sc->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (tid < 9) {
    const int gy = cy - 1 + tid / 3, gx = cx - 1 + tid % 3;
    SysDesc sd{};
    if (ca.use_l1 && gx >= 0 && gx < ca.ngx && gy >= 0 && gy < ca.ngy)
      sd = ca.sys_grid[gy * ca.ngx + gx];
    L.sx0[tid] = sd.x0;
    L.sy0[tid] = sd.y0;
    L.snx[tid] = sd.nxb;
    L.sny[tid] = sd.nyb;
    L.svoff[tid] = sd.voff;
  } else if (tid >= 64 && tid < 68) {
    const int k = tid - 64;
    CoarseNode cn{};
    if (ca.use_coarse) cn = ca.cnodes[(cy + (k >> 1)) * g.ncx + cx + (k & 1)];
    const bool on = ca.use_coarse && (2 * cn.nmodes + cn.nrot) > 0;
    L.cx0[k] = cn.x0;
    L.cy0[k] = cn.y0;
    L.cnxw[k] = cn.nxw;
    L.cnw[k] = cn.nxw * cn.nyw;
    L.cnm[k] = on ? cn.nmodes : 0;
    L.crot[k] = on ? cn.nrot : 0;
    L.ccol[k] = cn.col0;
    L.cpsi[k] = cn.psi_off;
  }
  uchar2 mk = reinterpret_cast<const uchar2*>(mask)[node];
  double2 rv = make_double2(0.0, 0.0), qv = make_double2(0.0, 0.0);
  if (MODE != 0) {
    rv = reinterpret_cast<const double2*>(a.r)[node];
    if (MODE == 1 && a.flex) qv = reinterpret_cast<const double2*>(a.q)[node];
  }
  if (tid == 0) L.shi = dn;
  __syncthreads();
  if (MODE != 0 && L.shi != DONE_RUNNING) return;
  for (int idx = tid; idx < 4 * CB_NCOL; idx += CB_NT) {
    const int k = idx / CB_NCOL, j = idx - (idx / CB_NCOL) * CB_NCOL;
    if (j < 2 * L.cnm[k] + L.crot[k]) L.c0[k][j] = ca.c0[L.ccol[k] + j];
  }
  // first level: the subdomains that contain the node, in candidate order
  // (at most four: the geometry guarantees it)
  long long li0 = 0, li1 = 0, li2 = 0, li3 = 0;
  int nh = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int sx = L.sx0[k], sy = L.sy0[k];
    if (x >= sx && x < sx + L.snx[k] && y >= sy && y < sy + L.sny[k]) {
      const long long li = L.svoff[k] + 2 * ((long long)(y - sy) * L.snx[k] + (x - sx));
      li0 = nh == 0 ? li : li0;
      li1 = nh == 1 ? li : li1;
      li2 = nh == 2 ? li : li2;
      li3 = nh == 3 ? li : li3;
      ++nh;
    }
  }
  const double2* ls = reinterpret_cast<const double2*>(ca.lsol);
  double2 lv0 = make_double2(0.0, 0.0), lv1 = lv0, lv2 = lv0, lv3 = lv0;
  if (nh > 0) lv0 = ls[li0 >> 1];
  if (nh > 1) lv1 = ls[li1 >> 1];
  if (nh > 2) lv2 = ls[li2 >> 1];
  if (nh > 3) lv3 = ls[li3 >> 1];
  // coarse part: every corner's modes at this node, one chunk of JC modes of
  // all four corners at a time (the first chunk goes out with the loads above)
  constexpr int JC = CB_JC;
  T pv[4][JC];
  const T* pp[4];
  int nmk[4];
  auto load_chunk = [&](int j0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (j0 < nmk[k]) {
#pragma unroll
        for (int u = 0; u < JC; ++u)
          pv[k][u] = pp[k][(long long)min(j0 + u, nmk[k] - 1) * L.cnw[k]];
      }
    }
  };
  int nmax = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    nmk[k] = L.cnm[k];
    nmax = max(nmax, nmk[k]);
    pp[k] = psi_of<T>(ca.psi, ca.psi32) + L.cpsi[k] + (long long)(y - L.cy0[k]) * L.cnxw[k] +
            (x - L.cx0[k]);
  }
  load_chunk(0);
  __syncthreads();
  double z0 = 0.0, z1 = 0.0;
  z0 += lv0.x;
  z1 += lv0.y;
  z0 += lv1.x;
  z1 += lv1.y;
  z0 += lv2.x;
  z1 += lv2.y;
  z0 += lv3.x;
  z1 += lv3.y;
  double s0[4] = {0.0, 0.0, 0.0, 0.0}, s1[4] = {0.0, 0.0, 0.0, 0.0};
  for (int j0 = 0; j0 < nmax; j0 += JC) {
    if (j0 > 0) load_chunk(j0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int nm = nmk[k];
      if (j0 >= nm) continue;
      const double* c = L.c0[k];
#pragma unroll
      for (int u = 0; u < JC; ++u) {
        const double w = j0 + u < nm ? pv[k][u] : 0.0;
        s0[k] += w * c[min(j0 + u, nm - 1)];
        s1[k] += w * c[nm + min(j0 + u, nm - 1)];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int nm = nmk[k];
    if (nm == 0) continue;
    const int ccx = cx + (k & 1), ccy = cy + (k >> 1);
    const double chi = chi_at(g, ccx, ccy, x, y);
    const double* c = L.c0[k];
    double t0 = s0[k] * chi, t1 = s1[k] * chi;
    if (L.crot[k]) {
      const double rx = (x - ccx * g.sx) * g.h * ca.invH;
      const double ry = (y - ccy * g.sy) * g.h * ca.invH;
      const double cr = c[2 * nm];
      t0 += -chi * ry * cr;
      t1 += chi * rx * cr;
    }
    z0 += t0;
    z1 += t1;
  }
  if (act && a.zadd != nullptr) {
    const double2 za = reinterpret_cast<const double2*>(a.zadd)[node];
    z0 += za.x;
    z1 += za.y;
  }
  if (mk.x) z0 = 0.0;
  if (mk.y) z1 = 0.0;
  if (act) reinterpret_cast<double2*>(a.z)[node] = make_double2(z0, z1);
  if (MODE == 0) return;
  double d_rz = 0.0, d_zq = 0.0;
  if (act) {
    d_rz = rv.x * z0 + rv.y * z1;
    if (MODE == 1 && a.flex) d_zq = qv.x * z0 + qv.y * z1;
  }
  const double s_rz = block_sum<CB_NT>(d_rz, L.red);
  const double s_zq = block_sum<CB_NT>(d_zq, L.red);
  if (tid == 0) {
    a.part[bid] = s_rz;
    a.part[nblk + bid] = s_zq;
    if (MODE == 1 && bid == 0) sc->iter = sc->iter + 1;
  }
}

template <int MODE>
__global__ void __launch_bounds__(CB_NT) k_combine(CombineCall a) {
  __shared__ CbLds L;
  if (a.ca.psi32 != nullptr)
    combine_body<MODE, float>(a, blockIdx.x, gridDim.x, L);
  else
    combine_body<MODE, double>(a, blockIdx.x, gridDim.x, L);
}

__global__ void __launch_bounds__(CB_NT)
k_combine_cg_batch(const CombineCall* __restrict__ tab, const int* __restrict__ start,
                   int nent) {
  __shared__ CbLds L;
  const int e = batch_entry(start, nent, blockIdx.x);
  if (tab[e].ca.psi32 != nullptr)
    combine_body<1, float>(tab[e], blockIdx.x - start[e], start[e + 1] - start[e], L);
  else
    combine_body<1, double>(tab[e], blockIdx.x - start[e], start[e + 1] - start[e], L);
}

// Dense export of the coarse basis (column-major n x Nc).
__global__ void __launch_bounds__(CK_NT)
k_export_basis(Geom g, const CoarseNode* __restrict__ cnodes,
               const int* __restrict__ col_node,
               const uint8_t* __restrict__ mask, const double* __restrict__ psi,
               double* __restrict__ out, double invH) {
  const int col = blockIdx.y;
  const int l = col_node[col];
  const CoarseNode cn = cnodes[l];
  const int lc = col - cn.col0;
  const long long nn = (long long)g.nnx * g.nny;
  const long long node = (long long)blockIdx.x * CK_NT + threadIdx.x;
  if (node >= nn) return;
  const int x = (int)(node % g.nnx), y = (int)(node / g.nnx);
  const double2 v = phi_at(g, cn, psi, mask, lc, x, y, invH);
  out[(long long)col * 2 * nn + 2 * node] = v.x;
  out[(long long)col * 2 * nn + 2 * node + 1] = v.y;
}

// ---------------------------------------------------------------- launchers

void launch_coarse_kphi(const Geom& g, const CoarseNode* cn, const int* col_node,
                        int ncols, const double* Ke, const double* E,
                        const uint8_t* mask, const double* psi, double* W,
                        double invH, hipStream_t s) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_coarse_kphi, dim3(ncols), dim3(CK_NT), 0, s, g, cn,
                     col_node, Ke, E, mask, psi, W, invH);
}

void launch_coarse_k0(const Geom& g, const CoarseNode* cn, const int2* pairs,
                      int npairs, const uint8_t* mask, const double* psi,
                      const double* W, double* K0, int ldk, double invH,
                      hipStream_t s) {
  if (npairs <= 0) return;
  hipLaunchKernelGGL(k_coarse_k0, dim3(npairs), dim3(CK_NT), 0, s, g, cn, pairs,
                     mask, psi, W, K0, ldk, invH);
}

// The block steps of the Gauss-Jordan elimination on nmat matrices of
// order ld (a multiple of 64) at once: matrix z at A + z bs.a, its pivot
// factors at LD + z bs.ld (4160 doubles each), its panels at Lp + z bs.p and
// Rp + z bs.p (64 ld doubles each).
void launch_gj_steps(double* A, int ld, int nmat, GjStride bs, double* LD,
                     double* Lp, double* Rp, double tol, int* dropped,
                     hipStream_t s) {
  const int nblk = ld / GJB;
  for (int kb = 0; kb < nblk; ++kb) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(1, 1, nmat), dim3(CK_NT), 0, s, A, ld,
                       kb, LD, tol, dropped, bs);
    hipLaunchKernelGGL(k_gj_panel, dim3(nblk, 1, nmat), dim3(GJP_NT), 0, s, A,
                       ld, kb, 0, LD, Lp, Rp, bs);
    hipLaunchKernelGGL(k_gj_update, dim3(nblk, nblk, nmat), dim3(CK_NT), 0, s,
                       A, ld, kb, 0, Lp, Rp, bs);
  }
}

// Block LDL^T of a block-tridiagonal matrix (slab k: blocks [sb[k],
// sb[k+1]) of 64 columns) by windowed Gauss-Jordan: slab k's pivot blocks
// are eliminated with the panel and update steps restricted to the window
// of slabs k and k+1.  Afterwards slab k's diagonal block holds the
// (generalised) inverse G_k of its Schur complement S_k, the block right of
// it G_k C_k and the block below it -C_k^T G_k (C_k the coupling of slab k
// with slab k+1), and slab k+1's diagonal block has received
// -C_k^T G_k C_k.
void launch_gj_slabs(double* A, int ld, const int* sb, int nslab, double* LD,
                     double* Lp, double* Rp, double tol, int* dropped,
                     hipStream_t s) {
  const GjStride bs{0, 0, 0};
  for (int k = 0; k < nslab; ++k) {
    const int w0 = sb[k], w1 = sb[std::min(k + 2, nslab)];
    const int nw = w1 - w0;
    for (int kb = sb[k]; kb < sb[k + 1]; ++kb) {
      hipLaunchKernelGGL(k_gj_pivot, dim3(1, 1, 1), dim3(CK_NT), 0, s, A, ld, kb, LD,
                         tol, dropped, bs);
      hipLaunchKernelGGL(k_gj_panel, dim3(nw, 1, 1), dim3(GJP_NT), 0, s, A, ld, kb,
                         w0, LD, Lp, Rp, bs);
      hipLaunchKernelGGL(k_gj_update, dim3(nw, nw, 1), dim3(CK_NT), 0, s, A, ld, kb,
                         w0, Lp, Rp, bs);
    }
  }
}

void launch_k0_pinv(double* K0, int ldk, int nc, int dep_col, int ndep,
                    const uint8_t* drop, double* sdiag, double* P, double* Lp,
                    double* Rp, double tol, int* dropped, hipStream_t s) {
  hipLaunchKernelGGL(k_k0_scale_factors, dim3((ldk + 255) / 256), dim3(256), 0,
                     s, K0, ldk, nc, dep_col, ndep, drop, sdiag);
  hipLaunchKernelGGL(k_k0_scale, dim3(k0_scale_grid(ldk)), dim3(256), 0, s, K0, ldk, sdiag);
  launch_gj_steps(K0, ldk, 1, GjStride{0, 0, 0}, P, Lp, Rp, tol, dropped, s);
  // undo the scaling: the same symmetric product with S
  hipLaunchKernelGGL(k_k0_scale, dim3(k0_scale_grid(ldk)), dim3(256), 0, s, K0, ldk, sdiag);
}

void launch_gj_slabs(double*, int, const int*, int, double*, double*, double*, double,
                     int*, hipStream_t);

// Scaled block LDL^T of a block-tridiagonal K_0 (3D, slabs of coarse
// nodes): unit-diagonal scaling (zero for padding, empty and flagged
// columns), then the windowed Gauss-Jordan over the slabs; the factors stay
// scaled (the solve applies sdiag on both sides).
void launch_k0_slab_factor(double* K0, int ldk, const int* sb, int nslab,
                           const uint8_t* drop, double* sdiag, double* P, double* Lp,
                           double* Rp, double tol, int* dropped, hipStream_t s) {
  hipLaunchKernelGGL(k_k0_scale_factors, dim3((ldk + 255) / 256), dim3(256), 0,
                     s, K0, ldk, ldk, -1, 0, drop, sdiag);
  hipLaunchKernelGGL(k_k0_scale, dim3(k0_scale_grid(ldk)), dim3(256), 0, s, K0, ldk, sdiag);
  launch_gj_slabs(K0, ldk, sb, nslab, P, Lp, Rp, tol, dropped, s);
}

void launch_restrict(const RestrictArgs& a, int ncn, hipStream_t s) {
  if (a.psi32 != nullptr)
    hipLaunchKernelGGL(k_restrict<float>, dim3(ncn * RS_CH), dim3(RS_NT), 0, s, a);
  else
    hipLaunchKernelGGL(k_restrict<double>, dim3(ncn * RS_CH), dim3(RS_NT), 0, s, a);
}

void launch_restrict_batch(const RestrictArgs* tab, const int* start, int nent,
                           int total, hipStream_t s) {
  hipLaunchKernelGGL(k_restrict_batch, dim3(total), dim3(RS_NT), 0, s, tab, start, nent);
}

int restrict_bands() { return RS_CH; }
int restrict_max_band_nodes() { return RS_NT * RS_NPT; }

int gemv_blocks(int nc) { return nc > 0 ? (nc + GV_ROWS - 1) / GV_ROWS : 0; }

void launch_coarse_gemv(const GemvArgs& a, hipStream_t s) {
  if (a.nc <= 0) return;
  hipLaunchKernelGGL(k_coarse_gemv, dim3(gemv_blocks(a.nc)), dim3(GV_NT), 0, s, a);
}

void launch_coarse_gemv_batch(const GemvArgs* tab, const int* start, int nent,
                              int total, hipStream_t s) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_coarse_gemv_batch, dim3(total), dim3(GV_NT), 0, s, tab, start, nent);
}

int combine_blocks(const Geom& g) {
  return (g.nx / g.sx) * (g.ny / g.sy) * cb_bands(g);
}

void launch_combine(int mode, const CombineCall& a, hipStream_t s) {
  const dim3 grid(combine_blocks(a.g));
  if (mode == 0)
    hipLaunchKernelGGL(k_combine<0>, grid, dim3(CB_NT), 0, s, a);
  else if (mode == 1)
    hipLaunchKernelGGL(k_combine<1>, grid, dim3(CB_NT), 0, s, a);
  else
    hipLaunchKernelGGL(k_combine<2>, grid, dim3(CB_NT), 0, s, a);
}

void launch_combine_cg_batch(const CombineCall* tab, const int* start, int nent,
                             int total, hipStream_t s) {
  hipLaunchKernelGGL(k_combine_cg_batch, dim3(total), dim3(CB_NT), 0, s, tab, start, nent);
}

void launch_export_basis(const Geom& g, const CoarseNode* cn,
                         const int* col_node, int ncols, const uint8_t* mask,
                         const double* psi, double* out, double invH,
                         hipStream_t s) {
  if (ncols <= 0) return;
  const long long nn = (long long)g.nnx * g.nny;
  hipLaunchKernelGGL(k_export_basis,
                     dim3((unsigned)((nn + CK_NT - 1) / CK_NT), ncols),
                     dim3(CK_NT), 0, s, g, cn, col_node, mask, psi, out, invH);
}

}  // namespace msp
