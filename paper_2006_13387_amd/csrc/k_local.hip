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
// The elasticity systems use the twisted form of the same elimination: rows
// 0..m-1 are eliminated top-down and rows nyb-1..m+1 bottom-up, both into
// the middle row m = (nyb-1)/2, so that each solve is two independent
// chains of half the length that meet at the middle row.
// Only the blocks S_k^{-1} and compressed couplings are stored, one record
// per row and chain, so one solve reads about 2 * nyb * bs^2 stored values.
// Clamped (Dirichlet) DOFs become identity rows with zero couplings, which
// keeps the principal submatrix of the free DOFs exact.
#include <algorithm>
#include <vector>
#include "common.h"
#include "dev.h"
#include "small_dense.h"

namespace msp {

constexpr int FT_NT = 256;    // factorisation workgroup
constexpr int AP_NT = 512;    // first-level apply workgroup
constexpr int EG_NT = 512;    // eigen workgroup
typedef double eg_d4 __attribute__((ext_vector_type(4)));   // FP64 MFMA accumulator
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

// In-place Gauss-Jordan inversion of an SPD block (no pivoting is needed
// for SPD matrices).  The block sits in LDS (row stride LDSTR) before and
// after; during the inversion each of the 16 x 16 threads holds a 5 x 5
// tile in registers (rows ti + 16u, columns tj + 16w), and only the pivot
// row and column go through LDS, double-buffered by pivot parity so that
// one barrier per pivot suffices.  The pivot vectors span the whole tile
// range (GJ_N entries, those at and beyond bs are zero), so that every
// access to them is unconditional.  The owner of the next pivot forms its
// reciprocal during the current update, off the barrier-to-barrier path.
// pv: LDS scratch of GJ_PV doubles.
constexpr int GJ_T = 5;                      // tile edge: 16 * 5 >= MAXBS
constexpr int GJ_N = 16 * GJ_T;              // padded pivot vector length
constexpr int GJ_PV = 4 * GJ_N + 2;          // two row/column pairs, two reciprocals
static_assert(GJ_N >= MAXBS, "Gauss-Jordan tiles do not cover a block");
static_assert(GJ_T == 5, "gj_invert unrolls five tile rows of pivots");

// One Gauss-Jordan pivot p = 16 PU + pt.  PU is a compile-time constant,
// so the pivot's tile row and column are static register indices and only
// the entries of that tile row / column need a select.  On entry nv / inv
// hold (on the pivot's owner, ti = tj = pt) the pivot and its reciprocal;
// on exit the same for pivot p + 1.  A pivot that is not positive and
// finite sets bad on its owner and is replaced by 1.
template <int PU>
__device__ __forceinline__ void gj_pivot_step(double (&a)[GJ_T][GJ_T], int p,
                                              int pt, int ti, int tj,
                                              double* pv, double& nv,
                                              double& inv, bool& bad) {
  double* rowv = pv + (p & 1) * 2 * GJ_N;
  double* colv = rowv + GJ_N;
  double* ipv = pv + 4 * GJ_N + (p & 1);
  const bool prow = ti == pt, pcol = tj == pt;
  // the owners publish the current pivot row and column, and its reciprocal
  if (prow) {
#pragma unroll
    for (int w = 0; w < GJ_T; ++w) rowv[tj + 16 * w] = a[PU][w];
    if (pcol) {
      const bool ok = nv > 0.0 && finite(nv);
      bad |= !ok;
      *ipv = ok ? inv : 1.0;
    }
  }
  if (pcol) {
#pragma unroll
    for (int u = 0; u < GJ_T; ++u) colv[ti + 16 * u] = a[u][PU];
  }
  __syncthreads();
  const double ip = *ipv;
  double cv[GJ_T], rv[GJ_T];
#pragma unroll
  for (int u = 0; u < GJ_T; ++u) cv[u] = colv[ti + 16 * u];
#pragma unroll
  for (int w = 0; w < GJ_T; ++w) rv[w] = rowv[tj + 16 * w] * ip;
  // the entry of pivot p + 1 first: (PU, PU), or (PU + 1, PU + 1) after the
  // last pivot of this tile row
  constexpr int PN = PU + 1 < GJ_T ? PU + 1 : PU;
  const bool wrap = pt == 15;
  const double e_pp = a[PU][PU] - cv[PU] * rv[PU];
  const double e_nn = a[PN][PN] - cv[PN] * rv[PN];
  nv = wrap ? e_nn : e_pp;
  inv = 1.0 / nv;
#pragma unroll
  for (int u = 0; u < GJ_T; ++u)
#pragma unroll
    for (int w = 0; w < GJ_T; ++w) {
      const double upd = a[u][w] - cv[u] * rv[w];
      if (u == PU && w == PU)
        a[u][w] = prow ? (pcol ? ip : rv[w]) : (pcol ? -cv[u] * ip : upd);
      else if (u == PU)
        a[u][w] = prow ? rv[w] : upd;
      else if (w == PU)
        a[u][w] = pcol ? -cv[u] * ip : upd;
      else
        a[u][w] = upd;
    }
}

template <int PU>
__device__ __forceinline__ void gj_pivot_tile(double (&a)[GJ_T][GJ_T], int ti,
                                              int tj, int bs, double* pv,
                                              double& nv, double& inv,
                                              bool& bad) {
  for (int pt = 0; pt < 16; ++pt) {
    const int p = 16 * PU + pt;
    if (p >= bs) break;                       // uniform: bs is per system
    gj_pivot_step<PU>(a, p, pt, ti, tj, pv, nv, inv, bad);
  }
}

__device__ __forceinline__ void gj_invert(double* S, int bs, double* pv,
                                          int* __restrict__ err) {
  static_assert(FT_NT == 256, "the Gauss-Jordan tiling assumes 256 threads");
  const int tid = threadIdx.x;
  const int ti = tid & 15, tj = tid >> 4;
  double a[GJ_T][GJ_T];
#pragma unroll
  for (int u = 0; u < GJ_T; ++u)
#pragma unroll
    for (int w = 0; w < GJ_T; ++w) {
      const int i = ti + 16 * u, j = tj + 16 * w;
      a[u][w] = (i < bs && j < bs) ? S[i * LDSTR + j] : 0.0;
    }
  bool bad = false;
  double nv = a[0][0], inv = 1.0 / nv;
  gj_pivot_tile<0>(a, ti, tj, bs, pv, nv, inv, bad);
  gj_pivot_tile<1>(a, ti, tj, bs, pv, nv, inv, bad);
  gj_pivot_tile<2>(a, ti, tj, bs, pv, nv, inv, bad);
  gj_pivot_tile<3>(a, ti, tj, bs, pv, nv, inv, bad);
  gj_pivot_tile<4>(a, ti, tj, bs, pv, nv, inv, bad);
  if (bad) atomicOr(err, ERR_NOT_SPD);
#pragma unroll
  for (int u = 0; u < GJ_T; ++u)
#pragma unroll
    for (int w = 0; w < GJ_T; ++w) {
      const int i = ti + 16 * u, j = tj + 16 * w;
      if (i < bs && j < bs) S[i * LDSTR + j] = a[u][w];
    }
  __syncthreads();
}

// K entry between DOF (ia, ca) of node row ra and DOF (ib, cb) of node row
// rb of the rows staged in LDS (r = 0, 1, 2: node rows y-1, y, y+1), from
// the staged element moduli er[e][t] of element row y-1+e, element column
// x0 - 1 + t (zero outside the system's element box), and the element
// matrix Kl.
template <int NDOF>
__device__ __forceinline__ double coupling_l(const double (*er)[MAXBS + 2],
                                             const double* Kl, int ia, int ra,
                                             int ca, int ib, int rb, int cb) {
  double v = 0.0;
  const int tlo = max(ia, ib), thi = min(ia, ib) + 1;   // element columns t
  const int elo = max(ra, rb) - 1, ehi = min(ra, rb);   // element rows e
  for (int e = max(elo, 0); e <= ehi; ++e)
    for (int t = tlo; t <= thi; ++t) {
      const int va = (ia + 1 - t) + 2 * (ra - e);
      const int vb = (ib + 1 - t) + 2 * (rb - e);
      v += er[e][t] * Kl[(NDOF * va + ca) * (4 * NDOF) + NDOF * vb + cb];
    }
  return v;
}

// LDS of the factorisation: three dense blocks (the current row's S, the
// previous inverse P and W = P B^T), the banded coupling B of the row with
// the previous row of the chain, and the staged element moduli of element
// rows y-1, y, y+1 and clamp flags of node rows y-1, y, y+1.
struct FactorLds {
  double buf[3][MAXBS * LDSTR];
  double Bv[MAXBS * 6];
  double pv[GJ_PV];
  double ddiag[MAXBS];
  double er[3][MAXBS + 2];
  uint8_t fr[3][MAXBS];
  double Kl[64];
  double red[FT_NT / 64 + 1];
};

// Stage element rows y-1, y, y+1 (element columns x0-1 .. x0+nxb-1, zero
// outside the element box) and node rows y-1, y, y+1 (rows outside the mesh
// are flagged).
template <int NDOF>
__device__ __forceinline__ void fac_stage(const Geom& g, const SysDesc& s, int y,
                                          const double* __restrict__ E,
                                          const uint8_t* __restrict__ flag,
                                          FactorLds& L) {
  const int tid = threadIdx.x;
  const int bs = NDOF * s.nxb;
  for (int idx = tid; idx < 3 * (s.nxb + 1); idx += FT_NT) {
    const int e = idx / (s.nxb + 1), t = idx - e * (s.nxb + 1);
    const int ex = s.x0 - 1 + t, ey = y - 1 + e;
    const bool in = ex >= s.ex0 && ex < s.ex1 && ey >= s.ey0 && ey < s.ey1;
    L.er[e][t] = in ? E[(long long)ey * g.nx + ex] : 0.0;
  }
  for (int idx = tid; idx < 3 * bs; idx += FT_NT) {
    const int r = idx / bs, a = idx - r * bs;
    const int yy = y - 1 + r;
    L.fr[r][a] = (yy >= 0 && yy < g.nny) ? flag[NDOF * ((long long)yy * g.nnx + s.x0) + a] : 1;
  }
}

// D of the staged node row into S (row stride LDSTR), its diagonal into
// ddiag; clamped DOFs become identity rows and columns.
template <int NDOF>
__device__ __forceinline__ void fac_diag(int bs, double* S, FactorLds& L) {
  for (int idx = threadIdx.x; idx < bs * bs; idx += FT_NT) {
    const int a = idx / bs, b = idx - (idx / bs) * bs;
    const int ia = a / NDOF, ca = a - ia * NDOF;
    const int ib = b / NDOF, cb = b - ib * NDOF;
    double v = 0.0;
    if (L.fr[1][a] || L.fr[1][b]) {
      v = (a == b) ? 1.0 : 0.0;
    } else if (abs(ia - ib) <= 1) {
      v = coupling_l<NDOF>(L.er, L.Kl, ia, 1, ca, ib, 1, cb);
    }
    S[a * LDSTR + b] = v;
    if (a == b) L.ddiag[a] = v;
  }
}

// Banded couplings of the staged node row with node row rb (0: the row
// above, 2: the row below): Bv[a][t] couples DOF a with DOF
// NDOF (ia + t / NDOF - 1) + t % NDOF of that row (zero outside the row and
// at clamped DOFs).
template <int NDOF>
__device__ __forceinline__ void fac_coupling(int nxb, int rb, FactorLds& L) {
  const int bs = NDOF * nxb;
  for (int idx = threadIdx.x; idx < bs * 3 * NDOF; idx += FT_NT) {
    const int a = idx / (3 * NDOF), t = idx - a * (3 * NDOF);
    const int ia = a / NDOF, ca = a - ia * NDOF;
    const int di = t / NDOF - 1, cb = t - (t / NDOF) * NDOF;
    const int ib = ia + di;
    double v = 0.0;
    if (ib >= 0 && ib < nxb && !L.fr[1][a] && !L.fr[rb][NDOF * ib + cb])
      v = coupling_l<NDOF>(L.er, L.Kl, ia, 1, ca, ib, rb, cb);
    L.Bv[idx] = v;
  }
}

// S -= B P B^T for the coupling in Bv and the inverse P of the eliminated
// row (both in LDS); W = P B^T is scratch.
template <int NDOF>
__device__ __forceinline__ void fac_schur(int bs, const double* P, double* W,
                                          double* S, const FactorLds& L) {
  const int tid = threadIdx.x;
  for (int idx = tid; idx < bs * bs; idx += FT_NT) {
    const int b = idx / bs, a = idx - (idx / bs) * bs;
    const int ia = a / NDOF;
    double v = 0.0;
#pragma unroll
    for (int t = 0; t < 3 * NDOF; ++t) {
      const int col = NDOF * (ia + t / NDOF - 1) + (t % NDOF);
      if (col >= 0 && col < bs) v += P[b * LDSTR + col] * L.Bv[a * 3 * NDOF + t];
    }
    W[b * LDSTR + a] = v;
  }
  __syncthreads();
  for (int idx = tid; idx < bs * bs; idx += FT_NT) {
    const int a = idx / bs, a2 = idx - (idx / bs) * bs;
    const int ia = a / NDOF;
    double v = 0.0;
#pragma unroll
    for (int t = 0; t < 3 * NDOF; ++t) {
      const int row = NDOF * (ia + t / NDOF - 1) + (t % NDOF);
      if (row >= 0 && row < bs) v += L.Bv[a * 3 * NDOF + t] * W[row * LDSTR + a2];
    }
    S[a * LDSTR + a2] -= v;
  }
}

// Records of one node row.  Heat pencils (NDOF = 1): heat_rec (S^{-1}
// column-major, F (bs x 3), G (bs x 3)).  Elasticity (NDOF = 2): the
// first-level layout of l1_rec (16-byte column groups, then F (bs x 6)).
__host__ __device__ inline long long fac_rec(int ndof, int nxb) {
  const int bs = ndof * nxb;
  return ndof == 2 ? l1_rec(bs) : (long long)heat_rec(bs);
}
__host__ __device__ inline long long fac_fpart(int ndof, int bs) {
  return ndof == 2 ? (long long)l1_cols(bs) * bs : (long long)bs * bs;
}
// the same for FP64 elasticity records (packed lower column pairs)
__host__ __device__ inline long long fac_fpart64(int ndof, int bs) {
  return ndof == 2 ? (long long)l1_s64(bs) : (long long)bs * bs;
}

// Inverse block of a record (layout as in fac_rec; padding columns zero).
template <int NDOF>
__device__ __forceinline__ void fac_write_inverse(int bs, const double* S,
                                                  double* o64, float* o32) {
  if (NDOF == 1) {
    for (int idx = threadIdx.x; idx < bs * bs; idx += FT_NT) {
      const int j = idx / bs, i = idx - (idx / bs) * bs;
      o64[idx] = S[i * LDSTR + j];
    }
    return;
  }
  const int nc = l1_cols(bs);
  // FP64: the symmetric part (X + X^T) / 2 of the computed inverse X (the
  // exact inverse of a slightly perturbed block, so it stays positive
  // definite where the raw lower triangle of an ill-conditioned X need not)
  for (int p = 0; 2 * p < bs; ++p) {
    const int off = l1_pair_off(bs, p);
    for (int e = threadIdx.x; e < 2 * (bs - 2 * p); e += FT_NT) {
      const int i = 2 * p + (e >> 1), j = 2 * p + (e & 1);
      o64[off + e] = 0.5 * (S[i * LDSTR + j] + S[j * LDSTR + i]);
    }
  }
  if (o32 != nullptr) {
    for (int idx = threadIdx.x; idx < nc * bs; idx += FT_NT) {
      const int jq = idx / (4 * bs), rem = idx - jq * (4 * bs);
      const int i = rem >> 2, j = 4 * jq + (rem & 3);
      o32[idx] = j < bs ? (float)S[i * LDSTR + j] : 0.0f;
    }
  }
}

// Coupling part F of a record (Bv, or zero for the first row of a chain).
template <int NDOF>
__device__ __forceinline__ void fac_write_coupling(int bs, bool coupled,
                                                   const FactorLds& L,
                                                   double* o64, float* o32) {
  const long long fo = fac_fpart(NDOF, bs), fo64 = fac_fpart64(NDOF, bs);
  for (int idx = threadIdx.x; idx < bs * 3 * NDOF; idx += FT_NT) {
    const double v = coupled ? L.Bv[idx] : 0.0;
    o64[fo64 + idx] = v;
    if (o32 != nullptr) o32[fo + idx] = (float)v;
  }
}

// max over the workgroup of v (fixed order); thread 0 holds the result
__device__ __forceinline__ double fac_wg_max(double v, FactorLds& L) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) L.red[threadIdx.x >> 6] = v;
  __syncthreads();
  double mm = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < FT_NT / 64; ++i) mm = fmax(mm, L.red[i]);
  return mm;
}

// Factorise one chain of node rows of system s: count rows starting at
// node row row0 (relative to the box) in direction dir (+1 downwards in row
// index, -1 upwards), each eliminating the previous row of the chain, with
// chain position j's record at record index rec0 + j.  Heat records also
// hold G, the coupling with the next row of the chain; for the chain's last
// row that is the row after it (the middle row of a twisted factorisation)
// when tail is set, else zero.  Returns this thread's share of
// max_i (S^-1)_ii (D)_ii.
template <int NDOF>
__device__ double factor_chain(const Geom& g, const SysDesc& s, int row0,
                               int dir, int count, int rec0, bool tail,
                               const double* __restrict__ E,
                               const uint8_t* __restrict__ flag,
                               double* __restrict__ out64,
                               float* __restrict__ out32, int* err,
                               FactorLds& L) {
  const int tid = threadIdx.x;
  const int bs = NDOF * s.nxb;
  const int rb = 1 - dir;              // staged node row of the previous row
  const long long rec = fac_rec(NDOF, s.nxb);
  double mloc = 0.0;
  int cur = 0, prev = 1, wb = 2;
  for (int j = 0; j < count; ++j) {
    const int y = s.y0 + row0 + dir * j;
    double* S = L.buf[cur];
    fac_stage<NDOF>(g, s, y, E, flag, L);
    __syncthreads();
    fac_diag<NDOF>(bs, S, L);
    if (j > 0) {
      fac_coupling<NDOF>(s.nxb, rb, L);
      __syncthreads();
      fac_schur<NDOF>(bs, L.buf[prev], L.buf[wb], S, L);
    }
    __syncthreads();
    gj_invert(S, bs, L.pv, err);
    const long long off = s.foff + (long long)(rec0 + j) * rec;
    fac_write_inverse<NDOF>(bs, S, out64 + off, out32 ? out32 + off : nullptr);
    fac_write_coupling<NDOF>(bs, j > 0, L, out64 + off, out32 ? out32 + off : nullptr);
    if (NDOF == 1) {
      // G: couplings with the next row of the chain
      __syncthreads();
      const bool nxt = j + 1 < count || tail;
      if (nxt) fac_coupling<NDOF>(s.nxb, 1 + dir, L);
      __syncthreads();
      for (int idx = tid; idx < 3 * bs; idx += FT_NT)
        out64[off + (long long)bs * bs + 3 * bs + idx] = nxt ? L.Bv[idx] : 0.0;
    }
    for (int a = tid; a < bs; a += FT_NT) mloc = fmax(mloc, S[a * LDSTR + a] * L.ddiag[a]);
    __syncthreads();
    const int t = prev;
    prev = cur;
    cur = t;
  }
  return mloc;
}

// Twisted factorisation, both outer parts: workgroup 2 i + h factorises
// system i's chain h: h = 0 eliminates rows 0..m-1 top-down (records
// 0..m-1), h = 1 rows nyb-1..m+1 bottom-up (records m+1..nyb-1), with
// m = (nyb - 1) / 2 the middle row.
//
// out64 receives the FP64 records; out32 (may be null) a rounded FP32
// copy.  metric (may be null) receives per system max_i (S_k^-1)_ii (D_k)_ii
// over all blocks: about 1 for DOFs held by stiff material and up to the
// contrast E0/Emin for DOFs of stiff islands that float in soft material,
// whose rigid motions then have amplitudes ~E0/Emin.  FP32 rounding of such
// values leaves spurious strains in the stiff phase, so the runtime keeps
// FP64 blocks for systems whose metric exceeds a bound.  Part metrics go to
// metric[nsys + 2 i + h], the system's to metric[i] (k_factor_middle).
//
// Workgroups take their chains from pack (see chain_items).
template <int NDOF>
__global__ void __launch_bounds__(FT_NT)
k_factor_twisted(Geom g, const SysDesc* __restrict__ systems, int nsys,
                 const double* __restrict__ E, const uint8_t* __restrict__ flag,
                 const double* __restrict__ Kel, double* __restrict__ out64,
                 float* __restrict__ out32, double* __restrict__ metric,
                 int* __restrict__ err, const int* __restrict__ pack) {
  __shared__ FactorLds L;
  for (int i = threadIdx.x; i < 16 * NDOF * NDOF; i += FT_NT) L.Kl[i] = Kel[i];
  const int q0 = pack[blockIdx.x], q1 = pack[blockIdx.x + 1];
  for (int q = q0; q < q1; ++q) {
    const int item = pack[gridDim.x + 1 + q];
    const int sys = item >> 1, half = item & 1;
    const SysDesc s = systems[sys];
    const int m = (s.nyb - 1) >> 1;
    __syncthreads();                          // (the previous chain's LDS)
    const double mloc =
        half == 0 ? factor_chain<NDOF>(g, s, 0, 1, m, 0, true, E, flag, out64, out32, err, L)
                  : factor_chain<NDOF>(g, s, s.nyb - 1, -1, s.nyb - 1 - m, m + 1, true,
                                       E, flag, out64, out32, err, L);
    const double mm = fac_wg_max(mloc, L);
    if (metric != nullptr && threadIdx.x == 0) metric[nsys + item] = mm;
  }
}

// Load the inverse block of a record (layout as in fac_rec) into LDS (row
// stride LDSTR).
template <int NDOF>
__device__ __forceinline__ void fac_load_inverse(int bs, const double* __restrict__ o,
                                                 double* P) {
  if (NDOF == 1) {
    for (int idx = threadIdx.x; idx < bs * bs; idx += FT_NT) {
      const int j = idx / bs, i = idx - (idx / bs) * bs;
      P[i * LDSTR + j] = o[idx];
    }
    return;
  }
  // packed lower column pairs; the mirror entries written alike (the
  // 2 x 2 diagonal blocks twice, with equal values)
  for (int p = 0; 2 * p < bs; ++p) {
    const int off = l1_pair_off(bs, p);
    for (int e = threadIdx.x; e < 2 * (bs - 2 * p); e += FT_NT) {
      const int i = 2 * p + (e >> 1), j = 2 * p + (e & 1);
      const double v = o[off + e];
      P[i * LDSTR + j] = v;
      P[j * LDSTR + i] = v;
    }
  }
}

// Twisted factorisation, the middle row m of system i (one workgroup each):
// S_m = D_m - B S_{m-1}^{-1} B^T - C S'_{m+1}^{-1} C^T with B, C the
// couplings of row m with rows m-1 and m+1, inverted.  Its inverse ends
// both chains: record m (top chain, with F = B) and record nyb (bottom
// chain, with F = C).  metric[i] = max over the system (metric may be
// null).  Heat records of the middle row get G = 0 (no row follows it).
template <int NDOF>
__global__ void __launch_bounds__(FT_NT)
k_factor_middle(Geom g, const SysDesc* __restrict__ systems, int nsys,
                const double* __restrict__ E, const uint8_t* __restrict__ flag,
                const double* __restrict__ Kel, double* __restrict__ out64,
                float* __restrict__ out32, double* __restrict__ metric,
                int* __restrict__ err) {
  __shared__ FactorLds L;
  const SysDesc s = systems[blockIdx.x];
  const int tid = threadIdx.x;
  const int bs = NDOF * s.nxb;
  const int m = (s.nyb - 1) >> 1;
  const long long rec = fac_rec(NDOF, s.nxb);
  for (int i = tid; i < 16 * NDOF * NDOF; i += FT_NT) L.Kl[i] = Kel[i];
  double* S = L.buf[0];
  fac_stage<NDOF>(g, s, s.y0 + m, E, flag, L);
  __syncthreads();
  fac_diag<NDOF>(bs, S, L);
  const long long otop = s.foff + (long long)m * rec;
  const long long obot = s.foff + (long long)s.nyb * rec;
  // top part: row m-1 eliminated
  if (m > 0) {
    fac_coupling<NDOF>(s.nxb, 0, L);
    fac_load_inverse<NDOF>(bs, out64 + s.foff + (long long)(m - 1) * rec, L.buf[1]);
    __syncthreads();
    fac_schur<NDOF>(bs, L.buf[1], L.buf[2], S, L);
    __syncthreads();
  }
  fac_write_coupling<NDOF>(bs, m > 0, L, out64 + otop, out32 ? out32 + otop : nullptr);
  __syncthreads();
  // bottom part: row m+1 eliminated (its record is the bottom chain's
  // record nyb-1)
  if (m + 1 < s.nyb) {
    fac_coupling<NDOF>(s.nxb, 2, L);
    fac_load_inverse<NDOF>(bs, out64 + s.foff + (long long)(s.nyb - 1) * rec, L.buf[1]);
    __syncthreads();
    fac_schur<NDOF>(bs, L.buf[1], L.buf[2], S, L);
    __syncthreads();
  }
  fac_write_coupling<NDOF>(bs, m + 1 < s.nyb, L, out64 + obot, out32 ? out32 + obot : nullptr);
  __syncthreads();
  gj_invert(S, bs, L.pv, err);
  fac_write_inverse<NDOF>(bs, S, out64 + otop, out32 ? out32 + otop : nullptr);
  fac_write_inverse<NDOF>(bs, S, out64 + obot, out32 ? out32 + obot : nullptr);
  if (NDOF == 1) {
    for (int idx = tid; idx < 3 * bs; idx += FT_NT) {
      out64[otop + (long long)bs * bs + 3 * bs + idx] = 0.0;
      out64[obot + (long long)bs * bs + 3 * bs + idx] = 0.0;
    }
  }
  double mloc = 0.0;
  for (int a = tid; a < bs; a += FT_NT) mloc = fmax(mloc, S[a * LDSTR + a] * L.ddiag[a]);
  const double mm = fac_wg_max(mloc, L);
  if (metric != nullptr && tid == 0)
    metric[blockIdx.x] = fmax(mm, fmax(metric[nsys + 2 * blockIdx.x],
                                       metric[nsys + 2 * blockIdx.x + 1]));
}

// ---------------------------------------------------------------------
// First level: z_i = K_i^{-1} R_i r for every subdomain (2D elasticity).
//
// Two passes (forward, backward) of two workgroups of 8 waves per
// subdomain, one per chain of the twisted factorisation; the chain's part
// of the local vector stays in LDS within a pass and goes through lsol
// between the passes.  Each chain position has a record in HBM: its inverse
// Schur block (column-major) followed by the couplings F of its row with
// the previous row of the chain, written by the factorisation.  Step c of a
// pass uses the record of one chain position:
//  * waves 4-7 ("loaders") copy records straight from HBM into a ring of R
//    LDS slots with direct-to-LDS loads (global_load_lds, 16 bytes a lane),
//    R-1 steps ahead, and wait with an explicit vmcnt for the record of the
//    next step only: the HBM latency of a record overlaps R-1 steps;
//  * waves 0-3 ("compute") only read and write LDS, so they never wait on
//    memory.  Phase 1 forms the block right-hand side w from the
//    neighbouring position (forward: F of this record; backward: F of the
//    previous step's record, read transposed); phase 2 multiplies w by the
//    inverse block, split over L1_NS column groups (thread (q, i) sums
//    row i over group q).  The group partial sums are added up where they
//    are next used, in the following step's phase 1, which also retires
//    the finished position into v.
// Two barriers per step.
constexpr int L1_NS = 3;                   // column groups of the block GEMV
constexpr int L1_GMAX = 4 * ((MAXBS / 4 + L1_NS - 1) / L1_NS);   // columns per group
constexpr int L1_COMPUTE = 256;            // threads of the compute waves
constexpr int L1_NLW = (AP_NT - L1_COMPUTE) / 64;   // loader waves
constexpr int L1_CHUNK = 1024;             // bytes of one wave's DMA load
constexpr int L1_VPT = 5;                  // local-vector entries a compute thread reads ahead
constexpr int L1_LDS = 160 * 1024 - 256;   // LDS of the apply kernel
static_assert(L1_NS * MAXBS <= L1_COMPUTE, "GEMV threads exceed the compute waves");

// ring geometry of one subdomain: R slots of nch 1 KiB chunks; chunk q is
// copied by loader wave q % L1_NLW
struct L1Ring {
  int rec;       // record elements (l1_rec)
  int nch;       // chunks per record
  int slot;      // slot bytes
  int R;         // ring depth, 2..8
};

// LDS elements beside the ring: v (nb*bs, rounded up to 4), w (l1_cols,
// padding zero), partial sums P[parity][row][group] (2 x MAXBS x 4)
__host__ __device__ inline int l1_vec_elems(int bs, int nb) {
  return ((nb * bs + 3) & ~3) + l1_cols(bs) + 2 * 4 * MAXBS;
}

// elements of a record a pass reads (FP64: the packed block and F)
template <typename T>
__host__ __device__ inline int l1_used(int bs) {
  return sizeof(T) == 8 ? l1_s64(bs) + 6 * bs : (int)l1_rec(bs);
}

template <typename T>
__host__ __device__ inline L1Ring l1_ring(int bs, int nb) {
  L1Ring g;
  g.rec = (int)l1_rec(bs);
  g.nch = (l1_used<T>(bs) * (int)sizeof(T) + L1_CHUNK - 1) / L1_CHUNK;
  g.slot = g.nch * L1_CHUNK;
  const int vbytes = l1_vec_elems(bs, nb) * (int)sizeof(T);
  const int per_wave = (g.nch + L1_NLW - 1) / L1_NLW;
  g.R = 2;
  // deeper rings while they fit and the vmcnt wait stays within 63
  while (g.R < 8 && (g.R + 1) * g.slot + vbytes <= L1_LDS &&
         (g.R - 1) * per_wave <= 63)
    ++g.R;
  return g;
}

template <typename T>
__host__ __device__ inline bool l1_fits(int bs, int nb) {
  const L1Ring g = l1_ring<T>(bs, nb);
  return g.R * g.slot + l1_vec_elems(bs, nb) * (int)sizeof(T) <= L1_LDS;
}

// s_waitcnt vmcnt(n) for a wave-uniform n in 0..63 (larger n waits for 63)
__device__ __forceinline__ void wait_vmcnt(int n) {
  switch (n) {
    case 0: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
    case 1: asm volatile("s_waitcnt vmcnt(1)" ::: "memory"); break;
    case 2: asm volatile("s_waitcnt vmcnt(2)" ::: "memory"); break;
    case 3: asm volatile("s_waitcnt vmcnt(3)" ::: "memory"); break;
    case 4: asm volatile("s_waitcnt vmcnt(4)" ::: "memory"); break;
    case 5: asm volatile("s_waitcnt vmcnt(5)" ::: "memory"); break;
    case 6: asm volatile("s_waitcnt vmcnt(6)" ::: "memory"); break;
    case 7: asm volatile("s_waitcnt vmcnt(7)" ::: "memory"); break;
    case 8: asm volatile("s_waitcnt vmcnt(8)" ::: "memory"); break;
    case 9: asm volatile("s_waitcnt vmcnt(9)" ::: "memory"); break;
    case 10: asm volatile("s_waitcnt vmcnt(10)" ::: "memory"); break;
    case 11: asm volatile("s_waitcnt vmcnt(11)" ::: "memory"); break;
    case 12: asm volatile("s_waitcnt vmcnt(12)" ::: "memory"); break;
    case 13: asm volatile("s_waitcnt vmcnt(13)" ::: "memory"); break;
    case 14: asm volatile("s_waitcnt vmcnt(14)" ::: "memory"); break;
    case 15: asm volatile("s_waitcnt vmcnt(15)" ::: "memory"); break;
    case 16: asm volatile("s_waitcnt vmcnt(16)" ::: "memory"); break;
    case 17: asm volatile("s_waitcnt vmcnt(17)" ::: "memory"); break;
    case 18: asm volatile("s_waitcnt vmcnt(18)" ::: "memory"); break;
    case 19: asm volatile("s_waitcnt vmcnt(19)" ::: "memory"); break;
    case 20: asm volatile("s_waitcnt vmcnt(20)" ::: "memory"); break;
    case 21: asm volatile("s_waitcnt vmcnt(21)" ::: "memory"); break;
    case 22: asm volatile("s_waitcnt vmcnt(22)" ::: "memory"); break;
    case 23: asm volatile("s_waitcnt vmcnt(23)" ::: "memory"); break;
    case 24: asm volatile("s_waitcnt vmcnt(24)" ::: "memory"); break;
    case 25: asm volatile("s_waitcnt vmcnt(25)" ::: "memory"); break;
    case 26: asm volatile("s_waitcnt vmcnt(26)" ::: "memory"); break;
    case 27: asm volatile("s_waitcnt vmcnt(27)" ::: "memory"); break;
    case 28: asm volatile("s_waitcnt vmcnt(28)" ::: "memory"); break;
    case 29: asm volatile("s_waitcnt vmcnt(29)" ::: "memory"); break;
    case 30: asm volatile("s_waitcnt vmcnt(30)" ::: "memory"); break;
    case 31: asm volatile("s_waitcnt vmcnt(31)" ::: "memory"); break;
    case 32: asm volatile("s_waitcnt vmcnt(32)" ::: "memory"); break;
    case 33: asm volatile("s_waitcnt vmcnt(33)" ::: "memory"); break;
    case 34: asm volatile("s_waitcnt vmcnt(34)" ::: "memory"); break;
    case 35: asm volatile("s_waitcnt vmcnt(35)" ::: "memory"); break;
    case 36: asm volatile("s_waitcnt vmcnt(36)" ::: "memory"); break;
    case 37: asm volatile("s_waitcnt vmcnt(37)" ::: "memory"); break;
    case 38: asm volatile("s_waitcnt vmcnt(38)" ::: "memory"); break;
    case 39: asm volatile("s_waitcnt vmcnt(39)" ::: "memory"); break;
    case 40: asm volatile("s_waitcnt vmcnt(40)" ::: "memory"); break;
    case 41: asm volatile("s_waitcnt vmcnt(41)" ::: "memory"); break;
    case 42: asm volatile("s_waitcnt vmcnt(42)" ::: "memory"); break;
    case 43: asm volatile("s_waitcnt vmcnt(43)" ::: "memory"); break;
    case 44: asm volatile("s_waitcnt vmcnt(44)" ::: "memory"); break;
    case 45: asm volatile("s_waitcnt vmcnt(45)" ::: "memory"); break;
    case 46: asm volatile("s_waitcnt vmcnt(46)" ::: "memory"); break;
    case 47: asm volatile("s_waitcnt vmcnt(47)" ::: "memory"); break;
    case 48: asm volatile("s_waitcnt vmcnt(48)" ::: "memory"); break;
    case 49: asm volatile("s_waitcnt vmcnt(49)" ::: "memory"); break;
    case 50: asm volatile("s_waitcnt vmcnt(50)" ::: "memory"); break;
    case 51: asm volatile("s_waitcnt vmcnt(51)" ::: "memory"); break;
    case 52: asm volatile("s_waitcnt vmcnt(52)" ::: "memory"); break;
    case 53: asm volatile("s_waitcnt vmcnt(53)" ::: "memory"); break;
    case 54: asm volatile("s_waitcnt vmcnt(54)" ::: "memory"); break;
    case 55: asm volatile("s_waitcnt vmcnt(55)" ::: "memory"); break;
    case 56: asm volatile("s_waitcnt vmcnt(56)" ::: "memory"); break;
    case 57: asm volatile("s_waitcnt vmcnt(57)" ::: "memory"); break;
    case 58: asm volatile("s_waitcnt vmcnt(58)" ::: "memory"); break;
    case 59: asm volatile("s_waitcnt vmcnt(59)" ::: "memory"); break;
    case 60: asm volatile("s_waitcnt vmcnt(60)" ::: "memory"); break;
    case 61: asm volatile("s_waitcnt vmcnt(61)" ::: "memory"); break;
    case 62: asm volatile("s_waitcnt vmcnt(62)" ::: "memory"); break;
    default: asm volatile("s_waitcnt vmcnt(63)" ::: "memory"); break;
  }
}

// 16 bytes of T: four floats or two doubles
template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float4 type; static constexpr int n = 4; };
template <> struct Vec16<double> { typedef double2 type; static constexpr int n = 2; };

// GEMV of one column group of a record block in 16-byte column groups:
// sum over j < n of S(i, j) * w[j] (n <= NJ, a multiple of the group
// width), where S points at the group's first 16-byte column group and
// column group u of row i sits at S + u*G*bs + G*i (G = 16 / sizeof(T)).
// Fully unrolled, every LDS read issued before the first use; column
// groups at or past n read group 0 and weigh it by 0.  Four accumulators,
// column j into accumulator j % 4.
template <typename T, int NJ>
__device__ __forceinline__ T lds_gemv_group(const T* S, int bs, int i,
                                            const T* w, int n) {
  typedef typename Vec16<T>::type V;
  constexpr int G = Vec16<T>::n;
  constexpr int NU = NJ / G;
  static_assert(NJ % 4 == 0, "column groups hold whole quads");
  V s[NU], x[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int uc = u * G < n ? u : 0;
    s[u] = *reinterpret_cast<const V*>(S + uc * G * bs + G * i);
    x[u] = *reinterpret_cast<const V*>(w + uc * G);
  }
  T a[4] = {0, 0, 0, 0};
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const T m = u * G < n ? (T)1 : (T)0;
    if constexpr (G == 4) {
      a[0] += s[u].x * (m * x[u].x);
      a[1] += s[u].y * (m * x[u].y);
      a[2] += s[u].z * (m * x[u].z);
      a[3] += s[u].w * (m * x[u].w);
    } else {
      a[(2 * u) & 3] += s[u].x * (m * x[u].x);
      a[(2 * u + 1) & 3] += s[u].y * (m * x[u].y);
    }
  }
  return (a[0] + a[1]) + (a[2] + a[3]);
}

// The same over the FP64 packed layout (lower part of each column pair,
// rows 2p..bs-1): for pair p = j0/2 + u, row i reads S(i, 2p) and
// S(i, 2p+1) from row i of pair p when i >= 2p, else S(2p, i) and
// S(2p+1, i) (component i%2) from rows 2p, 2p+1 of pair i/2.  Every lane
// reads two doubles at addresses chosen by selects, so the two cases do not
// diverge.  Pairs past the block (2p >= bs) weigh 0.
template <int NJ>
__device__ __forceinline__ double lds_gemv_sym(const double* S, int bs, int i,
                                               const double* w, int j0, int n) {
  constexpr int NU = NJ / 2;
  static_assert(NJ % 4 == 0, "column groups hold whole quads");
  const int q = i >> 1, comp = i & 1, ph = bs / 2 - 1;
  const int uoff = l1_pair_off(bs, q) + comp;   // row 0 of pair i/2, component
  double s0[NU], s1[NU];
  double2 x[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int p = min(j0 / 2 + u, ph);
    const bool lower = i >= 2 * p;
    const int a0 = lower ? l1_pair_off(bs, p) + 2 * (i - 2 * p) : uoff + 2 * (2 * p - 2 * q);
    const int a1 = lower ? a0 + 1 : a0 + 2;
    s0[u] = S[a0];
    s1[u] = S[a1];
    x[u] = *reinterpret_cast<const double2*>(w + (2 * u < n ? j0 + 2 * u : 0));
  }
  double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const double m = (2 * u < n && j0 + 2 * u < bs) ? 1.0 : 0.0;
    a[(2 * u) & 3] += s0[u] * (m * x[u].x);
    a[(2 * u + 1) & 3] += s1[u] * (m * x[u].y);
  }
  return (a[0] + a[1]) + (a[2] + a[3]);
}

typedef __attribute__((address_space(3))) void lds_void;

// loader wave lw: DMA its chunks of the record of row k into the LDS slot
template <typename T>
__device__ __forceinline__ void l1_dma(const T* base, int rec, int k,
                                       unsigned char* slot, int nch,
                                       int lw, int lane) {
  const unsigned char* src =
      reinterpret_cast<const unsigned char*>(base + (long long)k * rec);
  for (int q = lw; q < nch; q += L1_NLW) {
    const int off = q * L1_CHUNK;
    __builtin_amdgcn_global_load_lds((const void*)(src + off + 16 * lane),
                                     (lds_void*)(slot + off), 16, 0, 0);
  }
}

// Workgroup barrier ordering LDS accesses only.  __syncthreads(), and any
// release fence that covers LDS, makes every wave wait for all of its
// loads in flight, the direct-to-LDS record loads included; the ring waits
// for those itself with an explicit vmcnt before it reaches the barrier.
// The asm's memory clobber keeps the compiler from moving memory accesses
// across it.
__device__ __forceinline__ void l1_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// First-level solve of one system by the twisted factorisation: chain h
// (0: node rows 0..m from the top, 1: node rows nyb-1..m from the bottom,
// m = (nyb - 1) / 2) has L positions, the last being the middle row; its
// position j is node row j (h = 0) or nyb-1-j (h = 1) with record rec0 + j.
//  * forward (BWD = false): t_j = S_j^{-1} (r_j - F_j t_{j-1}) for
//    j = 0..L-2 into lsol, then the middle row's coupling to this chain,
//    g_h = F_{L-1} t_{L-2}, into gm[h];
//  * backward (BWD = true): x_m = S_m^{-1} (r_m - g_0 - g_1), then
//    x_j = t_j - S_j^{-1} F_{j+1}^T x_{j+1} for j = L-2..0, into lsol
//    (the middle row by chain 0 only).
// Step c of the sweep uses the record of position j(c) (forward j = c,
// backward j = L-1-c).
// gate: the CG stop test of the workgroup (may be null), run once the
// first record copies are in flight so that the two latencies overlap;
// when it says the solve is over the workgroup drains its copies and leaves.
template <typename T, bool BWD, typename Gate>
__device__ void level1_half(const Geom& g, const SysDesc& s, int half,
                            const uint8_t* __restrict__ mask,
                            const T* __restrict__ Sinv,
                            const double* __restrict__ r,
                            double* __restrict__ lsol, double* __restrict__ gm,
                            unsigned char* lds, const Gate& gate) {
  const int tid = threadIdx.x;
  const int bs = 2 * s.nxb;
  const int nb = s.nyb;
  const int ncols = l1_cols(bs);
  const int fo = sizeof(T) == 8 ? l1_s64(bs) : ncols * bs;   // F part of a record
  const int mid = (nb - 1) >> 1;
  const int L = half ? nb - mid : mid + 1;
  const int rec0 = half ? mid + 1 : 0;
  const int nsteps = BWD ? L : L - 1;
  const L1Ring ring = l1_ring<T>(bs, L);
  const int R = ring.R;
  const T* base = Sinv + s.foff + (long long)rec0 * ring.rec;
  double* o = lsol + s.voff;
  auto row_of = [&](int j) { return half ? nb - 1 - j : j; };
  auto pos_of = [&](int c) { return BWD ? L - 1 - c : c; };
  if (!BWD && L == 1) {
    // no row before the middle on this side
    if (gate()) return;
    for (int a = tid; a < bs; a += AP_NT) gm[half * MAXBS + a] = 0.0;
    return;
  }
  T* v = reinterpret_cast<T*>(lds + R * ring.slot);
  T* w = v + ((L * bs + 3) & ~3);             // 16-byte aligned
  T* P = w + ncols;                           // P[parity][row][4]: group sums
  const bool loader = tid >= L1_COMPUTE;
  const int lw = __builtin_amdgcn_readfirstlane((tid - L1_COMPUTE) >> 6);
  const int lane = tid & 63;
  // loads this wave issues per record
  const int cw = lw < ring.nch ? (ring.nch - lw + L1_NLW - 1) / L1_NLW : 0;
  // GEMV role: column group q (cs columns, whole quads), row i
  const int cs = 4 * ((ncols / 4 + L1_NS - 1) / L1_NS);
  const int gq = tid / bs, gi = tid - (tid / bs) * bs;
  const int j0 = gq * cs;
  const int jn = max(0, min(ncols, j0 + cs) - j0);
  const bool gemv = tid < L1_NS * bs;
  // phase-1 role: row entry tid, its node and component
  const int ia = tid >> 1, ca = tid & 1;

  // Records are copied in step order, record n into slot n % R: the
  // prologue issues the first R - 1, step c the record of step c + R - 1
  // (none past the last step), so that after step c's issue the first
  // min(c + R, nsteps) records are in flight or landed.
  const int npro = min(R - 1, nsteps);
  if (loader)
    for (int n = 0; n < npro; ++n)
      l1_dma<T>(base, ring.rec, pos_of(n), lds + n * ring.slot, ring.nch, lw, lane);
  // local vector: forward, r at the chain's rows before the middle;
  // backward, the forward results t_j and the middle row's right-hand side.
  // The compute waves read the first L1_VPT entries each before the stop
  // test, so that the two latencies overlap; the loader waves read nothing
  // but records, so that their memory counters count only record copies.
  const int nv = (L - 1) * bs;
  auto v_load = [&](int idx) -> T {
    const int j = idx / bs, a = idx - (idx / bs) * bs;
    const int k = row_of(j);
    if (!BWD) {
      const long long d = 2 * ((long long)(s.y0 + k) * g.nnx + s.x0 + a / 2) + (a & 1);
      const uint8_t mk = mask[d];
      const T rv = (T)r[d];
      return mk ? (T)0 : rv;
    }
    return (T)o[k * bs + a];
  };
  T vr[L1_VPT];
  T wr = 0;
  T fmid[6];                  // forward: F of the middle row, for g_h
  if (!loader) {
#pragma unroll
    for (int u = 0; u < L1_VPT; ++u) {
      const int idx = tid + u * L1_COMPUTE;
      vr[u] = idx < nv ? v_load(idx) : (T)0;
    }
    if (BWD && tid < bs) {
      const long long d = 2 * ((long long)(s.y0 + mid) * g.nnx + s.x0 + tid / 2) + (tid & 1);
      const uint8_t mk = mask[d];
      const T rv = (T)r[d], g0 = (T)gm[tid], g1 = (T)gm[MAXBS + tid];
      wr = mk ? (T)0 : rv - (g0 + g1);
    }
    if (!BWD && tid < bs) {
      const T* F = base + (long long)(L - 1) * ring.rec + fo + tid * 6;
#pragma unroll
      for (int t = 0; t < 6; ++t) fmid[t] = F[t];
    }
  }
  if (gate()) {
    if (loader) wait_vmcnt(0);
    return;
  }
  if (!loader) {
#pragma unroll
    for (int u = 0; u < L1_VPT; ++u) {
      const int idx = tid + u * L1_COMPUTE;
      if (idx < nv) v[idx] = vr[u];
    }
    for (int idx = tid + L1_VPT * L1_COMPUTE; idx < nv; idx += L1_COMPUTE) v[idx] = v_load(idx);
    if (BWD && tid < bs) w[tid] = wr;
  }
  if (tid >= bs && tid < ncols) w[tid] = (T)0;   // padding columns
  if (loader) wait_vmcnt((npro - 1) * cw);       // record of step 0 is in its slot
  l1_barrier();

  // Position jp, finished at the previous step (parity pp), at entry col:
  // the sum of the group partial sums (forward-type steps produce the row,
  // backward steps subtract it from t_jp).  fin_load issues the LDS reads,
  // fin_value combines them, so that callers can issue all reads before
  // the first use (the compiler otherwise waits for each read in turn).
  static_assert(L1_NS <= 4, "group sums of a row fill one 16-byte group");
  struct Fin {
    T p[4];
    T y;
  };
  auto fin_load = [&](int jp, int pp, int col) -> Fin {
    Fin f;
    const T* pr = P + pp * (4 * MAXBS) + 4 * col;
    if constexpr (sizeof(T) == 4) {
      const float4 q = *reinterpret_cast<const float4*>(pr);
      f.p[0] = q.x;
      f.p[1] = q.y;
      f.p[2] = q.z;
      f.p[3] = q.w;
    } else {
      const double2 q0 = *reinterpret_cast<const double2*>(pr);
      const double2 q1 = *reinterpret_cast<const double2*>(pr + 2);
      f.p[0] = q0.x;
      f.p[1] = q0.y;
      f.p[2] = q1.x;
      f.p[3] = q1.y;
    }
    f.y = v[jp * bs + col];
    return f;
  };
  auto fin_value = [&](const Fin& f, bool pfwd) -> T {
    T acc = f.p[0];
#pragma unroll
    for (int q = 1; q < L1_NS; ++q) acc += f.p[q];
    return pfwd ? acc : f.y - acc;
  };

  for (int c = 0; c < nsteps; ++c) {
    const int j = pos_of(c);
    const int cur = c % R;
    const int prev = (c + R - 1) % R;
    const int pp = (c + 1) & 1;               // parity of step c-1
    const bool pfwd = !BWD || c == 1;         // step c-1 produced its row
    const int jp = BWD ? j + 1 : j - 1;       // position finished at step c-1
    // phase 1: w = right-hand side of the step
    if (tid < bs && c > 0) {
      // forward: F_j (couplings of position j with j-1, this step's
      // record), zero towards nodes outside the row, so a clamped index
      // contributes nothing; backward: F_{j+1} (couplings of position j+1
      // with j, in the previous step's slot) read transposed, entries
      // outside the row masked
      const T* F = !BWD ? reinterpret_cast<const T*>(lds + cur * ring.slot) + fo + tid * 6
                        : reinterpret_cast<const T*>(lds + prev * ring.slot) + fo;
      T f[6];
      Fin y[6];
      bool ok[6];
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const int di = t / 2 - 1, cc = t & 1;
        const int a = 2 * (ia + di) + cc;
        ok[t] = a >= 0 && a < bs;
        const int ac = min(max(a, 0), bs - 1);
        f[t] = !BWD ? F[t] : F[ac * 6 + (1 - di) * 2 + ca];
        y[t] = fin_load(jp, pp, ac);
      }
      const T rk = v[j * bs + tid];
      __builtin_amdgcn_sched_barrier(0);
      T acc = 0;
#pragma unroll
      for (int t = 0; t < 6; ++t) acc += (ok[t] ? f[t] : (T)0) * fin_value(y[t], pfwd);
      w[tid] = !BWD ? rk - acc : acc;
    } else if (!BWD && tid < bs) {
      w[tid] = v[tid];
    }
    l1_barrier();
    // phase 2: retire position jp into v (phase 1 may read t_jp there, so
    // not before the barrier); partial block GEMV; loaders issue the next
    // records (slots freed by steps up to c-1) and wait for the record of
    // step c+1
    if (gemv) {
      if (c > 0 && tid < bs) v[jp * bs + tid] = fin_value(fin_load(jp, pp, tid), pfwd);
      const T* Sr = reinterpret_cast<const T*>(lds + cur * ring.slot);
      if constexpr (sizeof(T) == 8)
        P[(c & 1) * (4 * MAXBS) + 4 * gi + gq] =
            lds_gemv_sym<L1_GMAX>(Sr, bs, gi, w, j0, jn);
      else
        P[(c & 1) * (4 * MAXBS) + 4 * gi + gq] =
            lds_gemv_group<T, L1_GMAX>(Sr + j0 * bs, bs, gi, w + j0, jn);
    } else if (loader) {
      if (c + R - 1 < nsteps)
        l1_dma<T>(base, ring.rec, pos_of(c + R - 1), lds + prev * ring.slot,
                  ring.nch, lw, lane);
      // the record of step c+1 has landed once at most the copies of the
      // records after it are in flight
      if (c + 1 < nsteps) wait_vmcnt((min(c + R, nsteps) - (c + 2)) * cw);
    }
    l1_barrier();
  }
  // retire the position of the last step (every record copy has been
  // waited for; the loaders' wait is a guard that no copy into LDS outlives
  // this system)
  {
    const int c = nsteps;
    const int jl = pos_of(c - 1);
    if (tid < bs) v[jl * bs + tid] = fin_value(fin_load(jl, (c + 1) & 1, tid), !BWD || c == 1);
  }
  if (loader) wait_vmcnt(0);
  l1_barrier();
  if (!BWD) {
    // g = F_{L-1} t_{L-2}, F_{L-1} read from the middle row's record in
    // the prologue
    if (tid < bs) {
      T acc = 0;
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const int di = t / 2 - 1, cc = t & 1;
        const int a = 2 * (ia + di) + cc;
        if (a >= 0 && a < bs) acc += fmid[t] * v[(L - 2) * bs + a];
      }
      gm[half * MAXBS + tid] = (double)acc;
    }
  }
  const int nout = (BWD && half == 0) ? L : L - 1;
  for (int idx = tid; idx < nout * bs; idx += AP_NT) {
    const int j = idx / bs, a = idx - (idx / bs) * bs;
    o[row_of(j) * bs + a] = (double)v[idx];
  }
}

// use64[i] != 0 (or use64 == null) selects the FP64 records of system i,
// else its FP32 copy (applied and accumulated in FP32).
struct L1Shared {
  double red[AP_NT / 64 + 1];
  int shi;
};

// Workgroup vb of one problem's first-level pass: system vb / 2, chain
// vb % 2.  With a.sc set, the forward pass first runs the CG convergence
// test on the update kernel's partials (check = 1) or reads the done word
// (check = 0); the backward pass reads the done word.
template <bool BWD>
__device__ __forceinline__ void level1_item(const Level1Args& a, int vb,
                                            unsigned char* lds, L1Shared& L) {
  auto gate = [&]() -> bool {
    if (a.sc == nullptr) return false;
    if (!BWD && a.check)
      return cg_check_done<AP_NT, L1_COMPUTE>(a.sc, a.part_upd, a.nb_upd, L.red, &L.shi, vb == 0);
    return block_read_done(a.sc, &L.shi);
  };
  const int bid = vb >> 1, half = vb & 1;
  const SysDesc s = a.sys[bid];
  double* gm = a.gmid + (long long)bid * 2 * MAXBS;
  if (a.S32 == nullptr || a.use64 == nullptr || a.use64[bid])
    level1_half<double, BWD>(a.g, s, half, a.mask, a.S64, a.r, a.lsol, gm, lds, gate);
  else
    level1_half<float, BWD>(a.g, s, half, a.mask, a.S32, a.r, a.lsol, gm, lds, gate);
}

// One pass (forward or backward) of the first-level solves: two workgroups
// per system.
template <bool BWD>
__global__ void __launch_bounds__(AP_NT) k_level1(Level1Args a) {
  __shared__ __align__(1024) unsigned char lds[L1_LDS];
  __shared__ L1Shared L;
  level1_item<BWD>(a, blockIdx.x, lds, L);
}

// One pass of the first-level solves of several problems in one persistent
// launch: workgroup w takes items w, w + grid, w + 2 grid, ... of the
// concatenated list (problem by problem, two per system), or of that list
// permuted by `order` when given (an item's result does not depend on the
// workgroup that computes it), so a grid of one per CU covers any batch.
template <bool BWD>
__global__ void __launch_bounds__(AP_NT)
k_level1_batch(const Level1Args* __restrict__ tab, const int* __restrict__ start,
               int nent, int total, const int* __restrict__ order) {
  __shared__ __align__(1024) unsigned char lds[L1_LDS];
  __shared__ L1Shared L;
  for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const int item = order != nullptr ? order[vb] : vb;
    const int e = batch_entry(start, nent, item);
    level1_item<BWD>(tab[e], item - start[e], lds, L);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------
// Heat eigenproblems (paper Section 4.1): on each coarse neighbourhood
// omega_l, the smallest eigenpairs of A psi = lambda M psi with
// A = sum_e E_e int grad N grad N, M = sum_e E_e int N N over the elements
// of omega_l (Neumann boundary, clamped nodes removed).  Shift-invert
// block subspace iteration with C = A + sigma M (block-tridiagonal inverse
// blocks from k_factor_twisted<1> and k_factor_middle<1>),
// M-orthonormalisation by Cholesky QR applied
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

// sum_b S[b*ld + i] * w[b*MAXM] for b < n (4 independent accumulators)
__device__ __forceinline__ double eig_dot(const double* S, int ld, int i,
                                          const double* w, int n) {
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  int b = 0;
#pragma unroll 2
  for (; b + 4 <= n; b += 4) {
    a0 += S[(b + 0) * ld + i] * w[(b + 0) * MAXM];
    a1 += S[(b + 1) * ld + i] * w[(b + 1) * MAXM];
    a2 += S[(b + 2) * ld + i] * w[(b + 2) * MAXM];
    a3 += S[(b + 3) * ld + i] * w[(b + 3) * MAXM];
  }
  for (; b < n; ++b) a0 += S[b * ld + i] * w[b * MAXM];
  return (a0 + a1) + (a2 + a3);
}


// K Y on node rows r0 <= k < r1 of a neighbourhood, K = sum_e kappa_e Kel4
// over the neighbourhood's elements (Kel4 the 4 x 4 element matrix, kappa_e
// the modulus; Dirichlet rows zero), through a rolling window of three node
// rows of Y in LDS: every Y value is read from memory once, and the reads
// of row k+2 go out before row k is formed.  Per row k, with the product
// row P_k (m x nxb) in LDS:
//   GRAM:  out (m x m, stride m, not symmetrised) += Y_k^T P_k on the FP64
//          matrix cores, wave w < 4 owning the 16 x 16 tile (w / 2, w % 2)
//          (lane l supplies Y(16R + l%16, t), P(16C + l%16, t) for the
//          row node t = 4K + l/16 and receives (16R + l/16 + 4r,
//          16C + l%16) in register r; rows past m hold stale values that
//          reach only dropped rows and columns);
//   else:  P_k is stored to Zout (rows k of its m columns).
// LDS (doubles, at win): three Y rows, P, three element-moduli rows, three
// flag rows, Kel4 (SW_DOUBLES in all).
constexpr int SW_RL = 74;                        // row stride (>= MAXBS + 1; banks)
constexpr int SW_Z = 3 * MAXM * SW_RL;           // product row
constexpr int SW_E = SW_Z + MAXM * SW_RL;        // moduli rows (columns x0-1 ..)
constexpr int SW_F = SW_E + 3 * SW_RL;           // Dirichlet flags (1.0 / 0.0)
constexpr int SW_K = SW_F + 3 * SW_RL;           // element matrix
constexpr int SW_DOUBLES = SW_K + 16;
constexpr int SW_PF = (MAXM * MAXBS + EG_NT - 1) / EG_NT;   // Y prefetch regs
static_assert(MAXBS + 1 <= SW_RL, "a moduli row needs nxb + 1 entries");
template <bool GRAM>
__device__ void stencil_rows(const Geom& g, const SysDesc& s,
                             const double* __restrict__ E,
                             const uint8_t* __restrict__ dflag,
                             const double* __restrict__ Kel4,
                             const double* __restrict__ Y, int n, int m, int r0,
                             int r1, double* __restrict__ out,
                             double* __restrict__ Zout, double* win) {
  const int tid = threadIdx.x;
  const int nxb = s.nxb, nyb = s.nyb;
  const int nrow = m * nxb;                    // Y values of a node row
  const int kpad = (nxb + 3) & ~3;             // K extent of the Gram tiles
  auto slot = [&](int kk) { return ((kk % 3) + 3) % 3; };
  // one node row kk of Y, its flags and the moduli row below it (element
  // row y0 + kk - 1), into registers / into the window
  double py[SW_PF], pe, pf;
  auto fetch = [&](int kk) {
    const bool rin = kk >= 0 && kk < nyb;
#pragma unroll
    for (int u = 0; u < SW_PF; ++u) {
      const int q = tid + u * EG_NT;
      const int j = q / nxb, i = q - (q / nxb) * nxb;
      py[u] = (rin && q < nrow) ? Y[(long long)j * n + kk * nxb + i] : 0.0;
    }
    pe = 0.0;
    pf = 0.0;
    if (tid <= nxb) {
      const int ex = s.x0 - 1 + tid, ey = s.y0 + kk - 1;
      if (ex >= s.ex0 && ex < s.ex1 && ey >= s.ey0 && ey < s.ey1)
        pe = E[(long long)ey * g.nx + ex];
    }
    if (tid < nxb && rin) pf = dflag[(long long)(s.y0 + kk) * g.nnx + s.x0 + tid] ? 1.0 : 0.0;
  };
  auto place = [&](int kk) {
    double* yw = win + slot(kk) * MAXM * SW_RL;
#pragma unroll
    for (int u = 0; u < SW_PF; ++u) {
      const int q = tid + u * EG_NT;
      if (q < nrow) {
        const int j = q / nxb, i = q - (q / nxb) * nxb;
        yw[j * SW_RL + i] = py[u];
      }
    }
    if (tid <= nxb) win[SW_E + slot(kk) * SW_RL + tid] = pe;
    if (tid < nxb) win[SW_F + slot(kk) * SW_RL + tid] = pf;
  };
  // Y and P padding columns nxb .. kpad-1 stay zero (the Gram's K padding)
  for (int q = tid; q < 4 * MAXM * (kpad - nxb); q += EG_NT) {
    const int r = q / (kpad - nxb), c = nxb + q % (kpad - nxb);
    win[r * SW_RL + c] = 0.0;
  }
  if (tid < 16) win[SW_K + tid] = Kel4[tid];
  fetch(r0 - 1);
  place(r0 - 1);
  fetch(r0);
  place(r0);
  fetch(r0 + 1);
  place(r0 + 1);
  __syncthreads();
  // stencil role: node i, columns jg, jg + ng, ...
  const int ng = EG_NT / nxb;
  const int i = tid % nxb, jg = tid / nxb;
  const bool st = jg < ng;
  // Gram role
  const int wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int R = wave >> 1, C = wave & 1;
  const bool act = GRAM && wave < 4 && 16 * R < m && 16 * C < m;
  eg_d4 acc = {0.0, 0.0, 0.0, 0.0};
  double* P = win + SW_Z;
  for (int k = r0; k < r1; ++k) {
    const bool pre = k + 2 <= r1;
    if (pre) fetch(k + 2);
    if (st) {
      // weights of the nine neighbours from the four elements around the
      // node (moduli rows k: above, k+1: below)
      double w9[9];
#pragma unroll
      for (int t = 0; t < 9; ++t) w9[t] = 0.0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int ex_ = e & 1, ey_ = e >> 1;
        const double ke = win[SW_E + slot(k + ey_) * SW_RL + i + ex_];
        const int va = (1 - ex_) + 2 * (1 - ey_);
#pragma unroll
        for (int vb = 0; vb < 4; ++vb) {
          const int ddx = ex_ - 1 + (vb & 1), ddy = ey_ - 1 + (vb >> 1);
          w9[(ddy + 1) * 3 + (ddx + 1)] += ke * win[SW_K + va * 4 + vb];
        }
      }
      const bool dir = win[SW_F + slot(k) * SW_RL + i] != 0.0;
      bool ok[9];
      int ofs[9];
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const int ddx = t % 3 - 1, ddy = t / 3 - 1;
        ok[t] = i + ddx >= 0 && i + ddx < nxb && k + ddy >= 0 && k + ddy < nyb;
        ofs[t] = slot(k + ddy) * MAXM * SW_RL + (ok[t] ? i + ddx : i);
      }
      for (int j = jg; j < m; j += ng) {
        double z = 0.0;
#pragma unroll
        for (int t = 0; t < 9; ++t) z += (ok[t] ? w9[t] : 0.0) * win[ofs[t] + j * SW_RL];
        z = dir ? 0.0 : z;
        if (GRAM) P[j * SW_RL + i] = z;
        else Zout[(long long)j * n + k * nxb + i] = z;
      }
    }
    __syncthreads();                           // P complete, row k-1 free
    if (act) {
      const double* ya = win + slot(k) * MAXM * SW_RL + (16 * R + li) * SW_RL + lk;
      const double* zb = P + (16 * C + li) * SW_RL + lk;
      for (int K = 0; K < kpad / 4; ++K)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ya[4 * K], zb[4 * K], acc, 0, 0, 0);
    }
    // (after the products, so that row k+2's reads had the longest time)
    if (pre) place(k + 2);
    __syncthreads();
  }
  if (act) {
    const int j = 16 * C + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ii = 16 * R + lk + 4 * r;
      if (ii < m && j < m) out[ii * m + j] = acc[r];
    }
  }
}


// Y <- Y L^{-T} on nodes n0 <= node < n1 (each node's row of m values
// solved with L).
__device__ void apply_linvT(const double* Yin, double* Y, int n, int m,
                            const double* L, int n0, int n1) {
  for (int node = n0 + threadIdx.x; node < n1; node += EG_NT) {
    double yv[MAXM];
#pragma unroll
    for (int j = 0; j < MAXM; ++j)
      if (j < m) yv[j] = Yin[(long long)j * n + node];
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
}


// X[:, c] = Y V[:, order[c]] (the Ritz vectors, ascending) on nodes
// n0 <= node < n1; one node per thread.
__device__ void ritz_vectors(const double* Y, double* X, const double* V,
                             const int* order, int n, int m, int n0, int n1) {
  for (int node = n0 + threadIdx.x; node < n1; node += EG_NT) {
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
}

// Shift-invert sweeps (k_eig_chain): block products S_k^{-1} Wl on the
// FP64 matrix cores, K steps of 4 over a block row.
constexpr int EG_NK = (MAXBS + 3) / 4;     // K steps of 4 over a block row
static_assert(EG_NK % 2 == 0, "the block GEMM pairs its K steps");
constexpr int EG_PFZ = (MAXBS * MAXM + EG_NT - 1) / EG_NT;               // row regs
constexpr int EG_RAW = 18176;              // doubles of the kernel's carved LDS
static_assert(SW_DOUBLES <= EG_RAW, "the sweep's LDS holds the stencil window");

// LDS doubles the sweep needs for bs, m (2 record slots, 2 vector rows,
// the right-hand side, the result rows and one more coupling block)
__host__ __device__ inline int eig_sweep_doubles(int bs, int m) {
  return 2 * heat_rec(bs) + 4 * bs * m + 3 * bs;
}

// the block size m fits the kernel for rows of bs nodes
__host__ __device__ inline bool eig_fits(int bs, int m) {
  // (the block GEMM's operand reads reach up to 2 m + 32 doubles past the
  // sweep buffers)
  return m >= 4 && m <= MAXM && bs <= MAXBS &&
         eig_sweep_doubles(bs, m) + 2 * m + 32 <= EG_RAW && 2 * MAXM * 64 <= EG_RAW;
}

// LDS-only workgroup barrier (the register prefetch stays in flight)
__device__ __forceinline__ void eg_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Per-neighbourhood state of the subspace iteration, kept in device memory
// between the iteration's kernels.
constexpr int EG_OB = 3;                   // row bands of a neighbourhood's streaming kernels
struct EigState {
  int done;                  // converged (or failed): later launches skip it
  int conv;                  // the last Rayleigh-Ritz step converged
  double theta[MAXM];        // Ritz values of the last Rayleigh-Ritz step
  double theta_old[MAXM];
  double gp[EG_OB][MAXM * MAXM];   // band parts of a Gram matrix
  double L[MAXM * MAXM];     // Cholesky factor, or the Ritz rotation V
  int order[MAXM];           // Ritz values ascending: their columns of V
};

size_t eig_state_bytes() { return sizeof(EigState); }

// X = random start block (a counter-based hash of neighbourhood, column and
// node: the same on every run), zero on Dirichlet nodes; state reset.
__global__ void __launch_bounds__(EG_NT)
k_eig_start(Geom g, const SysDesc* __restrict__ systems,
            const uint8_t* __restrict__ dflag, double* __restrict__ Xw,
            int m, EigState* __restrict__ st) {
  const SysDesc s = systems[blockIdx.x];
  const int tid = threadIdx.x;
  const int n = s.nxb * s.nyb;
  double* X = Xw + s.voff * (long long)m;
  for (int idx = tid; idx < n * m; idx += EG_NT) {
    const int j = idx / n, node = idx - (idx / n) * n;
    const int x = s.x0 + node % s.nxb, y = s.y0 + node / s.nxb;
    const bool d = dflag[(long long)y * g.nnx + x] != 0;
    const unsigned long long key =
        ((unsigned long long)blockIdx.x << 40) ^ ((unsigned long long)j << 24) ^ (unsigned long long)node;
    X[idx] = d ? 0.0 : hash_unit(key);
  }
  EigState& e = st[blockIdx.x];
  if (tid == 0) {
    e.done = 0;
    e.conv = 0;
  }
  if (tid < MAXM) e.theta_old[tid] = 0.0;
}

// Randomized setup (Section 3, applied to the heat pencils): X = nsnap
// uniform forcings in [-1, 1) per neighbourhood, SplitMix64 outputs at the
// state key ^ (seed * gamma), key = l * 2^40 + j * 2^24 + p (l the
// neighbourhood, j the snapshot, p the node's index in the neighbourhood's
// box, x fastest), zero on Dirichlet nodes, each shifted to zero M-mean over
// the kept nodes: f_j -= (w . f_j) / (w . 1), w = M 1 (column sums of the
// kept mass matrix).  Column nsnap (the last) is zero; it becomes the
// constant function after the local solves.  Z's first column holds w.
__global__ void __launch_bounds__(EG_NT)
k_rand_start(Geom g, const SysDesc* __restrict__ systems,
             const uint8_t* __restrict__ dflag, const double* __restrict__ E,
             const double* __restrict__ Me, double* __restrict__ Xw,
             double* __restrict__ Zw, int m, int nsnap, unsigned int seed,
             EigState* __restrict__ st) {
  __shared__ double red[EG_NT / 64 + 1];
  __shared__ double me[16];
  const SysDesc s = systems[blockIdx.x];
  const int tid = threadIdx.x;
  const int n = s.nxb * s.nyb;
  double* X = Xw + s.voff * (long long)m;
  double* w = Zw + s.voff * (long long)m;
  if (tid < 16) me[tid] = Me[tid];
  __syncthreads();
  double wsum = 0.0;
  for (int node = tid; node < n; node += EG_NT) {
    const int x = s.x0 + node % s.nxb, y = s.y0 + node / s.nxb;
    double wi = 0.0;
    if (!dflag[(long long)y * g.nnx + x]) {
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const int ex = x - 1 + dx, ey = y - 1 + dy;
          if (ex < s.ex0 || ex >= s.ex1 || ey < s.ey0 || ey >= s.ey1) continue;
          const double kap = E[(long long)ey * g.nx + ex];
          const int a = (1 - dx) + 2 * (1 - dy);
          for (int b = 0; b < 4; ++b) {
            const int bx = ex + (b & 1), by = ey + (b >> 1);
            if (!dflag[(long long)by * g.nnx + bx]) wi += kap * me[4 * a + b];
          }
        }
    }
    w[node] = wi;
    wsum += wi;
  }
  const double W = block_sum<EG_NT>(wsum, red);
  const unsigned long long sg = (unsigned long long)seed * 0x9E3779B97F4A7C15ull;
  for (int j = 0; j < m; ++j) {
    double sj = 0.0;
    for (int node = tid; node < n; node += EG_NT) {
      const int x = s.x0 + node % s.nxb, y = s.y0 + node / s.nxb;
      double f = 0.0;
      if (j < nsnap && !dflag[(long long)y * g.nnx + x]) {
        const unsigned long long key = ((unsigned long long)blockIdx.x << 40) |
                                       ((unsigned long long)j << 24) |
                                       (unsigned long long)node;
        f = hash_unit(key ^ sg);
      }
      X[(long long)j * n + node] = f;
      sj += w[node] * f;
    }
    const double mean = block_sum<EG_NT>(sj, red) / W;
    for (int node = tid; node < n; node += EG_NT) {
      const int x = s.x0 + node % s.nxb, y = s.y0 + node / s.nxb;
      if (j < nsnap && !dflag[(long long)y * g.nnx + x]) X[(long long)j * n + node] -= mean;
    }
  }
  EigState& e = st[blockIdx.x];
  if (tid == 0) {
    e.done = 0;
    e.conv = 0;
  }
  if (tid < MAXM) e.theta_old[tid] = 0.0;
}

// Column m-1 of Y := the constant function on the kept nodes.
__global__ void __launch_bounds__(EG_NT)
k_rand_const(Geom g, const SysDesc* __restrict__ systems,
             const uint8_t* __restrict__ dflag, double* __restrict__ Yw, int m) {
  const SysDesc s = systems[blockIdx.x];
  const int n = s.nxb * s.nyb;
  double* Y = Yw + s.voff * (long long)m + (long long)(m - 1) * n;
  for (int node = threadIdx.x; node < n; node += EG_NT) {
    const int x = s.x0 + node % s.nxb, y = s.y0 + node / s.nxb;
    Y[node] = dflag[(long long)y * g.nnx + x] ? 0.0 : 1.0;
  }
}

// One shift-invert step of every neighbourhood still iterating: Z = M X,
// then Y = C^{-1} Z by node rows in the factorisation's twisted order.
// Workgroup 2 l + h runs chain h of neighbourhood l (h = 0: rows 0..mid-1
// top-down; h = 1: rows nb-1..mid+1 bottom-up; mid = (nb - 1) / 2).
//   BWD = false: Z = M X on the chain's rows (h = 0 also on the middle
//     row), then the chain's forward steps; every forward row goes to Y,
//     the chain's last one also to its own Z row (Z rows mid-1 and mid+1
//     are not read again before the next Z = M X).
//   BWD = true: both workgroups solve the middle row from Z_mid and the
//     two chain ends (h = 0 stores it), then run their chain backwards.
// Record of row k: [S_k^{-1} (bs x bs, column-major) | F (bs x 3: coupling
// with the previous row of its chain) | G (bs x 3: with the next row; for
// a chain's last row, the middle row)]; the middle row has two records,
// index mid (F: coupling with row mid-1) and index nb (F: with row mid+1).
// Step c: phase A forms the right-hand side Wl from the previous step's
// result rows T (LDS) and the record's coupling (forward Wl = Z_k - F T,
// backward Wl = G T, middle Wl = Z_mid - F T_top - F' T_bottom) and
// stores the previous T to Y; phase B computes T = S_k^{-1} Wl (forward,
// middle) or T = Y_k - S_k^{-1} Wl (backward) on the matrix cores.  While
// step c runs, the record of step c+1 is copied into the other LDS slot
// (direct-to-LDS loads) and its vector row (Z forward, the forward Y
// backward) is held in registers.
template <bool BWD>
__device__ void eig_chain_item(const Geom& g, const SysDesc* __restrict__ systems,
                               const double* __restrict__ E,
                               const uint8_t* __restrict__ dflag,
                               const double* __restrict__ Me,
                               const double* __restrict__ Sinv,
                               const double* __restrict__ Xw, double* __restrict__ Yw,
                               double* __restrict__ Zw, int m,
                               const EigState* __restrict__ st, int sys, int h,
                               double* raw) {
  if (st[sys].done) return;
  const SysDesc s = systems[sys];
  const int tid = threadIdx.x;
  const int n = s.nxb * s.nyb;
  const int bs = s.nxb, nb = s.nyb;
  const int mid = (nb - 1) >> 1;
  const int len = h == 0 ? mid : nb - 1 - mid;          // rows of the chain
  const long long wo = s.voff * (long long)m;
  const double* X = Xw + wo;
  double* Y = Yw + wo;
  double* Z = Zw + wo;
  if (!BWD) {
    const int r0 = h == 0 ? 0 : mid + 1, r1 = h == 0 ? mid + 1 : nb;
    stencil_rows<false>(g, s, E, dflag, Me, X, n, m, r0, r1, nullptr, Z, raw);
    __syncthreads();
    if (len == 0) return;
  }
  // node row and record index of step c
  auto row_of = [&](int c) {
    return BWD ? (h == 0 ? mid - c : mid + c) : (h == 0 ? c : nb - 1 - c);
  };
  auto rec_of = [&](int c) {
    return BWD ? (h == 0 ? mid - c : (c == 0 ? mid : nb - c))
               : (h == 0 ? c : mid + 1 + c);
  };
  const int nsteps = BWD ? len + 1 : len;
  // sweep buffers in LDS, addressed by offsets into raw (so that every
  // access stays an LDS access): two record slots, two vector rows, the
  // right-hand side Wl and the result rows T ([a][j], stride m), and the
  // middle row's second coupling
  const int rec = heat_rec(bs);              // even
  const int bm = bs * m;
  const int o_z = 2 * rec, o_w = o_z + 2 * bm, o_t = o_w + bm, o_fb = o_t + bm;
  const double* recs = Sinv + s.foff;
  // vector-row role: entries q = tid + u * EG_NT, q = j * bs + a
  int qa[EG_PFZ], qj[EG_PFZ];
#pragma unroll
  for (int u = 0; u < EG_PFZ; ++u) {
    const int q = tid + u * EG_NT;
    qj[u] = q < bm ? q / bs : -1;
    qa[u] = q < bm ? q - (q / bs) * bs : 0;
  }
  {
    const double* r0p = recs + (long long)rec_of(0) * rec;
    for (int q = tid; q < rec; q += EG_NT) raw[q] = r0p[q];
  }
#pragma unroll
  for (int u = 0; u < EG_PFZ; ++u)
    if (qj[u] >= 0)
      raw[o_z + tid + u * EG_NT] = Z[(long long)qj[u] * n + row_of(0) * bs + qa[u]];
  if (BWD) {
    // the chain ends (forward rows mid-1 and mid+1, zero where a chain is
    // empty) as result rows, the bottom one in the other vector slot, and
    // the coupling of the middle row with row mid+1
    for (int q = tid; q < bm; q += EG_NT) {
      const int j = q / bs, a = q - (q / bs) * bs;
      raw[o_t + a * m + j] = mid > 0 ? Z[(long long)j * n + (mid - 1) * bs + a] : 0.0;
      raw[o_z + bm + a * m + j] =
          mid + 1 < nb ? Z[(long long)j * n + (mid + 1) * bs + a] : 0.0;
    }
    const double* fb = recs + (long long)nb * rec + bs * bs;
    for (int q = tid; q < 3 * bs; q += EG_NT) raw[o_fb + q] = fb[q];
  }
  __syncthreads();
  // block GEMM roles: 16-row tiles on the matrix cores (wave w takes tiles
  // w, w + 8, ...; the last tile row zero-padded)
  const int nrt = (bs + 15) >> 4, nct = (m + 15) >> 4;
  const int nk = (bs + 3) >> 2;
  const int wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  for (int c = 0; c < nsteps; ++c) {
    const int kp = c > 0 ? row_of(c - 1) : 0;      // row of the previous step
    const int cur = c & 1;
    const int o_s = cur ? rec : 0, o_sn = cur ? 0 : rec;       // this / other slot
    const int o_zc = o_z + (cur ? bm : 0), o_zn = o_z + (cur ? 0 : bm);
    const bool mstep = BWD && c == 0;            // the middle row
    const bool sub = BWD && c > 0;               // T = Y_k - S_k^{-1} Wl
    const bool keep = c > 0 && !(BWD && c == 1 && h == 1);   // store the previous T
    // prefetch step c+1: the record straight into the other LDS slot
    // (direct-to-LDS loads of 16 bytes a lane, 1 KiB a wave, clipped at the
    // record's end; this step reads only its own record), and the vector
    // row into registers
    double pz[EG_PFZ];
    const bool pf = c + 1 < nsteps;
    if (pf) {
      const unsigned char* rsrc =
          reinterpret_cast<const unsigned char*>(recs + (long long)rec_of(c + 1) * rec);
      unsigned char* rdst = reinterpret_cast<unsigned char*>(raw + o_sn);
      const int rbytes = 8 * rec;
      for (int q = wave; q * 1024 < rbytes; q += EG_NT / 64) {
        const int off = q * 1024 + 16 * lane;
        if (off < rbytes)
          __builtin_amdgcn_global_load_lds((const void*)(rsrc + off),
                                           (lds_void*)(rdst + q * 1024), 16, 0, 0);
      }
      const double* vsrc = (BWD ? Y : Z) + (long long)row_of(c + 1) * bs;
#pragma unroll
      for (int u = 0; u < EG_PFZ; ++u) pz[u] = vsrc[(long long)max(qj[u], 0) * n + qa[u]];
    }
    // phase A (all of a thread's reads come first: the writes go to the
    // same LDS array)
    auto phase_a = [&](auto u0c, auto u1c) {
      constexpr int U0 = decltype(u0c)::value, U1 = decltype(u1c)::value;
      const int o_f = o_s + bs * bs + (sub ? 3 * bs : 0);
      double fa[U1 - U0][3], ta[U1 - U0][3], za[U1 - U0];
#pragma unroll
      for (int u = U0; u < U1; ++u) {
        const int j = max(qj[u], 0), a = qa[u];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const int b = min(max(a + t - 1, 0), bs - 1);
          fa[u - U0][t] = raw[o_f + a * 3 + t];
          ta[u - U0][t] = raw[o_t + b * m + j];
        }
        za[u - U0] = raw[o_zc + (qj[u] >= 0 ? tid + u * EG_NT : 0)];
      }
#pragma unroll
      for (int u = U0; u < U1; ++u) {
        const int j = qj[u], a = qa[u];
        if (j < 0) continue;
        double w = sub ? 0.0 : za[u - U0];
        if (keep) Y[(long long)j * n + kp * bs + a] = ta[u - U0][1];
        if (c > 0 || mstep) {
          // (at step 0 of a forward chain the result rows hold nothing)
#pragma unroll
          for (int t = 0; t < 3; ++t) {
            const bool ok = (a + t - 1) >= 0 && (a + t - 1) < bs;
            const double f = ok ? fa[u - U0][t] : 0.0;
            w = sub ? w + f * ta[u - U0][t] : w - f * ta[u - U0][t];
          }
        }
        raw[o_w + a * m + j] = w;
      }
    };
    phase_a(std::integral_constant<int, 0>(), std::integral_constant<int, EG_PFZ / 2 + 1>());
    if (qj[EG_PFZ / 2 + 1] >= 0)
      phase_a(std::integral_constant<int, EG_PFZ / 2 + 1>(), std::integral_constant<int, EG_PFZ>());
    if (mstep) {
      // the middle row's coupling with the bottom chain's end
#pragma unroll
      for (int u = 0; u < EG_PFZ; ++u) {
        const int j = qj[u], a = qa[u];
        if (j < 0) continue;
        double w = raw[o_w + a * m + j];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const int b = a + t - 1;
          if (b >= 0 && b < bs) w -= raw[o_fb + a * 3 + t] * raw[o_zn + b * m + j];
        }
        raw[o_w + a * m + j] = w;
      }
    }
    eg_barrier();
    // phase B: per FP64 MFMA 16x16x4, lane l supplies S(16R + l%16, b) and
    // Wl(b, 16C + l%16) for b = 4K + l/16 (zero outside the block) and
    // receives T(16R + l/16 + 4r, 16C + l%16) in register r.  Operand reads
    // run EG_PD K steps ahead; two accumulators take alternate K steps.
    for (int tl = wave; tl < nrt * nct; tl += EG_NT / 64) {
      const int R = tl / nct, C = tl - (tl / nct) * nct;
      const int ia = 16 * R + li, jb = 16 * C + li;
      // Rows ia >= bs and columns jb >= m of the operands read neighbouring
      // LDS data: they reach only output rows and columns that are
      // dropped.  Only the last K step, whose b can pass the block, is
      // masked.
      const double* pa = raw + o_s + lk * bs + ia;
      const double* pw = raw + o_w + lk * m + jb;
      const int sa = 4 * bs, sw = 4 * m;
      constexpr int EG_PD = 4;
      double av[EG_PD], wv[EG_PD];
      const int kl = max(nk - 2, 0);            // last unmasked K step
#pragma unroll
      for (int K = 0; K < EG_PD; ++K) {
        const int Kc = min(K, kl);
        av[K] = pa[Kc * sa];
        wv[K] = pw[Kc * sw];
      }
      eg_d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int K = 0; K < EG_NK; ++K) {
        const double ae = av[K % EG_PD], we = wv[K % EG_PD];
        if (K + EG_PD < EG_NK) {
          const int Kc = min(K + EG_PD, kl);
          av[K % EG_PD] = pa[Kc * sa];
          wv[K % EG_PD] = pw[Kc * sw];
        }
        if (K < nk - 1) {
          if (K & 1)
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ae, we, acc1, 0, 0, 0);
          else
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ae, we, acc0, 0, 0, 0);
        }
      }
      {
        // last K step: b past the block reads as zero
        const bool ok = 4 * (nk - 1) + lk < bs;
        const double ae = ok ? pa[(nk - 1) * sa] : 0.0, we = ok ? pw[(nk - 1) * sw] : 0.0;
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ae, we, acc0, 0, 0, 0);
      }
      if (jb < m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * R + lk + 4 * r;
          if (i < bs) {
            const double t = acc0[r] + acc1[r];
            raw[o_t + i * m + jb] = sub ? raw[o_zc + jb * bs + i] - t : t;
          }
        }
      }
    }
    if (pf) {
#pragma unroll
      for (int u = 0; u < EG_PFZ; ++u)
        if (qj[u] >= 0) raw[o_zn + tid + u * EG_NT] = pz[u];
    }
    // this wave's record copies have landed in LDS
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    eg_barrier();
  }
  // the last step's result rows (a forward chain's end also into its Z row)
  const int kl = row_of(nsteps - 1);
  const bool keep = !(BWD && nsteps == 1 && h == 1);
#pragma unroll
  for (int u = 0; u < EG_PFZ; ++u)
    if (qj[u] >= 0) {
      const long long gi = (long long)qj[u] * n + kl * bs + qa[u];
      const double v = raw[o_t + qa[u] * m + qj[u]];
      if (keep) Y[gi] = v;
      if (!BWD) Z[gi] = v;
    }
}

// Workgroups take their (neighbourhood, chain) items from pack (see
// chain_items): one workgroup per CU covers every chain.
template <bool BWD>
__global__ void __launch_bounds__(EG_NT)
k_eig_chain(Geom g, const SysDesc* __restrict__ systems,
            const double* __restrict__ E, const uint8_t* __restrict__ dflag,
            const double* __restrict__ Me, const double* __restrict__ Sinv,
            const double* __restrict__ Xw, double* __restrict__ Yw,
            double* __restrict__ Zw, int m, const EigState* __restrict__ st,
            const int* __restrict__ pack) {
  __shared__ __align__(16) double raw[EG_RAW];
  const int q0 = pack[blockIdx.x], q1 = pack[blockIdx.x + 1];
  for (int q = q0; q < q1; ++q) {
    const int item = pack[gridDim.x + 1 + q];
    eig_chain_item<BWD>(g, systems, E, dflag, Me, Sinv, Xw, Yw, Zw, m, st,
                        item >> 1, item & 1, raw);
    __syncthreads();
  }
}

// M-orthonormalisation of Y by Cholesky QR into X (twice at a
// Rayleigh-Ritz step), and Rayleigh-Ritz with A on span(X): the Ritz
// vectors replace X, ascending, and the Ritz values that decide the
// selection (those below the threshold, at most kmax, and the next one)
// are tested for convergence.  Streaming work runs in EG_OB row bands per
// neighbourhood (workgroup EG_OB l + b), the small dense work in one
// workgroup per neighbourhood:
//   k_orth_gram   Z = M_e src on the band's rows, the band's part of src^T Z
//   k_orth_chol   G = sum of the parts (band order), symmetrised; L L^T = G
//   k_orth_linvT  dst = src L^{-T} on the band's rows
//   k_orth_rr     G as above (A_e), Jacobi, Ritz values ascending, test
//   k_orth_ritz   X = X V (columns in ascending Ritz order) on the band

// node range [n0, n1) of band b (whole node rows)
__device__ __forceinline__ void eig_band(const SysDesc& s, int b, int* n0, int* n1) {
  *n0 = ((b * s.nyb) / EG_OB) * s.nxb;
  *n1 = (((b + 1) * s.nyb) / EG_OB) * s.nxb;
}

// (at most 128 registers: two workgroups per CU)
__global__ void __launch_bounds__(EG_NT, 4)
k_orth_gram(Geom g, const SysDesc* __restrict__ systems,
            const double* __restrict__ E, const uint8_t* __restrict__ dflag,
            const double* __restrict__ Kel4, const double* __restrict__ Srcw,
            double* __restrict__ Zw, int m, EigState* __restrict__ st) {
  __shared__ __align__(16) double win[SW_DOUBLES];
  const int sys = blockIdx.x / EG_OB, b = blockIdx.x - (blockIdx.x / EG_OB) * EG_OB;
  EigState& es = st[sys];
  if (es.done) return;
  const SysDesc s = systems[sys];
  const int n = s.nxb * s.nyb;
  const long long wo = s.voff * (long long)m;
  int n0, n1;
  eig_band(s, b, &n0, &n1);
  (void)Zw;
  stencil_rows<true>(g, s, E, dflag, Kel4, Srcw + wo, n, m, n0 / s.nxb, n1 / s.nxb,
                     es.gp[b], nullptr, win);
}

// G (LDS, stride m) = the sum of the band parts in band order, symmetrised
__device__ void orth_gather(const EigState& es, int m, double* G) {
  for (int e = threadIdx.x; e < m * m; e += EG_NT) {
    double v = 0.0;
#pragma unroll
    for (int b = 0; b < EG_OB; ++b) v += es.gp[b][e];
    G[e] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < m * m; e += EG_NT) {
    const int a = e / m, c = e - (e / m) * m;
    if (a < c) {
      const double v = 0.5 * (G[a * m + c] + G[c * m + a]);
      G[a * m + c] = v;
      G[c * m + a] = v;
    }
  }
  __syncthreads();
}

__global__ void __launch_bounds__(EG_NT)
k_orth_chol(int m, EigState* __restrict__ st, int* __restrict__ err) {
  __shared__ double G[MAXM * MAXM];
  EigState& es = st[blockIdx.x];
  if (es.done) return;
  orth_gather(es, m, G);
  chol_small<EG_NT>(G, m, err);
  for (int e = threadIdx.x; e < m * m; e += EG_NT) es.L[e] = G[e];
}

__global__ void __launch_bounds__(EG_NT)
k_orth_linvT(const SysDesc* __restrict__ systems, const double* __restrict__ Srcw,
             double* __restrict__ Dstw, int m, const EigState* __restrict__ st) {
  __shared__ double L[MAXM * MAXM];
  const int sys = blockIdx.x / EG_OB, b = blockIdx.x - (blockIdx.x / EG_OB) * EG_OB;
  const EigState& es = st[sys];
  if (es.done) return;
  const SysDesc s = systems[sys];
  const long long wo = s.voff * (long long)m;
  for (int e = threadIdx.x; e < m * m; e += EG_NT) L[e] = es.L[e];
  __syncthreads();
  int n0, n1;
  eig_band(s, b, &n0, &n1);
  apply_linvT(Srcw + wo, Dstw + wo, s.nxb * s.nyb, m, L, n0, n1);
}

__global__ void __launch_bounds__(EG_NT)
k_orth_rr(EigParams prm, int first_rr, EigState* __restrict__ st) {
  __shared__ double G[MAXM * MAXM];
  __shared__ double V[MAXM * MAXM];
  __shared__ double rc[MAXM], rs[MAXM];
  __shared__ int rp[MAXM], rq[MAXM], order[MAXM];
  EigState& es = st[blockIdx.x];
  if (es.done) return;
  const int tid = threadIdx.x;
  const int m = prm.m;
  orth_gather(es, m, G);
  jacobi_small<EG_NT>(G, V, m, rc, rs, rp, rq);
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
    int nbelow = 0;
    for (int i = 0; i < m; ++i) {
      es.theta[i] = G[order[i] * m + order[i]];
      if (es.theta[i] < prm.lim) ++nbelow;
    }
    const int nchk = min(m - 1, min(nbelow, prm.kmax) + 1);
    double dmax = 0.0;
    for (int i = 0; i < nchk; ++i) {
      const double rel = fabs(es.theta[i] - es.theta_old[i]) / (fabs(es.theta[i]) + prm.lim);
      dmax = fmax(dmax, rel);
    }
    for (int i = 0; i < m; ++i) es.theta_old[i] = es.theta[i];
    // k_eig_count turns this into done once the Ritz vectors are formed
    es.conv = (!first_rr && dmax < prm.tol) ? 1 : 0;
  }
  __syncthreads();
  for (int e = tid; e < m * m; e += EG_NT) es.L[e] = V[e];
  if (tid < m) es.order[tid] = order[tid];
}

__global__ void __launch_bounds__(EG_NT)
k_orth_ritz(const SysDesc* __restrict__ systems, double* __restrict__ Xw, int m,
            const EigState* __restrict__ st) {
  __shared__ double V[MAXM * MAXM];
  __shared__ int order[MAXM];
  const int sys = blockIdx.x / EG_OB, b = blockIdx.x - (blockIdx.x / EG_OB) * EG_OB;
  const EigState& es = st[sys];
  if (es.done) return;
  const SysDesc s = systems[sys];
  const long long wo = s.voff * (long long)m;
  for (int e = threadIdx.x; e < m * m; e += EG_NT) V[e] = es.L[e];
  if (threadIdx.x < m) order[threadIdx.x] = es.order[threadIdx.x];
  __syncthreads();
  int n0, n1;
  eig_band(s, b, &n0, &n1);
  ritz_vectors(Xw + wo, Xw + wo, V, order, s.nxb * s.nyb, m, n0, n1);
}

// After a Rayleigh-Ritz step: neighbourhoods whose Ritz values converged
// stop iterating; the number still iterating goes to *count (one
// workgroup).
__global__ void __launch_bounds__(256)
k_eig_count(EigState* __restrict__ st, int nsys, int* __restrict__ count) {
  __shared__ int c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  int mine = 0;
  for (int i = threadIdx.x; i < nsys; i += 256) {
    if (!st[i].done && st[i].conv) st[i].done = 1;
    mine += st[i].done ? 0 : 1;
  }
  if (mine) atomicAdd(&c, mine);
  __syncthreads();
  if (threadIdx.x == 0) *count = c;
}

// X holds the Ritz vectors (ascending): select lambda < lim, at most kmax.
__global__ void __launch_bounds__(EG_NT)
k_eig_select(const SysDesc* __restrict__ systems, const double* __restrict__ Xw,
             EigParams prm, const EigState* __restrict__ st,
             double* __restrict__ psi_out, float* __restrict__ psi32_out,
             double* __restrict__ lam_out, int* __restrict__ nsel_out,
             int* __restrict__ cap_out) {
  __shared__ int nsel;
  const SysDesc s = systems[blockIdx.x];
  const int tid = threadIdx.x;
  const int n = s.nxb * s.nyb;
  const EigState& es = st[blockIdx.x];
  const double* X = Xw + s.voff * (long long)prm.m;
  if (tid == 0) {
    int cnt = 0;
    for (int i = 0; i < prm.m; ++i)
      if (es.theta[i] < prm.lim) ++cnt;
    nsel = min(cnt, prm.kmax);
    nsel_out[blockIdx.x] = nsel;
    cap_out[blockIdx.x] = (cnt > prm.kmax) ? 1 : 0;
    for (int i = 0; i < prm.kmax; ++i)
      lam_out[(long long)blockIdx.x * prm.kmax + i] = (i < nsel) ? es.theta[i] : __builtin_nan("");
  }
  __syncthreads();
  // with psi32_out the modes are rounded to FP32 and both copies hold the
  // rounded values: the coarse space is the span of the rounded modes
  double* po = psi_out + s.voff * (long long)prm.kmax;
  float* po32 = psi32_out ? psi32_out + s.voff * (long long)prm.kmax : nullptr;
  for (int idx = tid; idx < nsel * n; idx += EG_NT) {
    const double x = X[idx];
    if (po32 != nullptr) {
      const float f = (float)x;
      po32[idx] = f;
      po[idx] = (double)f;
    } else {
      po[idx] = x;
    }
  }
}

// ---------------------------------------------------------------- launchers

// Work items of the twisted chain kernels: item 2 i + h is chain h of
// system i (h = 0: node rows 0..m with the middle row m = (nyb - 1) / 2,
// h = 1: rows nyb-1..m).  They are packed onto at most ncu workgroups,
// longest first onto the least loaded one (cost: rows x (nxb^2 + 64^2), the
// constant standing for a step's fixed latency), so that on a mesh whose
// boundary systems are smaller, short chains share a workgroup and one
// workgroup per CU covers all.  pack: per workgroup the first item's
// position (P + 1 offsets), then the items; returns P.
int chain_items(const std::vector<SysDesc>& sys, int ncu, std::vector<int>& pack) {
  struct It {
    double cost;
    int item;
  };
  std::vector<It> its;
  for (size_t i = 0; i < sys.size(); ++i) {
    const int m = (sys[i].nyb - 1) / 2;
    for (int h = 0; h < 2; ++h) {
      const int rows = h == 0 ? m + 1 : sys[i].nyb - m;
      its.push_back({(double)rows * ((double)sys[i].nxb * sys[i].nxb + 4096.0),
                     (int)(2 * i + h)});
    }
  }
  std::stable_sort(its.begin(), its.end(),
                   [](const It& a, const It& b) { return a.cost > b.cost; });
  const int P = std::max(1, std::min(ncu, (int)its.size()));
  std::vector<double> load(P, 0.0);
  std::vector<std::vector<int>> bins(P);
  for (const It& it : its) {
    int best = 0;
    for (int b = 1; b < P; ++b)
      if (load[b] < load[best]) best = b;
    load[best] += it.cost;
    bins[best].push_back(it.item);
  }
  pack.assign(P + 1 + its.size(), 0);
  int q = 0;
  for (int b = 0; b < P; ++b) {
    pack[b] = q;
    for (int it : bins[b]) pack[P + 1 + q++] = it;
  }
  pack[P] = q;
  return P;
}

void launch_factor_elastic(const Geom& g, const SysDesc* sys, int nsys,
                           const double* E, const uint8_t* mask,
                           const double* Ke, double* out64, float* out32,
                           double* metric, int* err, const int* pack, int npack,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_factor_twisted<2>, dim3(npack), dim3(FT_NT), 0, s, g,
                     sys, nsys, E, mask, Ke, out64, out32, metric, err, pack);
  hipLaunchKernelGGL(k_factor_middle<2>, dim3(nsys), dim3(FT_NT), 0, s, g, sys,
                     nsys, E, mask, Ke, out64, out32, metric, err);
}

void launch_factor_heat(const Geom& g, const SysDesc* sys, int nsys,
                        const double* E, const uint8_t* dflag,
                        const double* Cel, double* out, int* err,
                        const int* pack, int npack, hipStream_t s) {
  hipLaunchKernelGGL(k_factor_twisted<1>, dim3(npack), dim3(FT_NT), 0, s, g,
                     sys, nsys, E, dflag, Cel, out, (float*)nullptr,
                     (double*)nullptr, err, pack);
  hipLaunchKernelGGL(k_factor_middle<1>, dim3(nsys), dim3(FT_NT), 0, s, g, sys,
                     nsys, E, dflag, Cel, out, (float*)nullptr, (double*)nullptr,
                     err);
}

void launch_level1(const Level1Args& a, int nsys, hipStream_t s) {
  hipLaunchKernelGGL(k_level1<false>, dim3(2 * nsys), dim3(AP_NT), 0, s, a);
  hipLaunchKernelGGL(k_level1<true>, dim3(2 * nsys), dim3(AP_NT), 0, s, a);
}

void launch_level1_batch(const Level1Args* tab, const int* start, int nent,
                         int total, int grid, const int* order, hipStream_t s) {
  hipLaunchKernelGGL(k_level1_batch<false>, dim3(grid), dim3(AP_NT), 0, s, tab,
                     start, nent, total, order);
  hipLaunchKernelGGL(k_level1_batch<true>, dim3(grid), dim3(AP_NT), 0, s, tab,
                     start, nent, total, order);
}

bool eig_fits_host(int bs, int m) { return eig_fits(bs, m); }

bool level1_fits(int bs, int nb, bool fp32) {
  const int L = nb - (nb - 1) / 2;     // the longer chain of the twisted sweep
  return l1_fits<double>(bs, L) && (!fp32 || l1_fits<float>(bs, L));
}

// Returns the number of neighbourhoods whose deciding Ritz values had not
// settled when the iteration limit was reached (0 when all converged), or
// -1 if a HIP call failed (the selection is then not launched).
int launch_heat_eigen(const Geom& g, const SysDesc* sys, int nsys,
                      const double* E, const uint8_t* dflag, const double* Ae,
                      const double* Me, const double* Sinv, double* X,
                      double* Y, double* Z, int m, int kmax, int maxit,
                      int rr_every, double lim, double tol, void* state,
                      int* d_count, int* h_count, double* psi, float* psi32,
                      double* lam, int* nsel, int* cap, int* err,
                      const int* pack, int npack, int nsnap,
                      unsigned int seed, hipStream_t s) {
  EigParams p{m, kmax, maxit, rr_every, lim, tol};
  EigState* st = static_cast<EigState*>(state);
  if (nsnap > 0) {
    // randomized (Section 3): one pass of local solves on zero-mean random
    // forcings, the constant function appended, an M-orthonormal basis of
    // the snapshot space (Cholesky QR twice) and Rayleigh-Ritz on it
    hipLaunchKernelGGL(k_rand_start, dim3(nsys), dim3(EG_NT), 0, s, g, sys, dflag,
                       E, Me, X, Z, m, nsnap, seed, st);
    hipLaunchKernelGGL(k_eig_chain<false>, dim3(npack), dim3(EG_NT), 0, s, g,
                       sys, E, dflag, Me, Sinv, X, Y, Z, m, st, pack);
    hipLaunchKernelGGL(k_eig_chain<true>, dim3(npack), dim3(EG_NT), 0, s, g,
                       sys, E, dflag, Me, Sinv, X, Y, Z, m, st, pack);
    hipLaunchKernelGGL(k_rand_const, dim3(nsys), dim3(EG_NT), 0, s, g, sys, dflag, Y, m);
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(k_orth_gram, dim3(EG_OB * nsys), dim3(EG_NT), 0, s, g,
                         sys, E, dflag, Me, pass ? X : Y, Z, m, st);
      hipLaunchKernelGGL(k_orth_chol, dim3(nsys), dim3(EG_NT), 0, s, m, st, err);
      hipLaunchKernelGGL(k_orth_linvT, dim3(EG_OB * nsys), dim3(EG_NT), 0, s,
                         sys, pass ? X : Y, X, m, st);
    }
    hipLaunchKernelGGL(k_orth_gram, dim3(EG_OB * nsys), dim3(EG_NT), 0, s, g,
                       sys, E, dflag, Ae, X, Z, m, st);
    hipLaunchKernelGGL(k_orth_rr, dim3(nsys), dim3(EG_NT), 0, s, p, 1, st);
    hipLaunchKernelGGL(k_orth_ritz, dim3(EG_OB * nsys), dim3(EG_NT), 0, s, sys,
                       X, m, st);
    hipLaunchKernelGGL(k_eig_select, dim3(nsys), dim3(EG_NT), 0, s, sys, X, p, st,
                       psi, psi32, lam, nsel, cap);
    if (hipGetLastError() != hipSuccess) return -1;
    return 0;
  }
  hipLaunchKernelGGL(k_eig_start, dim3(nsys), dim3(EG_NT), 0, s, g, sys, dflag, X, m, st);
  bool first_rr = true;
  int unconverged = nsys;
  for (int it = 0; it < maxit; ++it) {
    hipLaunchKernelGGL(k_eig_chain<false>, dim3(npack), dim3(EG_NT), 0, s, g,
                       sys, E, dflag, Me, Sinv, X, Y, Z, m, st, pack);
    hipLaunchKernelGGL(k_eig_chain<true>, dim3(npack), dim3(EG_NT), 0, s, g,
                       sys, E, dflag, Me, Sinv, X, Y, Z, m, st, pack);
    const bool rr = ((it + 1) % rr_every == 0) || (it + 1 == maxit);
    // X = Y L^{-T} with L L^T = Y^T M Y (in place with src = dst = X)
    auto orth_pass = [&](const double* src, double* dst) {
      hipLaunchKernelGGL(k_orth_gram, dim3(EG_OB * nsys), dim3(EG_NT), 0, s, g,
                         sys, E, dflag, Me, src, Z, m, st);
      hipLaunchKernelGGL(k_orth_chol, dim3(nsys), dim3(EG_NT), 0, s, m, st, err);
      hipLaunchKernelGGL(k_orth_linvT, dim3(EG_OB * nsys), dim3(EG_NT), 0, s,
                         sys, src, dst, m, st);
    };
    orth_pass(Y, X);
    if (rr) {
      orth_pass(X, X);
      hipLaunchKernelGGL(k_orth_gram, dim3(EG_OB * nsys), dim3(EG_NT), 0, s, g,
                         sys, E, dflag, Ae, X, Z, m, st);
      hipLaunchKernelGGL(k_orth_rr, dim3(nsys), dim3(EG_NT), 0, s, p,
                         first_rr ? 1 : 0, st);
      hipLaunchKernelGGL(k_orth_ritz, dim3(EG_OB * nsys), dim3(EG_NT), 0, s, sys,
                         X, m, st);
    }
    if (rr) {
      first_rr = false;
      hipLaunchKernelGGL(k_eig_count, dim3(1), dim3(256), 0, s, st, nsys, d_count);
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(h_count, d_count, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return -1;
      unconverged = *h_count;
      if (unconverged == 0) break;
    }
  }
  hipLaunchKernelGGL(k_eig_select, dim3(nsys), dim3(EG_NT), 0, s, sys, X, p, st,
                     psi, psi32, lam, nsel, cap);
  if (hipGetLastError() != hipSuccess) return -1;
  return unconverged;
}

}  // namespace msp
