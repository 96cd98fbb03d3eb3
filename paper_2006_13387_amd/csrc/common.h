// Shared host/device definitions of libmsp (2D Q1 path).
//
// Layout conventions (all device arrays, interleaved DOFs):
//   vectors   : n_dofs doubles, DOF 2*node + c
//   E         : n_elems doubles (SIMP moduli), element i + nx*j
//   mask      : n_dofs bytes, 1 = clamped
//   local systems (subdomains D'_i and neighbourhoods omega_l) are node
//   boxes [x0, x0+nxb) x [y0, y0+nyb); their block rows are node rows, so
//   each system is block tridiagonal with nyb blocks of bs = ndof*nxb.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msp {

constexpr int MAXBS = 72;      // largest block row (DOFs) of a local system
constexpr int MAXM = 32;       // largest eigen subspace block

// Record of one node row of a first-level (elasticity) system with bs DOFs
// per row (bs even): the symmetric inverse Schur block in 16-byte column
// groups, then the couplings F (bs x 6).
//  * FP32 copies hold every column, zero-padded to a multiple of 4, in
//    quads: element (i, j) at (j/4)*4*bs + 4*i + j%4; F at l1_cols(bs)*bs.
//  * FP64 copies hold the lower part of each column pair p (columns 2p,
//    2p+1, rows 2p..bs-1): element (i, j) with i >= 2(j/2) at
//    l1_pair_off(bs, j/2) + 2*(i - 2*(j/2)) + j%2; the rest is read
//    transposed.  F at l1_s64(bs).
// Both use the record stride l1_rec(bs); an FP64 record's used part is
// l1_s64(bs) + 6 bs.
__host__ __device__ inline int l1_cols(int bs) { return (bs + 3) & ~3; }
__host__ __device__ inline int l1_pair_off(int bs, int p) { return 2 * p * (bs - p + 1); }
__host__ __device__ inline int l1_s64(int bs) { return l1_pair_off(bs, bs / 2); }

// Record of one node row of a heat pencil factor (bs nodes per row): the
// inverse Schur block column-major (bs^2), the couplings F of the row with
// the row before (bs x 3) and G with the row after (bs x 3), padded to an
// even length so that every record starts on 16 bytes.
__host__ __device__ inline int heat_rec(int bs) { return (bs * bs + 6 * bs + 1) & ~1; }
__host__ __device__ inline long long l1_rec(int bs) {
  return (long long)l1_cols(bs) * bs + 6LL * bs;
}
constexpr int RED_THREADS = 256;

// One block-tridiagonal local system.
struct SysDesc {
  int x0, y0;          // first node of the box
  int nxb, nyb;        // nodes per row, rows
  int ex0, ex1;        // elements that contribute: [ex0, ex1) x [ey0, ey1)
  int ey0, ey1;
  long long foff;      // offset (entries) of the inverse Schur blocks
  long long voff;      // offset (entries) of the local vector
};

// Coarse node record (2D): neighbourhood box and column layout.
struct CoarseNode {
  int cx, cy;          // coarse grid index
  int x0, y0;          // omega node box origin (closed box)
  int nxw, nyw;        // omega node box size
  int nmodes;          // selected heat modes
  int nrot;            // rotation columns (0 or 1)
  int col0;            // first coarse column (mode j of component c at
                       // col0 + c*nmodes + j; rotation at col0 + 2*nmodes)
  int sys;             // index of this omega in the eigen system table
  long long psi_off;   // offset of psi_j (nmodes x nxw*nyw doubles)
  long long w_off;     // offset of K Phi columns (ncols x 2*nxw*nyw)
};

// Per-matrix strides (doubles) of a batched Gauss-Jordan elimination: the
// matrices, their pivot-block factors and their panels.
struct GjStride {
  long long a, ld, p;
};

// First-level subdomain of a 3D mesh: node box [x0, x0+nbx) x [y0, y0+nby)
// x [z0, z0+nbz), n = 3 nbx nby nbz local DOFs (DOF 3 local_node + c,
// local nodes x fastest), its dense inverse at moff (entries; leading
// dimension ld, shared by all) and its local solution at voff.
struct Sub3 {
  int x0, y0, z0;
  int nbx, nby, nbz;
  int n, pad;
  long long moff, voff;
};

// Coarse node of a 3D mesh and its neighbourhood omega_l: closed node box
// [x0, x0+nbx) x [y0, y0+nby) x [z0, z0+nbz).  The heat pencil's factor is
// block tridiagonal by node planes of constant z (np = nbx nby nodes, padded
// to the shared order ldp): plane k's inverse Schur block at goff + k ldp^2
// (row-major, symmetric), the subspace block at xoff (row k ldp + a of the
// in-plane node a, m values a row).  After the setup: nmodes selected heat
// modes psi_j at psi_off (box node b = k np + a, value b nmodes + j), the
// node's columns from col0 (mode j of component c at col0 + c nmodes + j,
// rotation k at col0 + 3 nmodes + k; in K_0, whose columns are grouped by
// slabs of coarse nodes, from kcol0) and their K Phi at woff (3 values per
// box node a column).
struct Nbh3 {
  int cx, cy, cz;
  int x0, y0, z0;
  int nbx, nby, nbz;
  int np;
  int nmodes, nrot, col0, kcol0;
  long long goff, xoff, psi_off, woff;
};

// Coarse part of the 3D preconditioner as the node-centric kernels see it.
struct Coarse3 {
  const Nbh3* nb;            // coarse nodes, x fastest
  int ncx, ncy, ncz;
  int S0, S1, S2;            // coarse block edge (elements)
  double invH;               // 1 / H (rotation scale)
  const double* psi;
  const double* c0;          // K_0^+ R_0 r in K_0's column order (null: no coarse part)
};

// Device scalars of one PCG run.
struct CGScalars {
  double rz, rz_old, pq, alpha, beta, rr, ff, zq, fx, rr0;
  double tol2;
  int iter, done, status, maxit;
  int flexible, pad0, pad1, pad2;
};

enum : int { DONE_RUNNING = 0, DONE_CONVERGED = 1, DONE_MAXIT = 2,
             DONE_BREAKDOWN = 3 };

// Error bits raised by kernels.
enum : int { ERR_NOT_SPD = 1, ERR_NONFINITE = 2, ERR_RANGE = 4,
             ERR_EIG = 8 };

// Arguments of the kernel that forms z = M^{-1} r at every node.
struct CombineArgs {
  const SysDesc* sys_grid;   // grid cell -> its subdomain (nxb = 0: none)
  int ngx, ngy;              // extent of that grid
  int sub_vertex;            // 1: grid = coarse nodes, 0: blocks
  const void* lsol;          // local solutions (double or float)
  int lsol_fp32;
  const CoarseNode* cnodes;
  const double* psi;
  const float* psi32;        // FP32 copy of psi (FP32-local path) or null
  const double* c0;
  double invH;
  int use_l1, use_coarse;
};

struct Geom {
  int nx, ny;          // elements
  int nnx, nny;        // nodes
  int sx, sy;          // coarse block edge S (elements)
  int ncx, ncy;        // coarse nodes per axis
  double h;
  int nz, nnz;         // 3D: elements and nodes along z (2D: 1, 1)
};

// Arguments of one problem's PCG-iteration kernels.  A single solve passes
// them by value; a batched launch passes a device table with one entry per
// problem and a prefix table of workgroup offsets (start[e] .. start[e+1]
// are problem e's workgroups).
struct MatvecArgs {
  Geom g;
  double ke[64];              // unit-modulus element matrix, read by every
                             // lane from the arguments (scalar loads)
  const double* E;
  const uint8_t* mask;
  const double* xin;         // APPLY: x, CG: z, RESID: x
  const double* pin;         // CG: p_old
  double* pout;              // CG: p_new
  double* yout;              // APPLY: y, CG: q, RESID: r
  const double* f;           // RESID: f
  CGScalars* sc;
  double* part;
  const double* part_comb;
  int nb_comb;
  int ty;                    // node rows per tile (4, 8 or 16)
  double* beta_hist;
};

struct UpdateArgs {
  long long n2;              // nodes (DOF pairs)
  double* x;
  double* r;
  const double* p;
  const double* q;
  CGScalars* sc;
  double* alpha_hist;
  double* part;
  const double* part_mv;
  int nb_mv;
  const double* part_comb;
  int nb_comb;
};

struct Level1Args {
  Geom g;
  const SysDesc* sys;
  const uint8_t* mask;
  const double* S64;
  const float* S32;
  const uint8_t* use64;
  const double* r;
  double* lsol;
  double* gmid;        // per system 2 x MAXBS: each chain's coupling into the middle row
  CGScalars* sc;
  const double* part_upd;
  int nb_upd;
  int check;
};

struct RestrictArgs {
  Geom g;
  const CoarseNode* cn;
  const uint8_t* mask;
  const double* psi;
  const float* psi32;        // FP32 copy of psi (FP32-local path) or null
  const double* r;
  double* cpart;
  int ldc;
  double invH;
  CGScalars* sc;
  const double* part_upd;
  int nb_upd;
  int check;
};

struct GemvArgs {
  const double* K0;
  int ldk, nc;
  const double* cpart;
  int ldc;
  double* c0;
  const CGScalars* sc;
};

struct CombineCall {
  Geom g;
  CombineArgs ca;
  const uint8_t* mask;
  const double* r;
  const double* q;
  double* z;
  CGScalars* sc;
  double* part;
  int flex;                  // flexible CG: also the partials of z.q
  const double* zadd;        // added to z at free DOFs when set (M_EE's coarse part)
};

// Problem of workgroup b in a batched launch: the last e with start[e] <= b
// (start has nent + 1 entries, start[0] = 0).  Uniform per workgroup.
__device__ __forceinline__ int batch_entry(const int* __restrict__ start,
                                           int nent, int b) {
  int lo = 0, hi = nent - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace msp
