// The 3D (H8) state solve with the first level of the two-level Schwarz
// preconditioner (Section 2: z = sum_i R_i^T K_i^{-1} R_i r over the
// overlapping subdomains, K_i the principal submatrix of K(rho) on the free
// DOFs of D'_i; Section 1.1 for the trilinear brick element).
//
// A 3D subdomain of S = 6 elements and one overlap layer holds up to 7^3
// nodes, 1,029 DOFs, in 7 node planes of 147 DOFs: too wide for the
// 72-DOF block rows of the 2D records.  K_i is factored block-
// tridiagonally by those planes: each plane's Schur complement is assembled
// from E and inverted by the blocked Gauss-Jordan elimination of the coarse
// solve, batched over all subdomains (its update runs on the FP64 matrix
// cores).  The inverse blocks are kept in FP64, and rounded to FP32 for
// the mixed path; the application is a forward and a backward sweep over
// a subdomain's planes in one workgroup.  The local solutions are summed
// per node in a fixed subdomain order (no atomics).
//
// The PCG kernels keep their scalars on the device (CGScalars); every
// kernel returns at once when the run is marked done, so a chunk of
// iterations can be enqueued without host round trips.  Sums are
// two-stage: per-workgroup partials, then the last workgroup adds them in
// workgroup order.
#include "common.h"
#include "dev.h"

namespace msp {

constexpr int T3_NT = 256;
constexpr int LD3_MAX = 2048;     // largest local order (the box vector in LDS)
// workgroups of the vector kernels: one per CU (each workgroup takes its
// ticket with one atomic on a shared counter, and those serialise)
constexpr int V3_MAXB = 256;

// s_j = 1 / sqrt(A_jj) (0 for a non-positive or non-finite diagonal, whose
// pivot is then dropped and reported).
__global__ void __launch_bounds__(T3_NT)
k3_scale_factors(const double* __restrict__ A, int ld, long long mstride,
                 double* __restrict__ sdiag) {
  const int j = blockIdx.x * T3_NT + threadIdx.x;
  if (j >= ld) return;
  const double d = A[blockIdx.y * mstride + (long long)j * ld + j];
  sdiag[(long long)blockIdx.y * ld + j] = (d > 0.0 && finite(d)) ? 1.0 / sqrt(d) : 0.0;
}

__global__ void __launch_bounds__(T3_NT)
k3_scale(double* __restrict__ A, int ld, long long mstride,
         const double* __restrict__ sdiag) {
  const long long idx = (long long)blockIdx.x * T3_NT + threadIdx.x;
  if (idx >= (long long)ld * ld) return;
  const int i = (int)(idx / ld), j = (int)(idx - (long long)(idx / ld) * ld);
  const double* sd = sdiag + (long long)blockIdx.y * ld;
  A[blockIdx.y * mstride + idx] *= sd[i] * sd[j];
}

// Undo the scaling of the inverse, symmetrised: B_ij = (A_ij + A_ji)/2 s_i
// s_j, in place (FP64), and rounded into the FP32 pool when given.  One
// workgroup per pair of mirror tiles (US_T x US_T, the upper triangle's
// tiles in row order): both tiles staged in LDS, then written row-wise.
constexpr int US_T = 32;
__global__ void __launch_bounds__(256)
k3_unscale(double* __restrict__ A, int ld, long long mstride,
           const double* __restrict__ sdiag, float* __restrict__ A32) {
  __shared__ double t1[US_T][US_T + 1], t2[US_T][US_T + 1];
  const int nt = ld / US_T;
  int p = blockIdx.x, I = 0;
  while (p >= nt - I) {       // tile pair (I, J), I <= J, row by row
    p -= nt - I;
    ++I;
  }
  const int J = I + p;
  double* M = A + blockIdx.y * mstride;
  float* M32 = A32 != nullptr ? A32 + blockIdx.y * mstride : nullptr;
  const double* sd = sdiag + (long long)blockIdx.y * ld;
  const int tx = threadIdx.x & (US_T - 1), ty = threadIdx.x / US_T;
  for (int r = ty; r < US_T; r += 256 / US_T) {
    t1[r][tx] = M[(long long)(I * US_T + r) * ld + J * US_T + tx];
    t2[r][tx] = M[(long long)(J * US_T + r) * ld + I * US_T + tx];
  }
  __syncthreads();
  // entry (i, j) from the symmetric pair A(lo, hi) + A(hi, lo), scaled by
  // sd_lo then sd_hi (lo = min(i, j)), so both halves get the same bits
  auto put = [&](int i, int j, double a_lohi, double a_hilo) {
    const int lo = min(i, j), hi = max(i, j);
    const double v = 0.5 * (a_lohi + a_hilo) * sd[lo] * sd[hi];
    M[(long long)i * ld + j] = v;
    if (M32 != nullptr) M32[(long long)i * ld + j] = (float)v;
  };
  for (int r = ty; r < US_T; r += 256 / US_T) {
    const int i = I * US_T + r, j = J * US_T + tx;
    if (i <= j) put(i, j, t1[r][tx], t2[tx][r]);     // A(i, j), A(j, i)
    else put(i, j, t2[tx][r], t1[r][tx]);            // diagonal tile, i > j
    if (I != J) {
      // the mirror tile, row J*US_T + r, column I*US_T + tx
      const int mi = J * US_T + r, mj = I * US_T + tx;
      put(mi, mj, t1[tx][r], t2[r][tx]);
    }
  }
}

// z at node (X, Y, Z) += sum over the (at most 8) coarse nodes whose hat is
// nonzero there of their columns times c0.
__device__ __forceinline__ double3 coarse3_prolong(const Geom& g, const Coarse3& cc,
                                                   int X, int Y, int Z) {
  double3 z = make_double3(0.0, 0.0, 0.0);
  for (int cz = Z / cc.S2; cz <= min(Z / cc.S2 + 1, cc.ncz - 1); ++cz) {
    const int dz = Z - cz * cc.S2;
    const double hz = 1.0 - fabs((double)dz) / cc.S2;
    if (!(hz > 0.0)) continue;
    for (int cy = Y / cc.S1; cy <= min(Y / cc.S1 + 1, cc.ncy - 1); ++cy) {
      const int dy = Y - cy * cc.S1;
      const double hy = 1.0 - fabs((double)dy) / cc.S1;
      if (!(hy > 0.0)) continue;
      for (int cx = X / cc.S0; cx <= min(X / cc.S0 + 1, cc.ncx - 1); ++cx) {
        const int dx = X - cx * cc.S0;
        const double hx = 1.0 - fabs((double)dx) / cc.S0;
        if (!(hx > 0.0)) continue;
        const Nbh3& w = cc.nb[((long long)cz * cc.ncy + cy) * cc.ncx + cx];
        const int nm = w.nmodes;
        if (3 * nm + w.nrot == 0) continue;
        const double chi = hx * hy * hz;
        const double* cw = cc.c0 + w.kcol0;
        const long long b = ((long long)(Z - w.z0) * w.nby + (Y - w.y0)) * w.nbx + (X - w.x0);
        const double* ps = cc.psi + w.psi_off + b * nm;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int j = 0; j < nm; ++j) {
          const double p = ps[j];
          s0 = fma(p, cw[j], s0);
          s1 = fma(p, cw[nm + j], s1);
          s2 = fma(p, cw[2 * nm + j], s2);
        }
        if (w.nrot) {
          const double x = dx * g.h * cc.invH, y = dy * g.h * cc.invH, zz = dz * g.h * cc.invH;
          const double a0 = cw[3 * nm], a1 = cw[3 * nm + 1], a2 = cw[3 * nm + 2];
          s0 += zz * a1 - y * a2;
          s1 += -zz * a0 + x * a2;
          s2 += y * a0 - x * a1;
        }
        z.x = fma(chi, s0, z.x);
        z.y = fma(chi, s1, z.y);
        z.z = fma(chi, s2, z.z);
      }
    }
  }
  return z;
}

// ---------------------------------------------------------------------
// First-level summation: z at every node = sum of the local solutions of the subdomains
// whose boxes hold the node, in ascending subdomain order (at most two
// blocks per axis hold a node when the overlap is below the block edge),
// plus the coarse part R_0^T c0 when cc.c0 is set; zero at fixed DOFs.
// use_l1 = 0 leaves the first level out (the coarse part alone).
__global__ void __launch_bounds__(T3_NT)
k3_level1_sum(Geom g, const Sub3* __restrict__ subs, int nbx, int nby, int nbz,
              int S0, int S1, int S2, const uint8_t* __restrict__ mask,
              const double* __restrict__ lsol, double* __restrict__ z,
              const CGScalars* __restrict__ sc, int use_l1, Coarse3 cc) {
  __shared__ int shd;
  if (sc != nullptr && block_read_done(sc, &shd)) return;
  const long long nn = (long long)g.nnx * g.nny * g.nnz;
  const long long node = (long long)blockIdx.x * T3_NT + threadIdx.x;
  if (node >= nn) return;
  const int X = (int)(node % g.nnx);
  const long long rr = node / g.nnx;
  const int Y = (int)(rr % g.nny), Z = (int)(rr / g.nny);
  double z0 = 0.0, z1 = 0.0, z2 = 0.0;
  if (use_l1)
  for (int bz = max(0, Z / S2 - 1); bz <= min(nbz - 1, Z / S2 + 1); ++bz)
    for (int by = max(0, Y / S1 - 1); by <= min(nby - 1, Y / S1 + 1); ++by)
      for (int bx = max(0, X / S0 - 1); bx <= min(nbx - 1, X / S0 + 1); ++bx) {
        const Sub3& s = subs[(bz * nby + by) * nbx + bx];
        const int lx = X - s.x0, ly = Y - s.y0, lz = Z - s.z0;
        if (lx < 0 || lx >= s.nbx || ly < 0 || ly >= s.nby || lz < 0 || lz >= s.nbz) continue;
        const double* l = lsol + s.voff + 3LL * ((lz * s.nby + ly) * s.nbx + lx);
        z0 += l[0];
        z1 += l[1];
        z2 += l[2];
      }
  if (cc.c0 != nullptr) {
    const double3 zc = coarse3_prolong(g, cc, X, Y, Z);
    z0 += zc.x;
    z1 += zc.y;
    z2 += zc.z;
  }
  const uint8_t* m = mask + 3 * node;
  z[3 * node] = m[0] ? 0.0 : z0;
  z[3 * node + 1] = m[1] ? 0.0 : z1;
  z[3 * node + 2] = m[2] ? 0.0 : z2;
}

// ---------------------------------------------------------------------
// First level by node planes.  K_i is block tridiagonal in the planes of
// constant z of its box (np = 3 nbx nby unknowns a plane, DOF 3 a + c of the
// in-plane node a, padded to the shared order ldp); its block LDL^T keeps
// the inverse Schur block G_k of every plane (row-major, symmetric), formed
// plane after plane: S_k = D_k - C_k^T G_{k-1} C_k from E (k3s_schur), then
// inverted by the batched Gauss-Jordan elimination.  The application is a
// forward and a backward sweep over the planes, each step a product with
// G_k and the couplings recomputed from E.  Fixed DOFs are identity rows.

// Coupling of DOF (X, Y, Z, ca) with (X + dx, Y + dy, Z + dz, cb) in K:
// the elements of the mesh holding both nodes (K_i is the principal
// submatrix of K, so elements outside the box count).
__device__ __forceinline__ double k3_coef(const Geom& g, const double* __restrict__ E,
                                          const double* Ke, int X, int Y, int Z,
                                          int dx, int dy, int dz, int ca, int cb) {
  double v = 0.0;
#pragma unroll
  for (int sz = 0; sz < 2; ++sz) {
    const int oz = sz + dz, ez = Z - sz;
    if (oz < 0 || oz > 1 || ez < 0 || ez >= g.nz) continue;
#pragma unroll
    for (int sy = 0; sy < 2; ++sy) {
      const int oy = sy + dy, ey = Y - sy;
      if (oy < 0 || oy > 1 || ey < 0 || ey >= g.ny) continue;
#pragma unroll
      for (int sx = 0; sx < 2; ++sx) {
        const int ox = sx + dx, ex = X - sx;
        if (ox < 0 || ox > 1 || ex < 0 || ex >= g.nx) continue;
        const int va = sx + 2 * sy + 4 * sz, vb = ox + 2 * oy + 4 * oz;
        v += E[((long long)ez * g.ny + ey) * g.nx + ex] * Ke[(3 * va + ca) * 24 + 3 * vb + cb];
      }
    }
  }
  return v;
}

__device__ __forceinline__ bool k3_fixed(const Geom& g, const uint8_t* __restrict__ mask,
                                         int X, int Y, int Z, int c) {
  return mask[3 * (((long long)Z * g.nny + Y) * g.nnx + X) + c] != 0;
}

constexpr int K3S_CB = 16;     // columns of a Schur-complement workgroup
constexpr int K3S_MAXP = 256;  // largest padded plane order
constexpr int K3S_MAXE = 1024; // largest element box (nbx+1)(nby+1)(nbz+1) staged in LDS

// k3_coef with the moduli of the subdomain's element box staged in LDS:
// El[(lz (nby+1) + ly) (nbx+1) + lx] for element (x0-1+lx, y0-1+ly, z0-1+lz)
// (zero outside the mesh), X, Y, Z global node coordinates of the box.
__device__ __forceinline__ double k3_coef_l(const Sub3& sb, const double* El, const double* Ke,
                                            int X, int Y, int Z, int dx, int dy, int dz,
                                            int ca, int cb) {
  const int ex1 = sb.nbx + 1, ey1 = sb.nby + 1;
  double v = 0.0;
#pragma unroll
  for (int sz = 0; sz < 2; ++sz) {
    const int oz = sz + dz;
    if (oz < 0 || oz > 1) continue;
    const int lz = Z - sz - sb.z0 + 1;
#pragma unroll
    for (int sy = 0; sy < 2; ++sy) {
      const int oy = sy + dy;
      if (oy < 0 || oy > 1) continue;
      const int ly = Y - sy - sb.y0 + 1;
#pragma unroll
      for (int sx = 0; sx < 2; ++sx) {
        const int ox = sx + dx;
        if (ox < 0 || ox > 1) continue;
        const int lx = X - sx - sb.x0 + 1;
        const int va = sx + 2 * sy + 4 * sz, vb = ox + 2 * oy + 4 * oz;
        v += El[(lz * ey1 + ly) * ex1 + lx] * Ke[(3 * va + ca) * 24 + 3 * vb + cb];
      }
    }
  }
  return v;
}

// stage the moduli of the box's elements (and the layer around it) in LDS
__device__ __forceinline__ void k3_stage_E(const Geom& g, const Sub3& sb,
                                           const double* __restrict__ E, double* El, int nt) {
  const int ex1 = sb.nbx + 1, ey1 = sb.nby + 1, ez1 = sb.nbz + 1;
  for (int q = threadIdx.x; q < ex1 * ey1 * ez1; q += nt) {
    const int lx = q % ex1, ly = (q / ex1) % ey1, lz = q / (ex1 * ey1);
    const int ex = sb.x0 - 1 + lx, ey = sb.y0 - 1 + ly, ez = sb.z0 - 1 + lz;
    const bool in = ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny && ez >= 0 && ez < g.nz;
    El[q] = in ? E[((long long)ez * g.ny + ey) * g.nx + ex] : 0.0;
  }
}

// Plane k of every subdomain: S_k = D_k - C_k^T G_{k-1} C_k into slot k
// (this workgroup's K3S_CB columns as rows), identity on padding, fixed DOFs
// and the slots of subdomains with fewer planes.  Grid (ldp / K3S_CB,
// subdomains); thread a forms row a.
__global__ void __launch_bounds__(T3_NT)
k3s_schur(Geom g, const Sub3* __restrict__ subs, int k, int ldp,
          const double* __restrict__ Ke_g, const double* __restrict__ E,
          const uint8_t* __restrict__ mask, double* __restrict__ G) {
  __shared__ double Ke[576];
  __shared__ double El[K3S_MAXE];
  __shared__ double T[K3S_MAXP * K3S_CB];
  __shared__ double Cb[K3S_CB * 27];
  __shared__ int Jb[K3S_CB * 27];
  const Sub3 sb = subs[blockIdx.y];
  const int tid = threadIdx.x;
  for (int q = tid; q < 576; q += T3_NT) Ke[q] = Ke_g[q];
  const long long ldp2 = (long long)ldp * ldp;
  double* Sk = G + sb.moff + k * ldp2;
  const int b0 = blockIdx.x * K3S_CB;
  if (k >= sb.nbz) {
    for (int idx = tid; idx < K3S_CB * ldp; idx += T3_NT) {
      const int t = idx / ldp, a = idx - t * ldp;
      Sk[(long long)(b0 + t) * ldp + a] = (a == b0 + t) ? 1.0 : 0.0;
    }
    return;
  }
  k3_stage_E(g, sb, E, El, T3_NT);
  __syncthreads();
  const int np = 3 * sb.nbx * sb.nby;
  const int Z = sb.z0 + k;
  // couplings of column b with the 27 DOFs of its 9 neighbours in plane k-1
  if (k > 0) {
    for (int idx = tid; idx < K3S_CB * 27; idx += T3_NT) {
      const int t = idx / 27, q = idx - 27 * (idx / 27);
      const int b = b0 + t;
      const int nq = q / 3, cj = q - 3 * (q / 3);
      const int dx = nq % 3 - 1, dy = nq / 3 - 1;
      double c = 0.0;
      int j = -1;
      if (b < np) {
        const int bn = b / 3, cb = b - 3 * (b / 3);
        const int bx = bn % sb.nbx, by = bn / sb.nbx;
        const int jx = bx + dx, jy = by + dy;
        if (jx >= 0 && jx < sb.nbx && jy >= 0 && jy < sb.nby) {
          j = 3 * (jy * sb.nbx + jx) + cj;
          const int X = sb.x0 + bx, Y = sb.y0 + by;
          if (!k3_fixed(g, mask, X, Y, Z, cb) && !k3_fixed(g, mask, X + dx, Y + dy, Z - 1, cj))
            c = k3_coef_l(sb, El, Ke, X, Y, Z, dx, dy, -1, cb, cj);
        }
      }
      Cb[idx] = c;
      Jb[idx] = j;
    }
  }
  __syncthreads();
  if (k > 0 && tid < ldp) {
    const double* Gp = Sk - ldp2;
    // every load of a column issued at once (an absent coupling reads row
    // 0 and weighs it by 0, which adds exactly nothing)
    for (int t = 0; t < K3S_CB; ++t) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < 27; ++q) {
        const int j = Jb[t * 27 + q];
        const double c = j >= 0 ? Cb[t * 27 + q] : 0.0;
        acc = fma(Gp[(long long)max(j, 0) * ldp + tid], c, acc);
      }
      T[tid * K3S_CB + t] = acc;
    }
  }
  __syncthreads();
  const int a = tid;
  if (a >= ldp) return;
  const bool arow = a < np;
  const int an = a / 3, ca = a - 3 * (a / 3);
  const int ax = arow ? an % sb.nbx : 0, ay = arow ? an / sb.nbx : 0;
  const bool rem = !arow || k3_fixed(g, mask, sb.x0 + ax, sb.y0 + ay, Z, ca);
  const int X = sb.x0 + ax, Y = sb.y0 + ay;
  // row a's couplings with the 27 DOFs of its neighbours in plane k-1,
  // formed once for all columns.  T is zero at clamped DOFs (their C
  // entries are zero and G_{k-1} is the identity there), so they need no
  // test here.
  double cq[27];
  int iq[27];
#pragma unroll
  for (int q = 0; q < 27; ++q) {
    const int nq = q / 3, ci = q - 3 * (q / 3);
    const int ix = ax + nq % 3 - 1, iy = ay + nq / 3 - 1;
    const bool ok = k > 0 && !rem && ix >= 0 && ix < sb.nbx && iy >= 0 && iy < sb.nby;
    iq[q] = ok ? 3 * (iy * sb.nbx + ix) + ci : 0;
    cq[q] = ok ? k3_coef_l(sb, El, Ke, X, Y, Z, nq % 3 - 1, nq / 3 - 1, -1, ca, ci) : 0.0;
  }
  for (int t = 0; t < K3S_CB; ++t) {
    const int b = b0 + t;
    double v;
    if (rem || b >= np) {
      v = (a == b) ? 1.0 : 0.0;
    } else {
      const int bn = b / 3, cb = b - 3 * (b / 3);
      const int dx = bn % sb.nbx - ax, dy = bn / sb.nbx - ay;
      v = 0.0;
      if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 &&
          !k3_fixed(g, mask, X + dx, Y + dy, Z, cb))
        v = k3_coef_l(sb, El, Ke, X, Y, Z, dx, dy, 0, ca, cb);
      if (k > 0) {
#pragma unroll
        for (int q = 0; q < 27; ++q) v -= cq[q] * T[iq[q] * K3S_CB + t];
      }
    }
    Sk[(long long)b * ldp + a] = v;
  }
}

// Per subdomain and plane: max over the plane's free DOFs of
// (S_k^-1)_ii K_ii, about 1 where the DOF is held by stiff material and up
// to the contrast for stiff islands floating in soft material (whose rigid
// motions FP32 inverse blocks cannot carry, as in 2D).  Grid (planes,
// subdomains).
__global__ void __launch_bounds__(K3S_MAXP)
k3s_metric(Geom g, const Sub3* __restrict__ subs, int ldp, const double* __restrict__ G,
           const double* __restrict__ Ke_g, const double* __restrict__ E,
           const uint8_t* __restrict__ mask, double* __restrict__ metric) {
  __shared__ double Ke[576];
  __shared__ double red[K3S_MAXP / 64];
  const Sub3 sb = subs[blockIdx.y];
  const int k = blockIdx.x, a = threadIdx.x;
  for (int q = a; q < 576; q += K3S_MAXP) Ke[q] = Ke_g[q];
  __syncthreads();
  const int np = 3 * sb.nbx * sb.nby;
  double v = 0.0;
  if (k < sb.nbz && a < np) {
    const int an = a / 3, c = a - 3 * (a / 3);
    const int X = sb.x0 + an % sb.nbx, Y = sb.y0 + an / sb.nbx, Z = sb.z0 + k;
    if (!k3_fixed(g, mask, X, Y, Z, c)) {
      const double gi = G[sb.moff + (long long)k * ldp * ldp + (long long)a * ldp + a];
      v = fabs(gi) * k3_coef(g, E, Ke, X, Y, Z, 0, 0, 0, c, c);
    }
  }
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if ((a & 63) == 0) red[a >> 6] = v;
  __syncthreads();
  if (a == 0) {
    double m = red[0];
    for (int w = 1; w < K3S_MAXP / 64; ++w) m = fmax(m, red[w]);
    metric[(long long)blockIdx.y * gridDim.x + k] = m;
  }
}

// z_i = K_i^{-1} r_i by the plane factors: one workgroup per subdomain,
// the box vector in LDS (r, then y, then x); each plane's product by groups
// of lanes over the inner index (G_k symmetric: row kk read along the
// rows), below.  The blocks are read in FP32 (G32) unless the subdomain is
// flagged in use64 or G32 is null.
constexpr int K3S_NT = 512;
constexpr int K3S_G = 8;       // inner-index groups of the FP32 plane product
constexpr int K3S_LB = 8;     // 16-byte loads of a group in flight together
constexpr int K3S_G64 = 4;     // inner-index groups of the FP64 plane product
static_assert(K3S_MAXP / 2 * K3S_G64 <= K3S_NT, "every row pair needs its K3S_G64 lanes");
static_assert(K3S_MAXP / 4 * K3S_G <= K3S_NT, "every row quad needs its K3S_G lanes");
__global__ void __launch_bounds__(K3S_NT)
k3s_apply(Geom g, const Sub3* __restrict__ subs, int ldp, const double* __restrict__ G64,
          const float* __restrict__ G32, const uint8_t* __restrict__ use64,
          const double* __restrict__ Ke_g, const double* __restrict__ E,
          const uint8_t* __restrict__ mask, const double* __restrict__ r,
          double* __restrict__ lsol, const CGScalars* __restrict__ sc) {
  __shared__ double Ke[576];
  __shared__ double El[K3S_MAXE];
  __shared__ double xl[LD3_MAX];
  __shared__ double rh[K3S_MAXP];
  __shared__ double ph[K3S_MAXP];
  __shared__ uint8_t fl[LD3_MAX];
  __shared__ int shd;
  if (sc != nullptr && block_read_done(sc, &shd)) return;
  const Sub3 sb = subs[blockIdx.x];
  const bool f32 = G32 != nullptr && !(use64 != nullptr && use64[blockIdx.x]);
  const int tid = threadIdx.x;
  for (int q = tid; q < 576; q += K3S_NT) Ke[q] = Ke_g[q];
  k3_stage_E(g, sb, E, El, K3S_NT);
  const int np = 3 * sb.nbx * sb.nby;
  for (int q = tid; q < sb.n; q += K3S_NT) {
    const int a = q / 3, c = q - 3 * (q / 3);
    const int lx = a % sb.nbx, ly = (a / sb.nbx) % sb.nby, lz = a / (sb.nbx * sb.nby);
    const long long node = ((long long)(sb.z0 + lz) * g.nny + sb.y0 + ly) * g.nnx + sb.x0 + lx;
    const uint8_t mq = mask[3 * node + c];
    fl[q] = mq;
    xl[q] = mq ? 0.0 : r[3 * node + c];
  }
  __syncthreads();
  const long long ldp2 = (long long)ldp * ldp;
  const int an = tid / 3, ca = tid - 3 * (tid / 3);
  const int ax = tid < np ? an % sb.nbx : 0, ay = tid < np ? an / sb.nbx : 0;
  // sum over the 27 DOFs of the 9 neighbours in plane k + dz of the coupling
  // times the box vector there
  // The box vector is zero at clamped DOFs from the start and stays zero
  // (their rows and columns of the plane factors are the identity's), so
  // clamped neighbours add exactly nothing and need no test; only the
  // thread's own DOF is checked, from the clamp flags staged in LDS.
  auto couple = [&](int k, int dz) -> double {
    if (fl[k * np + tid]) return 0.0;
    const int X = sb.x0 + ax, Y = sb.y0 + ay, Z = sb.z0 + k;
    const double* xp = xl + (k + dz) * np;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 27; ++q) {
      const int nq = q / 3, cj = q - 3 * (q / 3);
      const int dx = nq % 3 - 1, dy = nq / 3 - 1;
      const int jx = ax + dx, jy = ay + dy;
      if (jx < 0 || jx >= sb.nbx || jy < 0 || jy >= sb.nby) continue;
      s = fma(k3_coef_l(sb, El, Ke, X, Y, Z, dx, dy, dz, ca, cj), xp[3 * (jy * sb.nbx + jx) + cj], s);
    }
    return s;
  };
  // FP32 blocks: thread (q, g) forms rows 4q..4q+3 over group g of the
  // inner index (K3S_G groups of adjacent lanes, summed by a butterfly in a
  // fixed order); the group's 16-byte loads of a plane go out in batches of
  // K3S_LB, all of a batch before any of its values is used, so a plane
  // costs a memory latency or two instead of one per few inner indices.
  const int gq = tid / K3S_G, gg = tid & (K3S_G - 1);
  const int gc = (np + K3S_G - 1) / K3S_G;
  const int gkb = gg * gc, gke = min(np, gkb + gc);
  auto gemv32 = [&](int k) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    const bool rowq = 4 * gq < np;
    const float* Gk = G32 + sb.moff + k * ldp2 + 4 * min(gq, (ldp - 4) / 4);
    for (int b = gkb; rowq && b < gke; b += K3S_LB) {
      float4 v[K3S_LB];
#pragma unroll
      for (int u = 0; u < K3S_LB; ++u) {
        const int kk = min(b + u, gke - 1);
        v[u] = *reinterpret_cast<const float4*>(Gk + (long long)kk * ldp);
      }
#pragma unroll
      for (int u = 0; u < K3S_LB; ++u) {
        const double x = (b + u < gke) ? rh[min(b + u, gke - 1)] : 0.0;
        a0 = fma((double)v[u].x, x, a0);
        a1 = fma((double)v[u].y, x, a1);
        a2 = fma((double)v[u].z, x, a2);
        a3 = fma((double)v[u].w, x, a3);
      }
    }
#pragma unroll
    for (int o = 1; o < K3S_G; o <<= 1) {
      a0 += __shfl_xor(a0, o, 64);
      a1 += __shfl_xor(a1, o, 64);
      a2 += __shfl_xor(a2, o, 64);
      a3 += __shfl_xor(a3, o, 64);
    }
    if (gg == 0 && rowq) {
      ph[4 * gq] = a0;
      if (4 * gq + 1 < np) ph[4 * gq + 1] = a1;
      if (4 * gq + 2 < np) ph[4 * gq + 2] = a2;
      if (4 * gq + 3 < np) ph[4 * gq + 3] = a3;
    }
  };
  // FP64 blocks alike: thread (pair, g) forms rows 2 pair, 2 pair + 1 over
  // group g of K3S_G64 groups, 16-byte loads in batches of K3S_LB
  const int hq = tid / K3S_G64, hg = tid & (K3S_G64 - 1);
  const int hc = (np + K3S_G64 - 1) / K3S_G64;
  const int hkb = hg * hc, hke = min(np, hkb + hc);
  auto gemv64 = [&](int k) {
    double a0 = 0.0, a1 = 0.0;
    const bool rowp = 2 * hq < np;
    const double* Gk = G64 + sb.moff + k * ldp2 + 2 * min(hq, (ldp - 2) / 2);
    for (int b = hkb; rowp && b < hke; b += K3S_LB) {
      double2 v[K3S_LB];
#pragma unroll
      for (int u = 0; u < K3S_LB; ++u) {
        const int kk = min(b + u, hke - 1);
        v[u] = *reinterpret_cast<const double2*>(Gk + (long long)kk * ldp);
      }
#pragma unroll
      for (int u = 0; u < K3S_LB; ++u) {
        const double x = (b + u < hke) ? rh[min(b + u, hke - 1)] : 0.0;
        a0 = fma(v[u].x, x, a0);
        a1 = fma(v[u].y, x, a1);
      }
    }
#pragma unroll
    for (int o = 1; o < K3S_G64; o <<= 1) {
      a0 += __shfl_xor(a0, o, 64);
      a1 += __shfl_xor(a1, o, 64);
    }
    if (hg == 0 && rowp) {
      ph[2 * hq] = a0;
      if (2 * hq + 1 < np) ph[2 * hq + 1] = a1;
    }
  };
  for (int k = 0; k < sb.nbz; ++k) {
    if (tid < np) rh[tid] = xl[k * np + tid] - (k > 0 ? couple(k, -1) : 0.0);
    __syncthreads();
    if (f32) gemv32(k);
    else gemv64(k);
    __syncthreads();
    if (tid < np) xl[k * np + tid] = ph[tid];
    __syncthreads();
  }
  for (int k = sb.nbz - 2; k >= 0; --k) {
    if (tid < np) rh[tid] = couple(k, 1);
    __syncthreads();
    if (f32) gemv32(k);
    else gemv64(k);
    __syncthreads();
    if (tid < np) xl[k * np + tid] -= ph[tid];
    __syncthreads();
  }
  for (int q = tid; q < sb.n; q += K3S_NT) lsol[sb.voff + q] = xl[q];
}

// ---------------------------------------------------------------------
// PCG vector kernels.  Grid-stride loops over V3 workgroups; NV sums per
// kernel, finished by the last workgroup.

// Sums of this workgroup's values to part[b * NV + k]; in the last
// workgroup every thread gets the grid totals in out[] and true is
// returned (thread 0 then owns the scalars; it resets the ticket).
template <int NV>
__device__ bool grid_sums(const double (&v)[NV], double* part, unsigned int* ticket,
                          double (&out)[NV]) {
  __shared__ double red[T3_NT / 64 + 1];
  __shared__ unsigned int tk;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double t = block_sum<T3_NT>(v[k], red);
    if (threadIdx.x == 0) part[(long long)blockIdx.x * NV + k] = t;
  }
  if (!last_block(ticket, gridDim.x, &tk)) return false;
#pragma unroll
  for (int k = 0; k < NV; ++k) out[k] = reduce_partials<T3_NT>(part + k, gridDim.x, NV, red);
  if (threadIdx.x == 0) *ticket = 0u;
  return true;
}

// r = f - y (y = K x), zero at fixed DOFs; sums r.r, f.f, f.x.  mode 0:
// start of a segment (rr, ff); mode 1: true residual at the end (rr0, fx).
__global__ void __launch_bounds__(T3_NT)
k3_cg_resid(long long n, const double* __restrict__ f, const double* __restrict__ y,
            const double* __restrict__ x, const uint8_t* __restrict__ mask,
            double* __restrict__ r, CGScalars* __restrict__ sc,
            double* __restrict__ part, unsigned int* __restrict__ ticket, int mode) {
  double v[3] = {0.0, 0.0, 0.0};
  for (long long i = (long long)blockIdx.x * T3_NT + threadIdx.x; i < n;
       i += (long long)gridDim.x * T3_NT) {
    const bool fx = mask[i] != 0;
    const double fi = fx ? 0.0 : f[i];
    const double ri = fx ? 0.0 : fi - y[i];
    r[i] = ri;
    v[0] += ri * ri;
    v[1] += fi * fi;
    v[2] += fi * x[i];
  }
  double o[3];
  if (!grid_sums<3>(v, part, ticket, o)) return;
  if (threadIdx.x == 0) {
    if (mode == 0) {
      sc->rr = o[0];
      sc->ff = o[1];
    } else {
      sc->rr0 = o[0];
      sc->fx = o[2];
    }
  }
}

// p.q; alpha = r.z / p.q (breakdown if p.q <= 0 or not finite).
__global__ void __launch_bounds__(T3_NT)
k3_cg_pq(long long n, const double* __restrict__ p, const double* __restrict__ q,
         CGScalars* __restrict__ sc, double* __restrict__ part,
         unsigned int* __restrict__ ticket, double* __restrict__ ahist) {
  __shared__ int shd;
  if (block_read_done(sc, &shd)) return;
  double v[1] = {0.0};
  for (long long i = (long long)blockIdx.x * T3_NT + threadIdx.x; i < n;
       i += (long long)gridDim.x * T3_NT)
    v[0] += p[i] * q[i];
  double o[1];
  if (!grid_sums<1>(v, part, ticket, o)) return;
  if (threadIdx.x == 0) {
    const double pq = o[0];
    sc->pq = pq;
    if (!(pq > 0.0) || !finite(pq)) {
      sc->status = -5;
      __hip_atomic_store(&sc->done, DONE_BREAKDOWN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const double al = sc->rz / pq;
      sc->alpha = al;
      ahist[sc->iter] = al;
    }
  }
}

// x += alpha p, r -= alpha q; r.r; the iteration count and the stop test
// (recursive residual against tol * ||f||, iteration limit, non-finite).
__global__ void __launch_bounds__(T3_NT)
k3_cg_update(long long n, double* __restrict__ x, double* __restrict__ r,
             const double* __restrict__ p, const double* __restrict__ q,
             CGScalars* __restrict__ sc, double* __restrict__ part,
             unsigned int* __restrict__ ticket) {
  __shared__ int shd;
  if (block_read_done(sc, &shd)) return;
  const double al = sc->alpha;
  double v[1] = {0.0};
  for (long long i = (long long)blockIdx.x * T3_NT + threadIdx.x; i < n;
       i += (long long)gridDim.x * T3_NT) {
    x[i] = fma(al, p[i], x[i]);
    const double ri = fma(-al, q[i], r[i]);
    r[i] = ri;
    v[0] += ri * ri;
  }
  double o[1];
  if (!grid_sums<1>(v, part, ticket, o)) return;
  if (threadIdx.x == 0) {
    const double rr = o[0];
    const int it1 = sc->iter + 1;
    sc->iter = it1;
    sc->rr = rr;
    int d = DONE_RUNNING;
    if (!finite(rr)) {
      d = DONE_BREAKDOWN;
      sc->status = -5;
    } else if (rr <= sc->tol2 * sc->ff) {
      d = DONE_CONVERGED;
    } else if (it1 >= sc->maxit) {
      d = DONE_MAXIT;
    }
    if (d != DONE_RUNNING)
      __hip_atomic_store(&sc->done, d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// r.z (and z.q for the flexible variant); init: the segment's first r.z,
// beta = 0; else beta (Fletcher-Reeves (r.z)_new / (r.z)_old, or flexible
// Polak-Ribiere -alpha (z.q) / (r.z)_old), recorded for the Lanczos
// estimate.
__global__ void __launch_bounds__(T3_NT)
k3_cg_rz(long long n, const double* __restrict__ r, const double* __restrict__ z,
         const double* __restrict__ q, CGScalars* __restrict__ sc,
         double* __restrict__ part, unsigned int* __restrict__ ticket,
         double* __restrict__ bhist, int init) {
  __shared__ int shd;
  if (block_read_done(sc, &shd)) return;
  const bool flex = !init && sc->flexible;
  double v[2] = {0.0, 0.0};
  for (long long i = (long long)blockIdx.x * T3_NT + threadIdx.x; i < n;
       i += (long long)gridDim.x * T3_NT) {
    v[0] += r[i] * z[i];
    if (flex) v[1] += z[i] * q[i];
  }
  double o[2];
  if (!grid_sums<2>(v, part, ticket, o)) return;
  if (threadIdx.x == 0) {
    const double rzn = o[0];
    if (init) {
      sc->rz = rzn;
      sc->beta = 0.0;
    } else {
      const double be = flex ? -sc->alpha * o[1] / sc->rz : rzn / sc->rz;
      sc->zq = o[1];
      sc->rz_old = sc->rz;
      sc->rz = rzn;
      sc->beta = be;
      bhist[sc->iter - 1] = be;
      if (!finite(be)) {
        sc->status = -5;
        __hip_atomic_store(&sc->done, DONE_BREAKDOWN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// p = z + beta p.
__global__ void __launch_bounds__(T3_NT)
k3_cg_p(long long n, const double* __restrict__ z, double* __restrict__ p,
        const CGScalars* __restrict__ sc) {
  __shared__ int shd;
  if (block_read_done(sc, &shd)) return;
  const double be = sc->beta;
  for (long long i = (long long)blockIdx.x * T3_NT + threadIdx.x; i < n;
       i += (long long)gridDim.x * T3_NT)
    p[i] = fma(be, p[i], z[i]);
}

// ---------------------------------------------------------------- launchers

int level1_3d_max_order() { return LD3_MAX; }

int vec3_blocks(long long n) {
  const long long b = (n + T3_NT - 1) / T3_NT;
  return (int)(b < 1 ? 1 : (b > V3_MAXB ? V3_MAXB : b));
}

void launch_gj_steps(double*, int, int, GjStride, double*, double*, double*,
                     double, int*, hipStream_t);

// In place: A_i <- A_i^{-1} for the nsub matrices at stride ms (scaled to
// unit diagonal, batched Gauss-Jordan, unscaled and symmetrised; FP32 copy
// into A32 when given).  LD, Lp and Rp hold 4160, 64 ld and 64 ld doubles
// per matrix.
void launch_local_inverse3_strided(double* A, int ld, int nsub, long long ms,
                                   double* sdiag, double* LD, double* Lp, double* Rp,
                                   int* dropped, float* A32, hipStream_t s) {
  const unsigned nbe = (unsigned)(((long long)ld * ld + T3_NT - 1) / T3_NT);
  hipLaunchKernelGGL(k3_scale_factors, dim3((ld + T3_NT - 1) / T3_NT, nsub),
                     dim3(T3_NT), 0, s, A, ld, ms, sdiag);
  hipLaunchKernelGGL(k3_scale, dim3(nbe, nsub), dim3(T3_NT), 0, s, A, ld, ms, sdiag);
  // only a pivot that is not positive is dropped (K_i is SPD); a drop is
  // reported as a failed setup
  launch_gj_steps(A, ld, nsub, GjStride{ms, 64LL * 65, 64LL * ld}, LD, Lp, Rp,
                  0.0, dropped, s);
  const int nt = ld / US_T;
  hipLaunchKernelGGL(k3_unscale, dim3(nt * (nt + 1) / 2, nsub), dim3(256), 0, s, A, ld, ms,
                     sdiag, A32);
}

// Plane factors of every K_i: Schur complement and its inverse, plane by
// plane (FP32 copies into G32 when given, same layout).  G, G32: pmax
// slots of ldp^2 per subdomain (Sub3.moff).
void launch_level1_planes(const Geom& g, const Sub3* subs, int nsub, int pmax, int ldp,
                          const double* Ke, const double* E, const uint8_t* mask,
                          double* G, float* G32, double* sdiag, double* LD, double* Lp,
                          double* Rp, int* dropped, hipStream_t s) {
  const long long ldp2 = (long long)ldp * ldp;
  for (int k = 0; k < pmax; ++k) {
    hipLaunchKernelGGL(k3s_schur, dim3(ldp / K3S_CB, nsub), dim3(T3_NT), 0, s, g, subs, k,
                       ldp, Ke, E, mask, G);
    launch_local_inverse3_strided(G + k * ldp2, ldp, nsub, pmax * ldp2, sdiag, LD, Lp, Rp,
                                  dropped, G32 ? G32 + k * ldp2 : nullptr, s);
  }
}

int level1_planes_max() { return K3S_MAXP; }

void launch_level1_metric(const Geom& g, const Sub3* subs, int nsub, int pmax, int ldp,
                          const double* G, const double* Ke, const double* E,
                          const uint8_t* mask, double* metric, hipStream_t s) {
  hipLaunchKernelGGL(k3s_metric, dim3(pmax, nsub), dim3(K3S_MAXP), 0, s, g, subs, ldp, G,
                     Ke, E, mask, metric);
}

void launch_level1_3d(const Geom& g, const Sub3* subs, int nsub, int ld,
                      int nbx, int nby, int nbz, int S0, int S1, int S2,
                      const double* A64, const float* A32, const uint8_t* use64,
                      const double* Ke, const double* E, const uint8_t* mask,
                      const double* r, double* lsol, double* z,
                      const CGScalars* sc, int use_l1, const Coarse3& cc,
                      hipStream_t s) {
  if (use_l1)
    hipLaunchKernelGGL(k3s_apply, dim3(nsub), dim3(K3S_NT), 0, s, g, subs, ld, A64, A32,
                       use64, Ke, E, mask, r, lsol, sc);
  const long long nn = (long long)g.nnx * g.nny * g.nnz;
  hipLaunchKernelGGL(k3_level1_sum, dim3((unsigned)((nn + T3_NT - 1) / T3_NT)),
                     dim3(T3_NT), 0, s, g, subs, nbx, nby, nbz, S0, S1, S2, mask,
                     lsol, z, sc, use_l1, cc);
}

void launch_cg3_resid(long long n, const double* f, const double* y, const double* x,
                      const uint8_t* mask, double* r, CGScalars* sc, double* part,
                      unsigned int* ticket, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k3_cg_resid, dim3(vec3_blocks(n)), dim3(T3_NT), 0, s, n, f,
                     y, x, mask, r, sc, part, ticket, mode);
}

void launch_cg3_pq(long long n, const double* p, const double* q, CGScalars* sc,
                   double* part, unsigned int* ticket, double* ahist, hipStream_t s) {
  hipLaunchKernelGGL(k3_cg_pq, dim3(vec3_blocks(n)), dim3(T3_NT), 0, s, n, p, q,
                     sc, part, ticket, ahist);
}

void launch_cg3_update(long long n, double* x, double* r, const double* p,
                       const double* q, CGScalars* sc, double* part,
                       unsigned int* ticket, hipStream_t s) {
  hipLaunchKernelGGL(k3_cg_update, dim3(vec3_blocks(n)), dim3(T3_NT), 0, s, n, x,
                     r, p, q, sc, part, ticket);
}

void launch_cg3_rz(long long n, const double* r, const double* z, const double* q,
                   CGScalars* sc, double* part, unsigned int* ticket,
                   double* bhist, int init, hipStream_t s) {
  hipLaunchKernelGGL(k3_cg_rz, dim3(vec3_blocks(n)), dim3(T3_NT), 0, s, n, r, z,
                     q, sc, part, ticket, bhist, init);
}

void launch_cg3_p(long long n, const double* z, double* p, const CGScalars* sc,
                  hipStream_t s) {
  hipLaunchKernelGGL(k3_cg_p, dim3(vec3_blocks(n)), dim3(T3_NT), 0, s, n, z, p, sc);
}

}  // namespace msp
