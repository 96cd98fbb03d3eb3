// The 3D (H8) state solve with the first level of the two-level Schwarz
// preconditioner (Section 2: z = sum_i R_i^T K_i^{-1} R_i r over the
// overlapping subdomains, K_i the principal submatrix of K(rho) on the free
// DOFs of D'_i; Section 1.1 for the trilinear brick element).
//
// A 3D subdomain of S = 6 elements and one overlap layer holds up to 7^3
// nodes, 1,029 DOFs, and its node planes couple 147 DOFs each: too wide for
// the block-tridiagonal records of the 2D path.  Each K_i is instead
// gathered as a dense matrix, scaled to unit diagonal and inverted in place
// by the blocked Gauss-Jordan elimination of the coarse solve, batched over
// all subdomains (its update runs on the FP64 matrix cores).  The inverse
// is kept in FP64, or rounded to FP32 for the mixed path, and applied as
// one matrix-vector product per subdomain: the application streams every
// inverse once, so it is bound by HBM bandwidth.  The local solutions are
// summed per node in a fixed subdomain order (no atomics).
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
constexpr int LD3_MAX = 2048;     // largest local order (LDS of the apply)
// workgroups of the vector kernels: one per CU (each workgroup takes its
// ticket with one atomic on a shared counter, and those serialise)
constexpr int V3_MAXB = 256;

// ---------------------------------------------------------------------
// Dense local matrices.  Thread per local row DOF q = 3 a + c (node a of
// the box): for each of the 27 neighbours b of a inside the box and each
// component d, entry (q, 3 b + d) = sum over the elements holding both
// nodes of E_e K^_e(3 va + c, 3 vb + d) (va, vb the nodes' vertices in e).
// Rows and columns of fixed DOFs are those of the identity, as are the
// padding rows n .. ld-1 (so the inverse restricted to the free DOFs is
// K_i^{-1}).  The pool must be zero on entry.
__global__ void __launch_bounds__(T3_NT)
k3_assemble(Geom g, const Sub3* __restrict__ subs, int ld,
            const double* __restrict__ Ke, const double* __restrict__ E,
            const uint8_t* __restrict__ mask, double* __restrict__ A) {
  __shared__ double K[576];
  for (int q = threadIdx.x; q < 576; q += T3_NT) K[q] = Ke[q];
  __syncthreads();
  const Sub3 s = subs[blockIdx.y];
  const int q = blockIdx.x * T3_NT + threadIdx.x;
  if (q >= ld) return;
  double* row = A + s.moff + (long long)q * ld;
  if (q >= s.n) {
    row[q] = 1.0;
    return;
  }
  const int a = q / 3, c = q - 3 * (q / 3);
  const int lx = a % s.nbx, ly = (a / s.nbx) % s.nby, lz = a / (s.nbx * s.nby);
  const int ax = s.x0 + lx, ay = s.y0 + ly, az = s.z0 + lz;
  const long long anode = ((long long)az * g.nny + ay) * g.nnx + ax;
  if (mask[3 * anode + c]) {
    row[q] = 1.0;
    return;
  }
  // moduli of the eight elements around a: element (ax - sx, ay - sy, az - sz)
  double Ee[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int ex = ax - (v & 1), ey = ay - ((v >> 1) & 1), ez = az - (v >> 2);
    const bool in = ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny && ez >= 0 && ez < g.nz;
    Ee[v] = in ? E[((long long)ez * g.ny + ey) * g.nx + ex] : 0.0;
  }
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int bx = lx + dx, by = ly + dy, bz = lz + dz;
        if (bx < 0 || bx >= s.nbx || by < 0 || by >= s.nby || bz < 0 || bz >= s.nbz) continue;
        const int b = (bz * s.nby + by) * s.nbx + bx;
        const long long bnode = anode + ((long long)dz * g.nny + dy) * g.nnx + dx;
        double v0 = 0.0, v1 = 0.0, v2 = 0.0;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          const int sx = v & 1, sy = (v >> 1) & 1, sz = v >> 2;
          const int ox = sx + dx, oy = sy + dy, oz = sz + dz;   // b's vertex offsets in e
          if (ox < 0 || ox > 1 || oy < 0 || oy > 1 || oz < 0 || oz > 1) continue;
          const int vb = ox + 2 * oy + 4 * oz;
          const double* kr = K + (3 * v + c) * 24 + 3 * vb;
          v0 += Ee[v] * kr[0];
          v1 += Ee[v] * kr[1];
          v2 += Ee[v] * kr[2];
        }
        const uint8_t* mb = mask + 3 * bnode;
        row[3 * b] = mb[0] ? 0.0 : v0;
        row[3 * b + 1] = mb[1] ? 0.0 : v1;
        row[3 * b + 2] = mb[2] ? 0.0 : v2;
      }
}

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
// s_j, in place (FP64) or into the FP32 pool.
__global__ void __launch_bounds__(T3_NT)
k3_unscale(double* __restrict__ A, int ld, long long mstride,
           const double* __restrict__ sdiag, float* __restrict__ A32) {
  const long long idx = (long long)blockIdx.x * T3_NT + threadIdx.x;
  if (idx >= (long long)ld * ld) return;
  const int i = (int)(idx / ld), j = (int)(idx - (long long)(idx / ld) * ld);
  double* M = A + blockIdx.y * mstride;
  const double* sd = sdiag + (long long)blockIdx.y * ld;
  const double v = 0.5 * (M[(long long)i * ld + j] + M[(long long)j * ld + i]) * sd[i] * sd[j];
  if (A32 != nullptr) {
    A32[blockIdx.y * mstride + idx] = (float)v;
  } else if (j >= i) {
    M[(long long)i * ld + j] = v;
    M[(long long)j * ld + i] = v;
  }
}

// ---------------------------------------------------------------------
// First-level application, part 1: lsol_i = K_i^{-1} r_i.  Workgroup =
// (64-row block, subdomain); r_i is gathered into LDS (zero at fixed DOFs
// and past n), then each wave takes 16 rows, four at a time, the lanes
// striding along the rows with 16-byte loads (FP64 sums).
template <typename T> struct Vec3T;
template <> struct Vec3T<float> { typedef float4 type; static constexpr int n = 4; };
template <> struct Vec3T<double> { typedef double2 type; static constexpr int n = 2; };

__device__ __forceinline__ double vdot(const float4& a, const double* x) {
  return (double)a.x * x[0] + (double)a.y * x[1] + (double)a.z * x[2] + (double)a.w * x[3];
}
__device__ __forceinline__ double vdot(const double2& a, const double* x) {
  return a.x * x[0] + a.y * x[1];
}

template <typename T>
__global__ void __launch_bounds__(T3_NT)
k3_level1(Geom g, const Sub3* __restrict__ subs, int ld, const T* __restrict__ A,
          const uint8_t* __restrict__ mask, const double* __restrict__ r,
          double* __restrict__ lsol, const CGScalars* __restrict__ sc) {
  typedef typename Vec3T<T>::type V;
  constexpr int NV = Vec3T<T>::n;
  __shared__ double rl[LD3_MAX];
  __shared__ int shd;
  if (sc != nullptr && block_read_done(sc, &shd)) return;
  const Sub3 s = subs[blockIdx.y];
  const int row0 = blockIdx.x * 64;
  if (row0 >= s.n) return;
  const int ncol = (s.n + NV - 1) / NV * NV;
  for (int q = threadIdx.x; q < ncol; q += T3_NT) {
    double v = 0.0;
    if (q < s.n) {
      const int a = q / 3, c = q - 3 * (q / 3);
      const int lx = a % s.nbx, ly = (a / s.nbx) % s.nby, lz = a / (s.nbx * s.nby);
      const long long node = ((long long)(s.z0 + lz) * g.nny + s.y0 + ly) * g.nnx + s.x0 + lx;
      v = mask[3 * node + c] ? 0.0 : r[3 * node + c];
    }
    rl[q] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nvec = ncol / NV;
  const T* M = A + s.moff;
#pragma unroll 1
  for (int g4 = 0; g4 < 4; ++g4) {
    const int i0 = row0 + 16 * w + 4 * g4;
    if (i0 >= s.n) break;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const V* rows[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      rows[k] = reinterpret_cast<const V*>(M + (long long)min(i0 + k, s.n - 1) * ld);
    for (int cv = lane; cv < nvec; cv += 64) {
      V v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = rows[k][cv];
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] += vdot(v[k], rl + NV * cv);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = wave_sum(acc[k]);
    if (lane < 4 && i0 + lane < s.n) {
      const double o = lane == 0 ? acc[0] : lane == 1 ? acc[1] : lane == 2 ? acc[2] : acc[3];
      lsol[s.voff + i0 + lane] = o;
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

// Part 2: z at every node = sum of the local solutions of the subdomains
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

void launch_assemble3(const Geom& g, const Sub3* subs, int nsub, int ld,
                      const double* Ke, const double* E, const uint8_t* mask,
                      double* A, hipStream_t s) {
  hipLaunchKernelGGL(k3_assemble, dim3((ld + T3_NT - 1) / T3_NT, nsub), dim3(T3_NT),
                     0, s, g, subs, ld, Ke, E, mask, A);
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
  hipLaunchKernelGGL(k3_unscale, dim3(nbe, nsub), dim3(T3_NT), 0, s, A, ld, ms,
                     sdiag, A32);
}

void launch_local_inverse3(double* A, int ld, int nsub, double* sdiag,
                           double* LD, double* Lp, double* Rp, int* dropped,
                           float* A32, hipStream_t s) {
  launch_local_inverse3_strided(A, ld, nsub, (long long)ld * ld, sdiag, LD, Lp, Rp,
                                dropped, A32, s);
}

void launch_level1_3d(const Geom& g, const Sub3* subs, int nsub, int ld,
                      int nbx, int nby, int nbz, int S0, int S1, int S2,
                      const double* A64, const float* A32, const uint8_t* mask,
                      const double* r, double* lsol, double* z,
                      const CGScalars* sc, int use_l1, const Coarse3& cc,
                      hipStream_t s) {
  const dim3 gr(ld / 64, nsub);
  if (!use_l1) {
  } else if (A32 != nullptr)
    hipLaunchKernelGGL(k3_level1<float>, gr, dim3(T3_NT), 0, s, g, subs, ld, A32,
                       mask, r, lsol, sc);
  else
    hipLaunchKernelGGL(k3_level1<double>, gr, dim3(T3_NT), 0, s, g, subs, ld, A64,
                       mask, r, lsol, sc);
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
