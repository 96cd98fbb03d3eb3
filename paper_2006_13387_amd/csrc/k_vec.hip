// SIMP moduli, the matrix-free Q1 stiffness product and the CG vector
// kernels (2D).
//
// Stiffness product (paper Section 1.1: K = sum_e E_e P_e^T K^_e P_e with
// the SIMP modulus E_e): node-centric gather, so every output is written
// once and no atomics are needed.  A 64 x 4 tile of nodes stages its
// displacements (one-node halo) and the surrounding element moduli in LDS;
// each thread then sums the contributions of the four elements that share
// its node.  Rows of clamped DOFs are zero.
#include "common.h"
#include "dev.h"

namespace msp {

constexpr int MV_TX = 64;
constexpr int MV_TY = 4;
constexpr int MV_NT = MV_TX * MV_TY;

enum : int { MV_APPLY = 0, MV_CG = 1, MV_RESID = 2 };

__global__ void __launch_bounds__(256)
k_simp(const double* __restrict__ rho, double* __restrict__ E, int n,
       double E0, double Emin, double penal, int* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double r = rho[i];
  if (!(r >= 0.0 && r <= 1.0)) {   // also catches NaN
    atomicOr(err, ERR_RANGE);
    E[i] = Emin;
    return;
  }
  E[i] = Emin + pow(r, penal) * (E0 - Emin);
}

// MODE MV_APPLY : y = K x with x treated as 0 at clamped DOFs.
// MODE MV_CG    : p_new = z + beta p_old, q = K p_new, partial sums of
//                 p_new.q.  beta comes from the previous combine kernel's
//                 partials of r.z (and z.q), summed here by every
//                 workgroup in the same order: Fletcher-Reeves
//                 (r.z)_new/(r.z)_old, or, flexible, Polak-Ribiere
//                 -alpha (z.q)/(r.z)_old.  Workgroup 0 records beta.
//                 p_old and p_new are different buffers: neighbouring tiles
//                 read p_old in their halos while this tile writes p_new.
// MODE MV_RESID : r = f - K x (x is already 0 at clamped DOFs); partial
//                 sums of r.r, f.f and f.x over free DOFs.
template <int MODE>
__global__ void __launch_bounds__(MV_NT)
k_matvec(Geom g, const double* __restrict__ Ke, const double* __restrict__ E,
         const uint8_t* __restrict__ mask,
         const double* __restrict__ xin,     // APPLY: x, CG: z, RESID: x
         const double* __restrict__ pin,     // CG: p_old
         double* __restrict__ pout,          // CG: p_new
         double* __restrict__ yout,          // APPLY: y, CG: q, RESID: r
         const double* __restrict__ f,       // RESID: f
         CGScalars* __restrict__ sc, double* __restrict__ part,
         const double* __restrict__ part_comb, int nb_comb,
         double* __restrict__ beta_hist) {
  __shared__ double2 xs[(MV_TY + 2) * (MV_TX + 2)];
  __shared__ double es[(MV_TY + 1) * (MV_TX + 1)];
  __shared__ double ks[64];
  __shared__ double red[MV_NT / 64 + 1];
  __shared__ int shi;
  __shared__ double sh_beta;

  const int tid = threadIdx.x;
  double beta = 0.0;
  if (MODE == MV_CG) {
    if (block_read_done(sc, &shi)) return;
    const int it = sc->iter;                 // not written by this kernel
    if (it > 0) {
      const double rz = reduce_partials<MV_NT>(part_comb, nb_comb, 1, red);
      const double zq = sc->flexible ? reduce_partials<MV_NT>(part_comb + nb_comb, nb_comb, 1, red) : 0.0;
      if (tid == 0) {
        const double b = sc->flexible ? (-sc->alpha * zq / sc->rz) : (rz / sc->rz);
        sh_beta = b;
        if (blockIdx.x == 0 && blockIdx.y == 0) {
          sc->beta = b;
          if (it <= sc->maxit) beta_hist[it - 1] = b;
          if (!finite(b)) {
            sc->status = -5;
            __hip_atomic_store(&sc->done, (int)DONE_BREAKDOWN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
      __syncthreads();
      beta = sh_beta;
      if (!finite(beta)) return;
    }
  }
  const int bx0 = blockIdx.x * MV_TX - 1;   // node x of xs column 0
  const int by0 = blockIdx.y * MV_TY - 1;
  if (tid < 64) ks[tid] = Ke[tid];

  for (int t = tid; t < (MV_TY + 2) * (MV_TX + 2); t += MV_NT) {
    const int ii = t % (MV_TX + 2), jj = t / (MV_TX + 2);
    const int x = bx0 + ii, y = by0 + jj;
    double2 v = make_double2(0.0, 0.0);
    if (x >= 0 && x < g.nnx && y >= 0 && y < g.nny) {
      const long long node = (long long)y * g.nnx + x;
      const double2 a = reinterpret_cast<const double2*>(xin)[node];
      if (MODE == MV_CG) {
        const double2 po = reinterpret_cast<const double2*>(pin)[node];
        v = make_double2(a.x + beta * po.x, a.y + beta * po.y);
      } else if (MODE == MV_APPLY) {
        const uchar2 m = reinterpret_cast<const uchar2*>(mask)[node];
        v = make_double2(m.x ? 0.0 : a.x, m.y ? 0.0 : a.y);
      } else {
        v = a;
      }
    }
    xs[t] = v;
  }
  for (int t = tid; t < (MV_TY + 1) * (MV_TX + 1); t += MV_NT) {
    const int ii = t % (MV_TX + 1), jj = t / (MV_TX + 1);
    const int ex = bx0 + ii, ey = by0 + jj;
    double v = 0.0;
    if (ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny) v = E[(long long)ey * g.nx + ex];
    es[t] = v;
  }
  __syncthreads();

  const int i = tid % MV_TX, j = tid / MV_TX;
  const int x = blockIdx.x * MV_TX + i, y = blockIdx.y * MV_TY + j;
  const bool own = (x < g.nnx && y < g.nny);
  double y0 = 0.0, y1 = 0.0;
#pragma unroll
  for (int dy = 0; dy < 2; ++dy) {
#pragma unroll
    for (int dx = 0; dx < 2; ++dx) {
      const double ee = es[(j + dy) * (MV_TX + 1) + (i + dx)];
      const int a = (1 - dx) + 2 * (1 - dy);
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const double2 u = xs[(j + dy + (b >> 1)) * (MV_TX + 2) + (i + dx + (b & 1))];
        s0 += ks[(2 * a) * 8 + 2 * b] * u.x + ks[(2 * a) * 8 + 2 * b + 1] * u.y;
        s1 += ks[(2 * a + 1) * 8 + 2 * b] * u.x + ks[(2 * a + 1) * 8 + 2 * b + 1] * u.y;
      }
      y0 += ee * s0;
      y1 += ee * s1;
    }
  }

  double d0 = 0.0, d1 = 0.0, d2 = 0.0;
  if (own) {
    const long long node = (long long)y * g.nnx + x;
    const uchar2 m = reinterpret_cast<const uchar2*>(mask)[node];
    if (m.x) y0 = 0.0;
    if (m.y) y1 = 0.0;
    if (MODE == MV_APPLY) {
      reinterpret_cast<double2*>(yout)[node] = make_double2(y0, y1);
    } else if (MODE == MV_CG) {
      const double2 pn = xs[(j + 1) * (MV_TX + 2) + (i + 1)];
      reinterpret_cast<double2*>(pout)[node] = pn;
      reinterpret_cast<double2*>(yout)[node] = make_double2(y0, y1);
      d0 = pn.x * y0 + pn.y * y1;
    } else {
      const double2 ff = reinterpret_cast<const double2*>(f)[node];
      const double f0 = m.x ? 0.0 : ff.x, f1 = m.y ? 0.0 : ff.y;
      const double r0 = m.x ? 0.0 : f0 - y0, r1 = m.y ? 0.0 : f1 - y1;
      reinterpret_cast<double2*>(yout)[node] = make_double2(r0, r1);
      const double2 xx = xs[(j + 1) * (MV_TX + 2) + (i + 1)];
      d0 = r0 * r0 + r1 * r1;
      d1 = f0 * f0 + f1 * f1;
      d2 = f0 * xx.x + f1 * xx.y;
    }
  }
  if (MODE == MV_APPLY) return;

  const unsigned int nb = gridDim.x * gridDim.y;
  const unsigned int bid = blockIdx.y * gridDim.x + blockIdx.x;
  const double s0 = block_sum<MV_NT>(d0, red);
  if (MODE == MV_CG) {
    if (tid == 0) part[bid] = s0;
  } else {
    const double s1 = block_sum<MV_NT>(d1, red);
    const double s2 = block_sum<MV_NT>(d2, red);
    if (tid == 0) {
      part[bid] = s0;
      part[nb + bid] = s1;
      part[2 * nb + bid] = s2;
    }
  }
}

// One workgroup: sum the residual kernel's partials (r.r, f.f, f.x).
// slot 0 (start of a CG segment): rr, rr0 and ff; slot 1 (true residual at
// exit): rr0 = true r.r, ff and fx.
__global__ void __launch_bounds__(256)
k_resid_finish(CGScalars* __restrict__ sc, const double* __restrict__ part,
               int nb, int slot) {
  __shared__ double red[256 / 64 + 1];
  const double rr = reduce_partials<256>(part, nb, 1, red);
  const double ff = reduce_partials<256>(part + nb, nb, 1, red);
  const double fx = reduce_partials<256>(part + 2 * nb, nb, 1, red);
  if (threadIdx.x == 0) {
    if (slot == 0) {
      sc->rr = rr;
      sc->rr0 = rr;
      sc->ff = ff;
    } else {
      sc->rr0 = rr;
      sc->ff = ff;
      sc->fx = fx;
    }
  }
}

// x += alpha p ; r -= alpha q ; partial sums of r.r.  alpha = (r.z)/(p.q)
// from the partials of the combine and stiffness kernels, summed by every
// workgroup in the same order; workgroup 0 records alpha and r.z.
__global__ void __launch_bounds__(256)
k_update(long long n2, double* __restrict__ x, double* __restrict__ r,
         const double* __restrict__ p, const double* __restrict__ q,
         CGScalars* __restrict__ sc, double* __restrict__ alpha_hist,
         double* __restrict__ part, const double* __restrict__ part_mv,
         int nb_mv, const double* __restrict__ part_comb, int nb_comb) {
  __shared__ double red[256 / 64 + 1];
  __shared__ int shi;
  __shared__ double sh_alpha;
  if (block_read_done(sc, &shi)) return;
  const double pq = reduce_partials<256>(part_mv, nb_mv, 1, red);
  const double rz = reduce_partials<256>(part_comb, nb_comb, 1, red);
  if (threadIdx.x == 0) {
    const bool bad = !(pq > 0.0) || !finite(pq) || !finite(rz);
    const double alpha = bad ? 0.0 : rz / pq;
    sh_alpha = bad ? __builtin_nan("") : alpha;
    if (blockIdx.x == 0) {
      const int it = sc->iter;
      sc->pq = pq;
      sc->alpha = alpha;
      sc->rz = rz;
      if (it < sc->maxit) alpha_hist[it] = alpha;
      if (bad) {
        sc->status = -5;
        __hip_atomic_store(&sc->done, (int)DONE_BREAKDOWN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
  __syncthreads();
  const double alpha = sh_alpha;
  if (!finite(alpha)) return;
  double acc = 0.0;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n2) {
    double2 xx = reinterpret_cast<double2*>(x)[i];
    double2 rr = reinterpret_cast<double2*>(r)[i];
    const double2 pp = reinterpret_cast<const double2*>(p)[i];
    const double2 qq = reinterpret_cast<const double2*>(q)[i];
    xx.x += alpha * pp.x;
    xx.y += alpha * pp.y;
    rr.x -= alpha * qq.x;
    rr.y -= alpha * qq.y;
    reinterpret_cast<double2*>(x)[i] = xx;
    reinterpret_cast<double2*>(r)[i] = rr;
    acc = rr.x * rr.x + rr.y * rr.y;
  }
  const double s = block_sum<256>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256)
k_dot(long long n, const double* __restrict__ x, const double* __restrict__ y,
      double* __restrict__ part, unsigned int* __restrict__ counter,
      double* __restrict__ out) {
  __shared__ double red[256 / 64 + 1];
  __shared__ unsigned int ticket;
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)gridDim.x * 256)
    acc += x[i] * y[i];
  const double s = block_sum<256>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
  if (!last_block(counter, gridDim.x, &ticket)) return;
  const double t = reduce_partials<256>(part, gridDim.x, 1, red);
  if (threadIdx.x == 0) {
    *out = t;
    *counter = 0u;
  }
}

__global__ void __launch_bounds__(256)
k_mask(long long n, const uint8_t* __restrict__ mask, double* __restrict__ x) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n && mask[i]) x[i] = 0.0;
}

// ---------------------------------------------------------------- launchers

void launch_mask(long long n, const uint8_t* mask, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_mask, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     n, mask, x);
}

void launch_simp(const double* rho, double* E, int n, double E0, double Emin,
                 double penal, int* err, hipStream_t s) {
  hipLaunchKernelGGL(k_simp, dim3((n + 255) / 256), dim3(256), 0, s, rho, E, n,
                     E0, Emin, penal, err);
}

static dim3 mv_grid(const Geom& g) {
  return dim3((g.nnx + MV_TX - 1) / MV_TX, (g.nny + MV_TY - 1) / MV_TY);
}

int matvec_blocks(const Geom& g) {
  const dim3 gr = mv_grid(g);
  return gr.x * gr.y;
}

void launch_apply_K(const Geom& g, const double* Ke, const double* E,
                    const uint8_t* mask, const double* x, double* y,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_matvec<MV_APPLY>, mv_grid(g), dim3(MV_NT), 0, s, g, Ke,
                     E, mask, x, (const double*)nullptr, (double*)nullptr, y,
                     (const double*)nullptr, (CGScalars*)nullptr,
                     (double*)nullptr, (const double*)nullptr, 0,
                     (double*)nullptr);
}

void launch_cg_matvec(const Geom& g, const double* Ke, const double* E,
                      const uint8_t* mask, const double* z, const double* p_old,
                      double* p_new, double* q, CGScalars* sc, double* part_mv,
                      const double* part_comb, int nb_comb, double* beta_hist,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_matvec<MV_CG>, mv_grid(g), dim3(MV_NT), 0, s, g, Ke, E,
                     mask, z, p_old, p_new, q, (const double*)nullptr, sc,
                     part_mv, part_comb, nb_comb, beta_hist);
}

void launch_residual(const Geom& g, const double* Ke, const double* E,
                     const uint8_t* mask, const double* x, const double* f,
                     double* r, CGScalars* sc, double* part, int slot,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_matvec<MV_RESID>, mv_grid(g), dim3(MV_NT), 0, s, g, Ke,
                     E, mask, x, (const double*)nullptr, (double*)nullptr, r, f,
                     sc, part, (const double*)nullptr, 0, (double*)nullptr);
  hipLaunchKernelGGL(k_resid_finish, dim3(1), dim3(256), 0, s, sc, part,
                     matvec_blocks(g), slot);
}

int update_blocks(long long n) { return (int)((n / 2 + 255) / 256); }

void launch_update(long long n, double* x, double* r, const double* p,
                   const double* q, CGScalars* sc, double* alpha_hist,
                   double* part_upd, const double* part_mv, int nb_mv,
                   const double* part_comb, int nb_comb, hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(update_blocks(n)), dim3(256), 0, s, n / 2,
                     x, r, p, q, sc, alpha_hist, part_upd, part_mv, nb_mv,
                     part_comb, nb_comb);
}

void launch_dot(long long n, const double* x, const double* y, double* part,
                unsigned int* counter, double* out, hipStream_t s) {
  long long nb = (n + 255) / 256;
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_dot, dim3((unsigned)nb), dim3(256), 0, s, n, x, y, part,
                     counter, out);
}

}  // namespace msp
