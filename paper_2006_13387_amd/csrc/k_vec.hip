// SIMP moduli, the matrix-free Q1 stiffness product and the CG vector
// kernels (2D).
//
// Stiffness product (paper Section 1.1: K = sum_e E_e P_e^T K^_e P_e with
// the SIMP modulus E_e): node-centric gather, so every output is written
// once and no atomics are needed.  A tile of 64 x TY nodes stages its
// displacements (one-node halo) and the surrounding element moduli in LDS;
// each thread then sums the contributions of the four elements that share
// its node.  Rows of clamped DOFs are zero.  The tile height (4, 8, 16 or
// 32 node rows, 256 threads) is a function of the mesh: taller tiles re-read
// fewer halo nodes and moduli.  Tiles are ordered so that each XCD takes a
// contiguous range of them (overlapping halos meet in its L2); the product
// alone on large meshes runs in persistent workgroups that load the next
// tile while computing the current one.  The element matrix comes in the
// kernel arguments (scalar loads shared by the wave).
#include <algorithm>

#include "common.h"
#include "dev.h"

namespace msp {

constexpr int MV_TX = 64;        // nodes per tile row
constexpr int MV_NT = 256;       // threads: tile rows are processed 4 at a time
constexpr int MV_TYMAX = 16;     // tallest tile of the batched product
constexpr int MV_TYBIG = 32;     // tallest tile of the single-problem product
constexpr int NUM_XCD = 8;       // workgroups go round-robin to the chip's XCDs
constexpr int kNumCUsVec = 256;  // compute units of the chip

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

// LDS of one stiffness-product tile of TYL node rows (or fewer)
template <int TYL>
struct MvLdsT {
  double2 xs[(TYL + 2) * (MV_TX + 2)];
  double es[(TYL + 1) * (MV_TX + 1)];
  double red[2 * (MV_NT / 64)];
  int shi;
  double beta;
};
typedef MvLdsT<MV_TYMAX> MvLds;


// Tile (bx, by) of a gx x gy grid of 64 x TY node tiles.
// MODE MV_APPLY : y = K x with x treated as 0 at clamped DOFs.
// MODE MV_CG    : p_new = z + beta p_old, q = K p_new, partial sums of
//                 p_new.q.  beta comes from the previous combine kernel's
//                 partials of r.z (and z.q), summed here by every
//                 workgroup in the same order: Fletcher-Reeves
//                 (r.z)_new/(r.z)_old, or, flexible, Polak-Ribiere
//                 -alpha (z.q)/(r.z)_old.  Tile 0 records beta.
//                 p_old and p_new are different buffers: neighbouring tiles
//                 read p_old in their halos while this tile writes p_new.
// MODE MV_RESID : r = f - K x (x is already 0 at clamped DOFs); partial
//                 sums of r.r, f.f and f.x over free DOFs.
template <int MODE, int TY, typename LT>
__device__ __forceinline__ void matvec_body(const MatvecArgs& a, int bx, int by,
                                            int gx, int gy, LT& L) {
  static_assert(TY % 4 == 0 && sizeof(L.xs) >= (TY + 2) * (MV_TX + 2) * sizeof(double2),
                "tile height");
  constexpr int RPT = TY / 4;                // rows per thread
  constexpr int NXN = (TY + 2) * (MV_TX + 2);               // halo nodes
  constexpr int NEN = (TY + 1) * (MV_TX + 1);               // moduli
  constexpr int NXS = (NXN + MV_NT - 1) / MV_NT;            // per thread
  constexpr int NES = (NEN + MV_NT - 1) / MV_NT;
  const Geom& g = a.g;
  const int tid = threadIdx.x;
  const int bx0 = bx * MV_TX - 1;   // node x of xs column 0
  const int by0 = by * TY - 1;
  // Every read goes out before the first use (one memory latency): the
  // tile's halo of the input (CG: z and p_old), the moduli, the element
  // matrix and, CG, the done word, the scalars and the combine kernel's
  // partials of r.z and z.q (the z.q half is used only when flexible).
  int dn = DONE_RUNNING, it = 0, flex = 0, maxit = 0;
  double alpha_o = 0.0, rz_o = 0.0;
  double srz = 0.0, szq = 0.0;
  if (MODE == MV_CG) {
    if (tid == 0) {
      dn = __hip_atomic_load(&a.sc->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      it = a.sc->iter;                       // not written by this kernel
      flex = a.sc->flexible;
      maxit = a.sc->maxit;
      alpha_o = a.sc->alpha;
      rz_o = a.sc->rz;
    }
    for (int k = tid; k < a.nb_comb; k += MV_NT) {
      srz += load_coherent(a.part_comb + k);
      szq += load_coherent(a.part_comb + a.nb_comb + k);
    }
  }
  double2 xu[NXS], xp[NXS];
  uchar2 xm[NXS];
#pragma unroll
  for (int k = 0; k < NXS; ++k) {
    const int t = tid + k * MV_NT;
    const int ii = t % (MV_TX + 2), jj = t / (MV_TX + 2);
    const int x = bx0 + ii, y = by0 + jj;
    xu[k] = xp[k] = make_double2(0.0, 0.0);
    xm[k] = make_uchar2(1, 1);
    if (t < NXN && x >= 0 && x < g.nnx && y >= 0 && y < g.nny) {
      const long long node = (long long)y * g.nnx + x;
      xu[k] = reinterpret_cast<const double2*>(a.xin)[node];
      if (MODE == MV_CG) xp[k] = reinterpret_cast<const double2*>(a.pin)[node];
      if (MODE == MV_APPLY) xm[k] = reinterpret_cast<const uchar2*>(a.mask)[node];
    }
  }
  double ev[NES];
#pragma unroll
  for (int k = 0; k < NES; ++k) {
    const int t = tid + k * MV_NT;
    const int ii = t % (MV_TX + 1), jj = t / (MV_TX + 1);
    const int ex = bx0 + ii, ey = by0 + jj;
    ev[k] = (t < NEN && ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny)
                ? a.E[(long long)ey * g.nx + ex] : 0.0;
  }
  double beta = 0.0;
  if (MODE == MV_CG) {
    const double2 sums = block_sum2<MV_NT>(srz, szq, L.red);
    if (tid == 0) {
      bool stop = dn != DONE_RUNNING;
      double b = 0.0;
      if (!stop && it > 0) {
        b = flex ? (-alpha_o * sums.y / rz_o) : (sums.x / rz_o);
        if (bx == 0 && by == 0) {
          a.sc->beta = b;
          if (it <= maxit) a.beta_hist[it - 1] = b;
          if (!finite(b)) {
            a.sc->status = -5;
            __hip_atomic_store(&a.sc->done, (int)DONE_BREAKDOWN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
        stop = !finite(b);
      }
      L.beta = stop ? __builtin_nan("") : b;
    }
    __syncthreads();
    beta = L.beta;
    if (!finite(beta)) return;
  }
#pragma unroll
  for (int k = 0; k < NXS; ++k) {
    const int t = tid + k * MV_NT;
    if (t < NXN) {
      double2 v = xu[k];
      if (MODE == MV_CG) v = make_double2(fma(beta, xp[k].x, xu[k].x), fma(beta, xp[k].y, xu[k].y));
      if (MODE == MV_APPLY) v = make_double2(xm[k].x ? 0.0 : xu[k].x, xm[k].y ? 0.0 : xu[k].y);
      L.xs[t] = v;
    }
  }
#pragma unroll
  for (int k = 0; k < NES; ++k) {
    const int t = tid + k * MV_NT;
    if (t < NEN) L.es[t] = ev[k];
  }
  __syncthreads();

  const int i = tid % MV_TX;
  double d0 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int j = tid / MV_TX + 4 * rr;
    const int x = bx * MV_TX + i, y = by * TY + j;
    const bool own = (x < g.nnx && y < g.nny);
    double y0 = 0.0, y1 = 0.0;
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const double ee = L.es[(j + dy) * (MV_TX + 1) + (i + dx)];
        const int av = (1 - dx) + 2 * (1 - dy);
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const double2 u = L.xs[(j + dy + (b >> 1)) * (MV_TX + 2) + (i + dx + (b & 1))];
          // explicit FMAs: the single and the batched kernel round alike
          s0 = fma(a.ke[(2 * av) * 8 + 2 * b], u.x, s0);
          s0 = fma(a.ke[(2 * av) * 8 + 2 * b + 1], u.y, s0);
          s1 = fma(a.ke[(2 * av + 1) * 8 + 2 * b], u.x, s1);
          s1 = fma(a.ke[(2 * av + 1) * 8 + 2 * b + 1], u.y, s1);
        }
        y0 = fma(ee, s0, y0);
        y1 = fma(ee, s1, y1);
      }
    }
    if (own) {
      const long long node = (long long)y * g.nnx + x;
      const uchar2 m = reinterpret_cast<const uchar2*>(a.mask)[node];
      if (m.x) y0 = 0.0;
      if (m.y) y1 = 0.0;
      if (MODE == MV_APPLY) {
        reinterpret_cast<double2*>(a.yout)[node] = make_double2(y0, y1);
      } else if (MODE == MV_CG) {
        const double2 pn = L.xs[(j + 1) * (MV_TX + 2) + (i + 1)];
        reinterpret_cast<double2*>(a.pout)[node] = pn;
        reinterpret_cast<double2*>(a.yout)[node] = make_double2(y0, y1);
        d0 = fma(pn.y, y1, fma(pn.x, y0, d0));
      } else {
        const double2 ff = reinterpret_cast<const double2*>(a.f)[node];
        const double f0 = m.x ? 0.0 : ff.x, f1 = m.y ? 0.0 : ff.y;
        const double r0 = m.x ? 0.0 : f0 - y0, r1 = m.y ? 0.0 : f1 - y1;
        reinterpret_cast<double2*>(a.yout)[node] = make_double2(r0, r1);
        const double2 xx = L.xs[(j + 1) * (MV_TX + 2) + (i + 1)];
        d0 = fma(r1, r1, fma(r0, r0, d0));
        d1 = fma(f1, f1, fma(f0, f0, d1));
        d2 = fma(f1, xx.y, fma(f0, xx.x, d2));
      }
    }
  }
  if (MODE == MV_APPLY) return;

  const int nb = gx * gy;
  const int bid = by * gx + bx;
  const double s0 = block_sum<MV_NT>(d0, L.red);
  if (MODE == MV_CG) {
    if (tid == 0) a.part[bid] = s0;
  } else {
    const double s1 = block_sum<MV_NT>(d1, L.red);
    const double s2 = block_sum<MV_NT>(d2, L.red);
    if (tid == 0) {
      a.part[bid] = s0;
      a.part[nb + bid] = s1;
      a.part[2 * nb + bid] = s2;
    }
  }
}

template <int MODE>
__device__ __forceinline__ void matvec_dispatch(const MatvecArgs& a, int bx,
                                                int by, int gx, int gy, MvLds& L) {
  if (a.ty == 4) matvec_body<MODE, 4>(a, bx, by, gx, gy, L);
  else if (a.ty == 8) matvec_body<MODE, 8>(a, bx, by, gx, gy, L);
  else matvec_body<MODE, 16>(a, bx, by, gx, gy, L);
}

// Tile of workgroup k of a 1D grid of nb tiles: the hardware hands
// workgroups to the XCDs in turn (k % 8), so XCD x gets the contiguous
// range of tiles x * nb/8 .. and neighbouring tiles, whose halos overlap,
// meet in the same L2.
__device__ __forceinline__ int xcd_tile(int k, int nb) {
  const int q = nb / NUM_XCD, rem = nb - q * NUM_XCD;
  const int x = k % NUM_XCD, slot = k / NUM_XCD;
  return x * q + min(x, rem) + slot;
}

template <int MODE, int TY>
__global__ void __launch_bounds__(MV_NT) k_matvec(MatvecArgs a) {
  __shared__ MvLdsT<TY> L;
  const int gx = (a.g.nnx + MV_TX - 1) / MV_TX;
  const int gy = (a.g.nny + TY - 1) / TY;
  const int t = xcd_tile(blockIdx.x, gx * gy);
  matvec_body<MODE, TY>(a, t % gx, t / gx, gx, gy, L);
}

// y = K x (x treated as 0 at clamped DOFs, y = 0 there) on meshes of many
// tiles: persistent workgroups, eight groups of them, one per XCD, each
// group walking the contiguous range of tiles of its XCD with the group's
// stride (neighbouring tiles, whose halos overlap, meet in the same L2).
// The next tile's x halo, clamp flags and moduli are loaded into registers
// while the current tile is computed from LDS, so the loads of one tile
// overlap the arithmetic of the previous one.
template <int TY>
__global__ void __launch_bounds__(MV_NT)
k_matvec_apply_pf(MatvecArgs a) {
  __shared__ MvLdsT<TY> L;
  __shared__ uchar2 ms[(TY + 2) * (MV_TX + 2)];
  constexpr int RPT = TY / 4;
  constexpr int NXN = (TY + 2) * (MV_TX + 2);
  constexpr int NEN = (TY + 1) * (MV_TX + 1);
  constexpr int NXS = (NXN + MV_NT - 1) / MV_NT;
  constexpr int NES = (NEN + MV_NT - 1) / MV_NT;
  const Geom& g = a.g;
  const int tid = threadIdx.x;
  const int gx = (g.nnx + MV_TX - 1) / MV_TX, gy = (g.nny + TY - 1) / TY;
  const int nt = gx * gy;
  const int xcd = blockIdx.x % NUM_XCD, stride = gridDim.x / NUM_XCD;
  const int q = nt / NUM_XCD, rem = nt - q * NUM_XCD;
  const int t_end = xcd * q + min(xcd, rem) + q + (xcd < rem ? 1 : 0);
  int t = xcd * q + min(xcd, rem) + blockIdx.x / NUM_XCD;
  if (t >= t_end) return;
  double2 xu[NXS];
  uchar2 xm[NXS];
  double ev[NES];
  auto load = [&](int tile) {
    const int bx0 = (tile % gx) * MV_TX - 1, by0 = (tile / gx) * TY - 1;
#pragma unroll
    for (int k = 0; k < NXS; ++k) {
      const int u = tid + k * MV_NT;
      const int x = bx0 + u % (MV_TX + 2), y = by0 + u / (MV_TX + 2);
      xu[k] = make_double2(0.0, 0.0);
      xm[k] = make_uchar2(1, 1);
      if (u < NXN && x >= 0 && x < g.nnx && y >= 0 && y < g.nny) {
        const long long node = (long long)y * g.nnx + x;
        xu[k] = reinterpret_cast<const double2*>(a.xin)[node];
        xm[k] = reinterpret_cast<const uchar2*>(a.mask)[node];
      }
    }
#pragma unroll
    for (int k = 0; k < NES; ++k) {
      const int u = tid + k * MV_NT;
      const int ex = bx0 + u % (MV_TX + 1), ey = by0 + u / (MV_TX + 1);
      ev[k] = (u < NEN && ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny)
                  ? a.E[(long long)ey * g.nx + ex] : 0.0;
    }
  };
  load(t);
  for (;;) {
#pragma unroll
    for (int k = 0; k < NXS; ++k) {
      const int u = tid + k * MV_NT;
      if (u < NXN) {
        L.xs[u] = make_double2(xm[k].x ? 0.0 : xu[k].x, xm[k].y ? 0.0 : xu[k].y);
        ms[u] = xm[k];
      }
    }
#pragma unroll
    for (int k = 0; k < NES; ++k) {
      const int u = tid + k * MV_NT;
      if (u < NEN) L.es[u] = ev[k];
    }
    __syncthreads();
    const int bx = t % gx, by = t / gx;
    const int tn = t + stride;
    if (tn < t_end) load(tn);
    const int i = tid % MV_TX;
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
      const int j = tid / MV_TX + 4 * rr;
      const int x = bx * MV_TX + i, y = by * TY + j;
      double y0 = 0.0, y1 = 0.0;
#pragma unroll
      for (int dy = 0; dy < 2; ++dy) {
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
          const double ee = L.es[(j + dy) * (MV_TX + 1) + (i + dx)];
          const int av = (1 - dx) + 2 * (1 - dy);
          const double* ke = a.ke;
          double s0 = 0.0, s1 = 0.0;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const double2 u = L.xs[(j + dy + (b >> 1)) * (MV_TX + 2) + (i + dx + (b & 1))];
            s0 = fma(ke[(2 * av) * 8 + 2 * b], u.x, s0);
            s0 = fma(ke[(2 * av) * 8 + 2 * b + 1], u.y, s0);
            s1 = fma(ke[(2 * av + 1) * 8 + 2 * b], u.x, s1);
            s1 = fma(ke[(2 * av + 1) * 8 + 2 * b + 1], u.y, s1);
          }
          y0 = fma(ee, s0, y0);
          y1 = fma(ee, s1, y1);
        }
      }
      if (x < g.nnx && y < g.nny) {
        const uchar2 m = ms[(j + 1) * (MV_TX + 2) + (i + 1)];
        reinterpret_cast<double2*>(a.yout)[(long long)y * g.nnx + x] =
            make_double2(m.x ? 0.0 : y0, m.y ? 0.0 : y1);
      }
    }
    __syncthreads();
    if (tn >= t_end) break;
    t = tn;
  }
}

// The CG stiffness products of several problems in one launch.
__global__ void __launch_bounds__(MV_NT)
k_matvec_cg_batch(const MatvecArgs* __restrict__ tab, const int* __restrict__ start,
                  int nent) {
  __shared__ MvLds L;
  const int e = batch_entry(start, nent, blockIdx.x);
  const MatvecArgs a = tab[e];
  const int gx = (a.g.nnx + MV_TX - 1) / MV_TX;
  const int gy = (a.g.nny + a.ty - 1) / a.ty;
  const int lb = blockIdx.x - start[e];
  matvec_dispatch<MV_CG>(a, lb % gx, lb / gx, gx, gy, L);
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

struct UpLds {
  double red[2 * (256 / 64)];
  double alpha;
};

constexpr int UP_NPT = 2;   // nodes per thread (fewer workgroups re-reducing the partials)

// x += alpha p ; r -= alpha q ; partial sums of r.r.  alpha = (r.z)/(p.q)
// from the partials of the combine and stiffness kernels, summed by every
// workgroup in the same order; workgroup 0 records alpha and r.z.  Every
// read (the done word, both partial sets, this thread's entries) goes out
// at once, so the kernel waits for memory once before its stores.
__device__ __forceinline__ void update_body(const UpdateArgs& a, int bid, UpLds& L) {
  int d0 = DONE_RUNNING;
  if (threadIdx.x == 0)
    d0 = __hip_atomic_load(&a.sc->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  double spq = 0.0, srz = 0.0;
  for (int k = threadIdx.x; k < a.nb_mv; k += 256) spq += load_coherent(a.part_mv + k);
  for (int k = threadIdx.x; k < a.nb_comb; k += 256) srz += load_coherent(a.part_comb + k);
  long long i[UP_NPT];
  bool own[UP_NPT];
  double2 xx[UP_NPT], rr[UP_NPT], pp[UP_NPT], qq[UP_NPT];
#pragma unroll
  for (int k = 0; k < UP_NPT; ++k) {
    i[k] = ((long long)bid * UP_NPT + k) * 256 + threadIdx.x;
    own[k] = i[k] < a.n2;
    xx[k] = rr[k] = pp[k] = qq[k] = make_double2(0.0, 0.0);
    if (own[k]) {
      xx[k] = reinterpret_cast<double2*>(a.x)[i[k]];
      rr[k] = reinterpret_cast<double2*>(a.r)[i[k]];
      pp[k] = reinterpret_cast<const double2*>(a.p)[i[k]];
      qq[k] = reinterpret_cast<const double2*>(a.q)[i[k]];
    }
  }
  const double2 sums = block_sum2<256>(spq, srz, L.red);
  const double pq = sums.x, rz = sums.y;
  if (threadIdx.x == 0) {
    const bool bad = !(pq > 0.0) || !finite(pq) || !finite(rz);
    const double alpha = bad ? 0.0 : rz / pq;
    L.alpha = (bad || d0 != DONE_RUNNING) ? __builtin_nan("") : alpha;
    if (bid == 0 && d0 == DONE_RUNNING) {
      const int it = a.sc->iter;
      a.sc->pq = pq;
      a.sc->alpha = alpha;
      a.sc->rz = rz;
      if (it < a.sc->maxit) a.alpha_hist[it] = alpha;
      if (bad) {
        a.sc->status = -5;
        __hip_atomic_store(&a.sc->done, (int)DONE_BREAKDOWN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
  __syncthreads();
  const double alpha = L.alpha;
  if (!finite(alpha)) return;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < UP_NPT; ++k) {
    if (!own[k]) continue;
    xx[k].x += alpha * pp[k].x;
    xx[k].y += alpha * pp[k].y;
    rr[k].x -= alpha * qq[k].x;
    rr[k].y -= alpha * qq[k].y;
    reinterpret_cast<double2*>(a.x)[i[k]] = xx[k];
    reinterpret_cast<double2*>(a.r)[i[k]] = rr[k];
    acc += rr[k].x * rr[k].x + rr[k].y * rr[k].y;
  }
  const double s = block_sum<256>(acc, L.red);
  if (threadIdx.x == 0) a.part[bid] = s;
}

__global__ void __launch_bounds__(256) k_update(UpdateArgs a) {
  __shared__ UpLds L;
  update_body(a, blockIdx.x, L);
}

__global__ void __launch_bounds__(256)
k_update_batch(const UpdateArgs* __restrict__ tab, const int* __restrict__ start,
               int nent) {
  __shared__ UpLds L;
  const int e = batch_entry(start, nent, blockIdx.x);
  update_body(tab[e], blockIdx.x - start[e], L);
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

// 3D (H8) stiffness product on the free DOFs: y = K(E) x with x's fixed
// entries read as 0 and y = 0 at fixed DOFs (Section 1.1 in three
// dimensions).  One thread per node, x the fastest axis.  For each of the
// node's 27 neighbours the element matrix blocks of the elements that hold
// both nodes act on the neighbour's three values; the sums are kept per
// element and scaled by its modulus at the end.  Ke is the unit-modulus
// element matrix (24 x 24, vertex a = ax + 2 ay + 4 az, DOF 3a + c), staged
// in LDS and read at compile-time offsets (the same address for the whole
// wave).  nmask: per node, bit c set when DOF c is fixed.
__global__ void __launch_bounds__(256)
k_matvec3d(Geom g, const double* __restrict__ Ke, const double* __restrict__ E,
           const uint8_t* __restrict__ nmask, const double* __restrict__ x,
           double* __restrict__ y, const CGScalars* __restrict__ sc) {
  __shared__ double K[576];
  __shared__ int shd;
  if (sc != nullptr && block_read_done(sc, &shd)) return;   // PCG run over
  for (int q = threadIdx.x; q < 576; q += 256) K[q] = Ke[q];
  __syncthreads();
  const long long nn = (long long)g.nnx * g.nny * g.nnz;
  const long long node = min((long long)blockIdx.x * 256 + threadIdx.x, nn - 1);
  const bool own = (long long)blockIdx.x * 256 + threadIdx.x < nn;
  const int i = (int)(node % g.nnx);
  const long long rr = node / g.nnx;
  const int j = (int)(rr % g.nny), k = (int)(rr / g.nny);
  // element e around the node: (i - 1 + ex, j - 1 + ey, k - 1 + ez)
  double Ee[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int ei = i - 1 + (e & 1), ej = j - 1 + ((e >> 1) & 1), ek = k - 1 + (e >> 2);
    const bool in = ei >= 0 && ei < g.nx && ej >= 0 && ej < g.ny && ek >= 0 && ek < g.nz;
    Ee[e] = in ? E[((long long)ek * g.ny + ej) * g.nx + ei] : 0.0;
  }
  double acc[8][3];
#pragma unroll
  for (int e = 0; e < 8; ++e) acc[e][0] = acc[e][1] = acc[e][2] = 0.0;
  // neighbours (dx, dy, dz): dy, dz in uniform loops, dx unrolled
#pragma unroll 1
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll 1
    for (int dy = -1; dy <= 1; ++dy) {
      const int bj = j + dy, bk = k + dz;
      const bool inyz = bj >= 0 && bj < g.nny && bk >= 0 && bk < g.nnz;
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int bi = i + dx;
        const bool in = inyz && bi >= 0 && bi < g.nnx;
        const long long nb = in ? ((long long)bk * g.nny + bj) * g.nnx + bi : node;
        const unsigned mb = in ? nmask[nb] : 7u;
        const double v0 = x[3 * nb], v1 = x[3 * nb + 1], v2 = x[3 * nb + 2];
        const double x0 = (mb & 1u) ? 0.0 : v0;
        const double x1 = (mb & 2u) ? 0.0 : v1;
        const double x2 = (mb & 4u) ? 0.0 : v2;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int ex = e & 1, ey = (e >> 1) & 1, ez = e >> 2;
          // the element holds the neighbour iff each offset lies in {e - 1, e}
          if (dx < ex - 1 || dx > ex) continue;
          if (dy < ey - 1 || dy > ey || dz < ez - 1 || dz > ez) continue;
          const int a = (1 - ex) + 2 * (1 - ey) + 4 * (1 - ez);
          const int b = (dx + 1 - ex) + 2 * (dy + 1 - ey) + 4 * (dz + 1 - ez);
          const double* kr = K + 3 * a * 24 + 3 * b;
          acc[e][0] += kr[0] * x0 + kr[1] * x1 + kr[2] * x2;
          acc[e][1] += kr[24] * x0 + kr[25] * x1 + kr[26] * x2;
          acc[e][2] += kr[48] * x0 + kr[49] * x1 + kr[50] * x2;
        }
      }
    }
  double y0 = 0.0, y1 = 0.0, y2 = 0.0;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    y0 += Ee[e] * acc[e][0];
    y1 += Ee[e] * acc[e][1];
    y2 += Ee[e] * acc[e][2];
  }
  if (!own) return;
  const unsigned m = nmask[node];
  y[3 * node] = (m & 1u) ? 0.0 : y0;
  y[3 * node + 1] = (m & 2u) ? 0.0 : y1;
  y[3 * node + 2] = (m & 4u) ? 0.0 : y2;
}

void launch_apply_K3(const Geom& g, const double* Ke, const double* E,
                     const uint8_t* nmask, const double* x, double* y,
                     hipStream_t s, const CGScalars* sc) {
  const long long nn = (long long)g.nnx * g.nny * g.nnz;
  hipLaunchKernelGGL(k_matvec3d, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s,
                     g, Ke, E, nmask, x, y, sc);
}

void launch_mask(long long n, const uint8_t* mask, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_mask, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     n, mask, x);
}

void launch_simp(const double* rho, double* E, int n, double E0, double Emin,
                 double penal, int* err, hipStream_t s) {
  hipLaunchKernelGGL(k_simp, dim3((n + 255) / 256), dim3(256), 0, s, rho, E, n,
                     E0, Emin, penal, err);
}

int matvec_blocks(const Geom& g, int ty) {
  return ((g.nnx + MV_TX - 1) / MV_TX) * ((g.nny + ty - 1) / ty);
}

template <int MODE>
static void launch_mv(const MatvecArgs& a, hipStream_t s) {
  const dim3 gr(matvec_blocks(a.g, a.ty));
  if (a.ty == 4) hipLaunchKernelGGL((k_matvec<MODE, 4>), gr, dim3(MV_NT), 0, s, a);
  else if (a.ty == 8) hipLaunchKernelGGL((k_matvec<MODE, 8>), gr, dim3(MV_NT), 0, s, a);
  else if (a.ty == 16) hipLaunchKernelGGL((k_matvec<MODE, 16>), gr, dim3(MV_NT), 0, s, a);
  else hipLaunchKernelGGL((k_matvec<MODE, MV_TYBIG>), gr, dim3(MV_NT), 0, s, a);
}

static MatvecArgs mv_args(const Geom& g, int ty, const double* Ke, const double* E,
                          const uint8_t* mask) {
  MatvecArgs a{};
  a.g = g;
  a.ty = ty;
  for (int i = 0; i < 64; ++i) a.ke[i] = Ke[i];
  a.E = E;
  a.mask = mask;
  return a;
}

void launch_apply_K(const Geom& g, int ty, const double* Ke, const double* E,
                    const uint8_t* mask, const double* x, double* y,
                    hipStream_t s) {
  MatvecArgs a = mv_args(g, ty, Ke, E, mask);
  a.xin = x;
  a.yout = y;
  const int nt = matvec_blocks(g, ty);
  if (nt < 16 * kNumCUsVec || ty < 8) {
    launch_mv<MV_APPLY>(a, s);
    return;
  }
  // persistent: as many workgroups as fit on the chip at once (registers
  // allow four per CU with 8-row tiles, three with taller ones), a multiple
  // of the XCD count
  const int per_cu = ty == 8 ? 4 : 3;
  const int per_xcd = std::min((nt + NUM_XCD - 1) / NUM_XCD, per_cu * kNumCUsVec / NUM_XCD);
  const dim3 gr(per_xcd * NUM_XCD);
  if (ty == 8) hipLaunchKernelGGL(k_matvec_apply_pf<8>, gr, dim3(MV_NT), 0, s, a);
  else if (ty == 16) hipLaunchKernelGGL(k_matvec_apply_pf<16>, gr, dim3(MV_NT), 0, s, a);
  else hipLaunchKernelGGL(k_matvec_apply_pf<MV_TYBIG>, gr, dim3(MV_NT), 0, s, a);
}

MatvecArgs cg_matvec_args(const Geom& g, int ty, const double* Ke,
                          const double* E, const uint8_t* mask, const double* z,
                          const double* p_old, double* p_new, double* q,
                          CGScalars* sc, double* part_mv,
                          const double* part_comb, int nb_comb,
                          double* beta_hist) {
  MatvecArgs a = mv_args(g, ty, Ke, E, mask);
  a.xin = z;
  a.pin = p_old;
  a.pout = p_new;
  a.yout = q;
  a.sc = sc;
  a.part = part_mv;
  a.part_comb = part_comb;
  a.nb_comb = nb_comb;
  a.beta_hist = beta_hist;
  return a;
}

void launch_cg_matvec(const MatvecArgs& a, hipStream_t s) { launch_mv<MV_CG>(a, s); }

void launch_cg_matvec_batch(const MatvecArgs* tab, const int* start, int nent,
                            int total, hipStream_t s) {
  hipLaunchKernelGGL(k_matvec_cg_batch, dim3(total), dim3(MV_NT), 0, s, tab,
                     start, nent);
}

void launch_residual(const Geom& g, int ty, const double* Ke, const double* E,
                     const uint8_t* mask, const double* x, const double* f,
                     double* r, CGScalars* sc, double* part, int slot,
                     hipStream_t s) {
  MatvecArgs a = mv_args(g, ty, Ke, E, mask);
  a.xin = x;
  a.yout = r;
  a.f = f;
  a.sc = sc;
  a.part = part;
  launch_mv<MV_RESID>(a, s);
  hipLaunchKernelGGL(k_resid_finish, dim3(1), dim3(256), 0, s, sc, part,
                     matvec_blocks(g, ty), slot);
}

int update_blocks(long long n) { return (int)((n / 2 + 256 * UP_NPT - 1) / (256 * UP_NPT)); }

UpdateArgs update_args(long long n, double* x, double* r, const double* p,
                       const double* q, CGScalars* sc, double* alpha_hist,
                       double* part_upd, const double* part_mv, int nb_mv,
                       const double* part_comb, int nb_comb) {
  UpdateArgs a{};
  a.n2 = n / 2;
  a.x = x;
  a.r = r;
  a.p = p;
  a.q = q;
  a.sc = sc;
  a.alpha_hist = alpha_hist;
  a.part = part_upd;
  a.part_mv = part_mv;
  a.nb_mv = nb_mv;
  a.part_comb = part_comb;
  a.nb_comb = nb_comb;
  return a;
}

void launch_update(const UpdateArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(update_blocks(2 * a.n2)), dim3(256), 0, s, a);
}

void launch_update_batch(const UpdateArgs* tab, const int* start, int nent,
                         int total, hipStream_t s) {
  hipLaunchKernelGGL(k_update_batch, dim3(total), dim3(256), 0, s, tab, start, nent);
}

// largest grid of the dot product: the partial buffer holds this many
constexpr int kDotMaxBlocks = 1024;
int dot_max_blocks() { return kDotMaxBlocks; }

void launch_dot(long long n, const double* x, const double* y, double* part,
                unsigned int* counter, double* out, hipStream_t s) {
  long long nb = (n + 255) / 256;
  if (nb > kDotMaxBlocks) nb = kDotMaxBlocks;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_dot, dim3((unsigned)nb), dim3(256), 0, s, n, x, y, part,
                     counter, out);
}

}  // namespace msp
