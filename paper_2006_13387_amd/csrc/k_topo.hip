// The topology-optimisation consumer of the state solve (Section 1): the
// gradient of g = lam^T K(rho)^{-1}-weighted energy,
//   dg/drho_e = -p rho_e^(p-1) (E0 - Emin) lam_e^T K^_e u_e
// (lam = u for the compliance f^T u), and one optimality-criteria density
// update rho_e <- clamp(rho_e sqrt(B_e), rho_e -+ move, [0, 1]) with
// B_e = max(0, -dg_e) / Lam, the multiplier Lam bracketed and narrowed on
// the device until the volume sum(rho_new) meets volfrac * nel.
//
// Both are element-parallel and read each element's nodal values once
// (the elements of a row are consecutive threads, so the nodal loads of a
// wave are contiguous); they are bound by HBM bandwidth.
#include "common.h"
#include "dev.h"

namespace msp {

constexpr int TP_NT = 256;

// lam_e^T K^_e u_e of one 2D element (vertex a = ax + 2 ay, DOF 2a + c)
__global__ void __launch_bounds__(TP_NT)
k_sensitivity2d(Geom g, const double* __restrict__ Ke,
                const double* __restrict__ rho, const double* __restrict__ u,
                const double* __restrict__ lam, double scale, double pm1,
                double* __restrict__ out) {
  __shared__ double K[64];
  if (threadIdx.x < 64) K[threadIdx.x] = Ke[threadIdx.x];
  __syncthreads();
  const long long nel = (long long)g.nx * g.ny;
  const long long e = (long long)blockIdx.x * TP_NT + threadIdx.x;
  if (e >= nel) return;
  const int ex = (int)(e % g.nx), ey = (int)(e / g.nx);
  double ue[8], le[8];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const long long node = (long long)(ey + (a >> 1)) * g.nnx + ex + (a & 1);
    const double2 uv = reinterpret_cast<const double2*>(u)[node];
    const double2 lv = reinterpret_cast<const double2*>(lam)[node];
    ue[2 * a] = uv.x;
    ue[2 * a + 1] = uv.y;
    le[2 * a] = lv.x;
    le[2 * a + 1] = lv.y;
  }
  double q = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    double ki = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) ki += K[8 * i + j] * ue[j];
    q += le[i] * ki;
  }
  const double r = rho[e];
  out[e] = -scale * (pm1 == 0.0 ? 1.0 : pow(r, pm1)) * q;
}

// The same for a 3D trilinear element (vertex a = ax + 2 ay + 4 az,
// DOF 3a + c, K^_e 24 x 24 in LDS).
__global__ void __launch_bounds__(TP_NT)
k_sensitivity3d(Geom g, const double* __restrict__ Ke,
                const double* __restrict__ rho, const double* __restrict__ u,
                const double* __restrict__ lam, double scale, double pm1,
                double* __restrict__ out) {
  __shared__ double K[576];
  for (int q = threadIdx.x; q < 576; q += TP_NT) K[q] = Ke[q];
  __syncthreads();
  const long long nel = (long long)g.nx * g.ny * g.nz;
  const long long e = (long long)blockIdx.x * TP_NT + threadIdx.x;
  if (e >= nel) return;
  const int ex = (int)(e % g.nx);
  const long long rr = e / g.nx;
  const int ey = (int)(rr % g.ny), ez = (int)(rr / g.ny);
  double ue[24], le[24];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const long long node = ((long long)(ez + (a >> 2)) * g.nny + ey + ((a >> 1) & 1)) * g.nnx +
                           ex + (a & 1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      ue[3 * a + c] = u[3 * node + c];
      le[3 * a + c] = lam[3 * node + c];
    }
  }
  double q = 0.0;
#pragma unroll
  for (int i = 0; i < 24; ++i) {
    double ki = 0.0;
#pragma unroll
    for (int j = 0; j < 24; ++j) ki += K[24 * i + j] * ue[j];
    q += le[i] * ki;
  }
  const double r = rho[e];
  out[e] = -scale * (pm1 == 0.0 ? 1.0 : pow(r, pm1)) * q;
}

// ---- optimality criteria ------------------------------------------------

constexpr int OC_NC = 32;   // multipliers tried per pass

// State of the multiplier search, in device memory.
struct OcState {
  double lo, hi;            // bracket: volume(lo) > target >= volume(hi)
  double lam;               // the final multiplier
  int phase;                // 0: first pass on a logarithmic grid, 1: narrowing
  int done;
  unsigned int ticket;
};

__device__ __forceinline__ double oc_rho(double r, double dg, double lam, double move) {
  const double B = fmax(0.0, -dg) / lam;
  const double lo = fmax(0.0, r - move), hi = fmin(1.0, r + move);
  return fmin(fmax(r * sqrt(B), lo), hi);
}

// Candidate k of a pass: the first pass tries 2^-80, 2^-75, ..., 2^75;
// later passes split the bracket (lo, hi) into OC_NC + 1 equal parts.
__device__ __forceinline__ double oc_candidate(const OcState& st, int k) {
  if (st.phase == 0) return ldexp(1.0, 5 * k - 80);
  return st.lo + (st.hi - st.lo) * (double)(k + 1) / (double)(OC_NC + 1);
}

// One pass: every workgroup sums the volume of its elements for the
// OC_NC candidates; the last workgroup adds the partials in workgroup
// order and narrows the bracket to the two candidates around the target
// (the volume does not increase with the multiplier).  When the bracket is
// narrower than rel_tol * hi, the multiplier is its midpoint.  Passes after
// that return at once.  The multiplier is confined to [2^-80, 2^75]: if even
// 2^75 leaves the volume above the target, or 2^-80 already at or below it
// (out of reach within the move limits), it is that end of the range.
__global__ void __launch_bounds__(TP_NT)
k_oc_pass(long long nel, const double* __restrict__ rho,
          const double* __restrict__ dg, double move, double target,
          double rel_tol, OcState* __restrict__ st, double* __restrict__ part) {
  __shared__ double red[OC_NC][TP_NT / 64];
  __shared__ double vol[OC_NC];
  __shared__ unsigned int ticket;
  __shared__ OcState s;
  if (threadIdx.x == 0) s = *st;
  __syncthreads();
  if (s.done) return;
  double acc[OC_NC];
#pragma unroll
  for (int k = 0; k < OC_NC; ++k) acc[k] = 0.0;
  for (long long e = (long long)blockIdx.x * TP_NT + threadIdx.x; e < nel;
       e += (long long)gridDim.x * TP_NT) {
    const double r = rho[e], d = dg[e];
#pragma unroll
    for (int k = 0; k < OC_NC; ++k) acc[k] += oc_rho(r, d, oc_candidate(s, k), move);
  }
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < OC_NC; ++k) {
    const double v = wave_sum(acc[k]);
    if ((threadIdx.x & 63) == 0) red[k][w] = v;
  }
  __syncthreads();
  if (threadIdx.x < OC_NC) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < TP_NT / 64; ++i) t += red[threadIdx.x][i];
    part[(long long)blockIdx.x * OC_NC + threadIdx.x] = t;
  }
  if (!last_block(&st->ticket, gridDim.x, &ticket)) return;
  if (threadIdx.x < OC_NC) {
    double t = 0.0;
    for (unsigned int b = 0; b < gridDim.x; ++b)
      t += load_coherent(part + (long long)b * OC_NC + threadIdx.x);
    vol[threadIdx.x] = t;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  OcState n = s;
  n.ticket = 0u;
  int k = 0;
  while (k < OC_NC && vol[k] > target) ++k;
  if (s.phase == 0 && (k == OC_NC || k == 0)) {
    // the target is out of reach within the move limits: the multiplier
    // stops at the end of the range (2^75 above, 2^-80 below)
    n.lam = oc_candidate(s, k == 0 ? 0 : OC_NC - 1);
    n.done = 1;
  } else {
    const double c0 = k > 0 ? oc_candidate(s, k - 1) : s.lo;
    const double c1 = k < OC_NC ? oc_candidate(s, k) : s.hi;
    n.lo = c0;
    n.hi = c1;
    n.phase = 1;
    if (n.hi - n.lo <= rel_tol * n.hi) {
      n.lam = 0.5 * (n.lo + n.hi);
      n.done = 1;
    }
  }
  *st = n;
}

__global__ void __launch_bounds__(TP_NT)
k_oc_apply(long long nel, const double* __restrict__ rho,
           const double* __restrict__ dg, double move,
           const OcState* __restrict__ st, double* __restrict__ out) {
  const long long e = (long long)blockIdx.x * TP_NT + threadIdx.x;
  if (e >= nel) return;
  out[e] = oc_rho(rho[e], dg[e], st->lam, move);
}

__global__ void k_oc_init(OcState* st) {
  OcState s;
  s.lo = 0.0;
  s.hi = 1.0;
  s.lam = 0.0;
  s.phase = 0;
  s.done = 0;
  s.ticket = 0u;
  *st = s;
}

// ---- launchers ----------------------------------------------------------

void launch_sensitivity(const Geom& g, int dim, const double* Ke,
                        const double* rho, const double* u, const double* lam,
                        double scale, double pm1, double* out, hipStream_t s) {
  const long long nel = (long long)g.nx * g.ny * (dim == 3 ? g.nz : 1);
  const unsigned nb = (unsigned)((nel + TP_NT - 1) / TP_NT);
  if (dim == 3)
    hipLaunchKernelGGL(k_sensitivity3d, dim3(nb), dim3(TP_NT), 0, s, g, Ke, rho,
                       u, lam, scale, pm1, out);
  else
    hipLaunchKernelGGL(k_sensitivity2d, dim3(nb), dim3(TP_NT), 0, s, g, Ke, rho,
                       u, lam, scale, pm1, out);
}

size_t oc_state_bytes() { return sizeof(OcState); }
// multiplier and convergence flag of the last search (host copy of the state)
void oc_result(const void* host_state, double* lam, int* done) {
  const OcState* st = static_cast<const OcState*>(host_state);
  *lam = st->lam;
  *done = st->done;
}
int oc_blocks(long long nel) {
  long long nb = (nel + TP_NT - 1) / TP_NT;
  return (int)(nb < 1 ? 1 : (nb > 1024 ? 1024 : nb));
}
int oc_candidates() { return OC_NC; }

// The first pass brackets the multiplier within a factor 32; each later
// pass narrows the bracket 33-fold (nine reach 1e-13).  max_pass bounds
// the passes; oc_done reports whether the search converged.
void launch_oc(long long nel, const double* rho, const double* dg, double move,
               double target, double rel_tol, void* state, double* part,
               int max_pass, double* out, hipStream_t s) {
  OcState* st = static_cast<OcState*>(state);
  hipLaunchKernelGGL(k_oc_init, dim3(1), dim3(1), 0, s, st);
  const int nb = oc_blocks(nel);
  for (int i = 0; i < max_pass; ++i)
    hipLaunchKernelGGL(k_oc_pass, dim3(nb), dim3(TP_NT), 0, s, nel, rho, dg,
                       move, target, rel_tol, st, part);
  const unsigned na = (unsigned)((nel + TP_NT - 1) / TP_NT);
  hipLaunchKernelGGL(k_oc_apply, dim3(na), dim3(TP_NT), 0, s, nel, rho, dg,
                     move, st, out);
}

}  // namespace msp
