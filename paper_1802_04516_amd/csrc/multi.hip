// Restarted GMRES for several independent systems sharing every launch.
//
// The systems are contiguous segments [off_s, off_{s+1}) of one long vector:
// the columns of a batched solve (several right-hand sides on one mesh,
// stored column after column) or the meshes of a ragged batch (one
// concatenated mesh whose element ranges are the meshes).  Each system has
// its own Arnoldi process, Hessenberg matrix, Givens rotations, tolerance and
// convergence flag; the operator and preconditioner are applied to all
// segments in one launch, and every reduction is segmented: each reduction
// block covers rows of a single system, and the per-system sums are formed
// in a fixed order by a finalize kernel, so results are deterministic and a
// system's iterates do not depend on the others.
//
// A system whose residual estimate reaches its tolerance is switched off on
// the device (its Gram-Schmidt work is skipped); its correction is applied at
// the end of the cycle with the Arnoldi steps it took.  The host polls the
// device count of active systems every check_every iterations.  By default
// the Arnoldi steps delay each vector's second projection to the next step
// (as the single-system solver); with SDG_SOLVE_CGS2 both projections run
// within the step.
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <functional>

#include "context.hpp"
#include "reduce.hpp"

namespace sdg {

namespace {

constexpr int kT = 256;

__device__ inline double wsum64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

template <int NJ>
__device__ inline void block_partials_m(const double (&acc)[NJ], double* sh, double* partials, int nblocks) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    const double v = wsum64(acc[i]);
    if (lane == 0) sh[wid * NJ + i] = v;
  }
  __syncthreads();
  if (threadIdx.x < NJ) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sh[w * NJ + threadIdx.x];
    partials[(size_t)threadIdx.x * nblocks + blockIdx.x] = s;
  }
}

struct BlockMap {
  const int* seg;        // block -> system
  const int64_t* beg;    // first row of the block
  const int64_t* end;    // one past the last row
  int nblocks;
};

// h1[s][i] partials: V_i . w over the block's rows (i < NJ); all = 1 also
// covers inactive systems
template <int NJ>
__global__ __launch_bounds__(kT) void km_multidot(BlockMap bm, int64_t ld, const double* __restrict__ V,
                                                  const double* __restrict__ w, const SysScalars* ss,
                                                  double* partials, int all) {
  __shared__ double sh[4 * NJ];
  const int sys = bm.seg[blockIdx.x];
  if (!all && !ss[sys].active) return;
  double acc[NJ];
#pragma unroll
  for (int i = 0; i < NJ; ++i) acc[i] = 0.0;
  const int64_t e = bm.end[blockIdx.x];
  for (int64_t t = bm.beg[blockIdx.x] + threadIdx.x; t < e; t += kT) {
    const double wt = w[t];
    double vi[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) vi[i] = V[(size_t)i * ld + t];
#pragma unroll
    for (int i = 0; i < NJ; ++i) acc[i] += vi[i] * wt;
  }
  block_partials_m<NJ>(acc, sh, partials, bm.nblocks);
}

// w -= V h1[s]; partials of h2 = V . w
template <int NJ>
__global__ __launch_bounds__(kT) void km_cgs_pass(BlockMap bm, int64_t ld, const double* __restrict__ V,
                                                  double* __restrict__ w, const SysScalars* ss, double* partials) {
  __shared__ double sh[4 * NJ];
  const int sys = bm.seg[blockIdx.x];
  if (!ss[sys].active) return;
  double h[NJ], acc[NJ];
#pragma unroll
  for (int i = 0; i < NJ; ++i) { h[i] = ss[sys].h1[i]; acc[i] = 0.0; }
  const int64_t e = bm.end[blockIdx.x];
  for (int64_t t = bm.beg[blockIdx.x] + threadIdx.x; t < e; t += kT) {
    double vi[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) vi[i] = V[(size_t)i * ld + t];
    double wt = w[t];
#pragma unroll
    for (int i = 0; i < NJ; ++i) wt -= h[i] * vi[i];
    w[t] = wt;
#pragma unroll
    for (int i = 0; i < NJ; ++i) acc[i] += vi[i] * wt;
  }
  block_partials_m<NJ>(acc, sh, partials, bm.nblocks);
}

// w -= V h2[s]; partials of w . w
template <int NJ>
__global__ __launch_bounds__(kT) void km_cgs_final(BlockMap bm, int64_t ld, const double* __restrict__ V,
                                                   double* __restrict__ w, const SysScalars* ss, double* partials) {
  __shared__ double sh[4];
  const int sys = bm.seg[blockIdx.x];
  if (!ss[sys].active) return;
  double h[NJ];
#pragma unroll
  for (int i = 0; i < NJ; ++i) h[i] = ss[sys].h2[i];
  double acc[1] = {0.0};
  const int64_t e = bm.end[blockIdx.x];
  for (int64_t t = bm.beg[blockIdx.x] + threadIdx.x; t < e; t += kT) {
    double vi[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) vi[i] = V[(size_t)i * ld + t];
    double wt = w[t];
#pragma unroll
    for (int i = 0; i < NJ; ++i) wt -= h[i] * vi[i];
    w[t] = wt;
    acc[0] += wt * wt;
  }
  block_partials_m<1>(acc, sh, partials, bm.nblocks);
}

// x += sum_{i < k_s} y[s][i] V_i (y beyond k_s is zero)
template <int NJ>
__global__ __launch_bounds__(kT) void km_update(BlockMap bm, int64_t ld, const double* __restrict__ V,
                                                double* __restrict__ x, const SysScalars* ss) {
  const int sys = bm.seg[blockIdx.x];
  // a system that stopped after k < NJ steps never wrote V[k+1 ..): only its
  // own k columns are read (a zero coefficient times a stale NaN is NaN)
  const int k = ss[sys].k;
  if (k == 0) return;
  double ys[NJ];
#pragma unroll
  for (int i = 0; i < NJ; ++i) ys[i] = ss[sys].y[i];
  const int64_t e = bm.end[blockIdx.x];
  for (int64_t t = bm.beg[blockIdx.x] + threadIdx.x; t < e; t += kT) {
    double vi[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) vi[i] = i < k ? V[(size_t)i * ld + t] : 0.0;
    double acc = x[t];
#pragma unroll
    for (int i = 0; i < NJ; ++i)
      if (i < k) acc += ys[i] * vi[i];
    x[t] = acc;
  }
}

// v = w * inv_norm[s] on the rows of active systems
__global__ __launch_bounds__(kT) void km_scale(BlockMap bm, const double* __restrict__ w, double* __restrict__ v,
                                               const SysScalars* ss, int only_active) {
  const int sys = bm.seg[blockIdx.x];
  if (only_active && !ss[sys].active) return;
  const double sc = ss[sys].inv_norm;
  const int64_t e = bm.end[blockIdx.x];
  for (int64_t t = bm.beg[blockIdx.x] + threadIdx.x; t < e; t += kT) v[t] = w[t] * sc;
}

// x = 0 on the rows of systems with a zero right-hand side
__global__ __launch_bounds__(kT) void km_zero_null(BlockMap bm, double* __restrict__ x, const SysScalars* ss) {
  const int sys = bm.seg[blockIdx.x];
  if (ss[sys].bnorm != 0.0) return;
  const int64_t e = bm.end[blockIdx.x];
  for (int64_t t = bm.beg[blockIdx.x] + threadIdx.x; t < e; t += kT) x[t] = 0.0;
}

// Per-system sums of partials[i][blocks of s] for i < nslots; one wavefront
// per (system, slot).  dst selects the field written.
enum Dst { kH1 = 0, kH2 = 1, kDot = 2 };
__global__ void km_finalize(const double* partials, int nblocks, const int* seg_blk0, int S, int nslots,
                            SysScalars* ss, int dst, int all) {
  const int lane = threadIdx.x & 63;
  const int wv = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (wv >= S * nslots) return;
  const int s = wv / nslots, i = wv % nslots;
  if (!all && !ss[s].active) return;
  const int b0 = seg_blk0[s], b1 = seg_blk0[s + 1];
  double v = 0.0;
  for (int b = b0 + lane; b < b1; b += 64) v += partials[(size_t)i * nblocks + b];
  v = wsum64(v);
  if (lane == 0) {
    if (dst == kH1) ss[s].h1[i] = v;
    else if (dst == kH2) ss[s].h2[i] = v;
    else ss[s].dot = v;
  }
}

// Block-wide count of flags (one block of up to 1024 threads).
__device__ inline int block_count(int flag, int* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  int v = flag;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  int r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < nw; ++i) r += sh[i];
  return r;
}

// Norm of w per system, Hessenberg column j, Givens rotations, residual
// estimate, convergence flag.  One workgroup of 1024 threads: wavefront w
// handles systems w, w+16, ...; its lanes add the system's block partials
// (fixed order), lane 0 updates the system's scalars; then the workgroup
// counts the active systems.
__global__ __launch_bounds__(1024) void km_arnoldi_fin(const double* partials, int nblocks, const int* seg_blk0,
                                                       int S, int j, SysScalars* ss, int* nactive) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  // per wavefront: the system's Hessenberg column and rotations in LDS
  __shared__ double hcs[16][kMaxRestart + 1], css[16][kMaxRestart], sns[16][kMaxRestart];
  double* hc = hcs[wv];
  double* cs = css[wv];
  double* sn = sns[wv];
  for (int s = wv; s < S; s += nw) {
    if (!ss[s].active) continue;
    SysScalars& q = ss[s];
    double v = 0.0;
    for (int b = seg_blk0[s] + lane; b < seg_blk0[s + 1]; b += 64) v += partials[b];
    const double tot = wsum64(v);
    if (lane <= j) hc[lane] = q.h1[lane] + q.h2[lane];
    if (lane < j) { cs[lane] = q.cs[lane]; sn[lane] = q.sn[lane]; }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (lane == 0) {
      const double nrm = sqrt(tot);
      hc[j + 1] = nrm;
      q.norm = nrm;
      q.inv_norm = nrm > 0.0 ? 1.0 / nrm : 0.0;
      for (int i = 0; i < j; ++i) {
        const double a = hc[i], b = hc[i + 1];
        hc[i] = cs[i] * a + sn[i] * b;
        hc[i + 1] = -sn[i] * a + cs[i] * b;
      }
      const double a = hc[j], b = hc[j + 1];
      const double rad = hypot(a, b);
      const double c = rad > 0.0 ? a / rad : 1.0, sg = rad > 0.0 ? b / rad : 0.0;
      q.cs[j] = c;
      q.sn[j] = sg;
      hc[j] = rad;
      hc[j + 1] = 0.0;
      const double gj = q.g[j];
      q.g[j] = c * gj;
      q.g[j + 1] = -sg * gj;
      q.resid = fabs(q.g[j + 1]);
      q.k = j + 1;
      if (q.resid <= q.tol_abs || nrm == 0.0) q.active = 0;
      atomicAdd(&cnt, q.active);  // integer count in LDS: order-independent
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    double* Hc = q.H + (size_t)j * (kMaxRestart + 1);
    if (lane <= j + 1) Hc[lane] = hc[lane];
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  if (threadIdx.x == 0) *nactive = cnt;
}

// Start of a cycle from the per-system r.r in ss.dot.
__global__ void km_cycle_start(int S, SysScalars* ss, int* nactive) {
  __shared__ int sh[16];
  const int s = threadIdx.x;
  int act = 0;
  if (s < S) {
    SysScalars& q = ss[s];
    const double beta = sqrt(q.dot);
    q.rnorm = beta;
    for (int i = 0; i <= kMaxRestart; ++i) q.g[i] = 0.0;
    for (int i = 0; i < kMaxRestart; ++i) q.y[i] = 0.0;
    q.g[0] = beta;
    q.norm = beta;
    q.inv_norm = beta > 0.0 ? 1.0 / beta : 0.0;
    q.resid = beta;
    q.k = 0;
    q.active = (beta > q.tol_abs) ? 1 : 0;
    act = q.active;
  }
  const int n = block_count(act, sh);
  if (threadIdx.x == 0) *nactive = n;
}

// Outer ||b_s|| of iterative refinement from ss.dot = b.b.
__global__ void km_outer_bnorm(int S, const SysScalars* ss, double* outer) {
  const int s = threadIdx.x;
  if (s < S) outer[s] = sqrt(ss[s].dot);
}

// Outer test of iterative refinement from ss.dot = d.d (d = b - A x): the
// relative residual per system (outer[S + s]), the number of systems above
// rtol, and the targets of the next inner solve A e = d:
// max(inner_rtol ||d_s||, rtol ||b_s|| / 2), or +inf for a converged system,
// which km_cycle_start then leaves inactive (its correction stays zero).
__global__ void km_refine_check(int S, SysScalars* ss, double* outer, double rtol, double inner_rtol,
                                int* nouter) {
  __shared__ int sh[16];
  const int s = threadIdx.x;
  int act = 0;
  if (s < S) {
    SysScalars& q = ss[s];
    const double dn = sqrt(q.dot), bn = outer[s];
    const double rr = bn > 0.0 ? dn / bn : dn;
    outer[S + s] = rr;
    act = rr <= rtol ? 0 : 1;   // a NaN residual stays active (and is reported)
    q.bnorm = dn;
    // the inner solve reduces d by inner_rtol, or only to half of what is
    // left to rtol when that is looser (the last sweep does not over-solve)
    q.tol_abs = act ? fmax(inner_rtol * dn, 0.5 * rtol * (bn > 0.0 ? bn : 1.0)) : INFINITY;
    q.active = 1;
    q.k = 0;
  }
  const int n = block_count(act, sh);
  if (threadIdx.x == 0) *nouter = n;
}

// bnorm and tolerance per system from ss.dot = b.b
__global__ void km_set_tol(int S, SysScalars* ss, double rtol) {
  const int s = threadIdx.x;
  if (s < S) {
    ss[s].bnorm = sqrt(ss[s].dot);
    ss[s].tol_abs = rtol * ss[s].bnorm;
    ss[s].active = 1;
    ss[s].k = 0;
  }
}

// Back substitution R y = g per system with its k.
// Per system y = R^-1 g (R: the k x k upper triangle of its rotated
// Hessenberg matrix), one wavefront per system: lane l holds row l of R and
// the running right-hand side; column by column from the last, y_i is
// broadcast and the lanes above subtract R_li y_i.
__global__ __launch_bounds__(256) void km_trisolve(int S, SysScalars* ss) {
  const int s = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6), l = threadIdx.x & 63;
  if (s >= S) return;
  SysScalars& q = ss[s];
  constexpr int ld = kMaxRestart + 1;
  const int k = q.k;
  double hrow[kMaxRestart];
#pragma unroll
  for (int i = 0; i < kMaxRestart; ++i) hrow[i] = (l < k && i < k) ? q.H[(size_t)i * ld + l] : 0.0;
  double r = l < k ? q.g[l] : 0.0, y = 0.0;
#pragma unroll
  for (int i = kMaxRestart - 1; i >= 0; --i) {
    if (i < k) {
      const double ri = __shfl(r, i, 64);
      const double d = __shfl(hrow[i], i, 64);
      const double yi = d != 0.0 ? ri / d : 0.0;
      if (l == i) y = yi;
      if (l < i) r -= hrow[i] * yi;
    }
  }
  if (l < kMaxRestart) q.y[l] = y;
}

// ---- Delayed reorthogonalisation for every system (the scheme of the
// single-system solver: one segmented reduction and two sweeps per step).

// Slots [0, NJ) = Q^T u, [NJ, 2NJ) = Q^T z, 2NJ = u.u, 2NJ+1 = u.z per block
// of an active system, Q = V[0..NJ), u = V[NJ].  Block 0 also clears the
// count of active systems that the following finalize forms.
template <int NJ>
__global__ __launch_bounds__(kT) void km_dmultidot(BlockMap bm, int64_t ld, const double* __restrict__ V,
                                                   const double* __restrict__ z, const SysScalars* ss,
                                                   double* partials, int* nactive) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *nactive = 0;
  const int sys = bm.seg[blockIdx.x];
  if (!ss[sys].active) return;
  constexpr int NS = 2 * NJ + 2;
  double acc[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) acc[i] = 0.0;
  const double* __restrict__ u = V + (size_t)NJ * ld;
  const int64_t e = bm.end[blockIdx.x];
  for (int64_t t = bm.beg[blockIdx.x] + threadIdx.x; t < e; t += kT) {
    const double ut = u[t], zt = z[t];
    double vi[NJ > 0 ? NJ : 1];
#pragma unroll
    for (int i = 0; i < NJ; ++i) vi[i] = V[(size_t)i * ld + t];
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
      acc[i] += vi[i] * ut;
      acc[NJ + i] += vi[i] * zt;
    }
    acc[2 * NJ] += ut * ut;
    acc[2 * NJ + 1] += ut * zt;
  }
  block_partials_to<NS>(acc, partials, bm.nblocks);
}

// Finalize of step NJ, one workgroup per active system: its four
// wavefronts add the system's block partials of every slot (thread = block,
// then a butterfly reduce-scatter over the slots per wavefront and the
// wavefronts' sums in wave order), then wavefront 0 forms nu, Hessenberg
// column NJ-1 (unrotated and rotated), its Givens rotation, g, the residual
// estimate and k = NJ; with HZ also a_NJ, b, f, e, 1/nu, the convergence flag
// and the count of active systems; without (the completion of a cycle's
// last column, slots [0, NJ) = Q^T u and NJ = u.u) only the column.
template <int NJ, bool HZ>
__global__ __launch_bounds__(kT) void km_dfin(const double* partials, int nblocks, const int* seg_blk0, int S,
                                              SysScalars* ss, int* nactive) {
  constexpr int NS = HZ ? 2 * NJ + 2 : NJ + 1, IA = HZ ? 2 * NJ : NJ, ld = kMaxRestart + 1;
  constexpr int NC = NJ > 0 ? NJ : 1, NSP = pow2ceil(NS);
  __shared__ double sw[kT / 64][NSP];
  __shared__ double sv[NS];
  __shared__ double sHu[(NJ + 1) * NC];
  __shared__ double sHb[NJ + 1];
  __shared__ double scx[4];
  __shared__ double sa[NC], scs[NC], ssn[NC], sgj;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int s = blockIdx.x;
  if (s >= S || !ss[s].active) return;  // uniform over the workgroup
  SysScalars& q = ss[s];
  for (int i = threadIdx.x; i < (NJ + 1) * NJ; i += kT) {
    const int col = i / (NJ + 1), row = i % (NJ + 1);
    sHu[i] = col + 1 < NJ && row <= col + 1 ? q.Hu[(size_t)col * ld + row] : 0.0;
  }
  // what the serial part reads, staged with parallel loads
  if (threadIdx.x < NJ) {
    sa[threadIdx.x] = q.h1[threadIdx.x];
    if (threadIdx.x + 1 < NJ) {
      scs[threadIdx.x] = q.cs[threadIdx.x];
      ssn[threadIdx.x] = q.sn[threadIdx.x];
    }
  }
  if (NJ > 0 && threadIdx.x == 64) sgj = q.g[NJ > 0 ? NJ - 1 : 0];
  {
    double acc[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) acc[i] = 0.0;
    const int b0 = seg_blk0[s], nb = seg_blk0[s + 1] - b0;
    for (int b = threadIdx.x; b < nb; b += kT) {
#pragma unroll
      for (int i = 0; i < NS; ++i) acc[i] += partials[(size_t)i * nblocks + b0 + b];
    }
    int slot;
    bool first;
    const double v = wave_reduce_scatter<NS>(acc, lane, slot, first);
    if (first) sw[wv][slot] = v;
  }
  __syncthreads();
  if (threadIdx.x < NS) {
    double t = 0.0;
    for (int w = 0; w < kT / 64; ++w) t += sw[w][threadIdx.x];
    sv[threadIdx.x] = t;
  }
  __syncthreads();
  if (wv != 0) return;
  if (lane == 0) {
    double bb = 0.0;
    for (int i = 0; i < NJ; ++i) bb += sv[i] * sv[i];
    const double nu2 = sv[IA] - bb;
    const double nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
    const double inv = nu > 0.0 ? 1.0 / nu : 0.0;
    scx[0] = nu;
    scx[1] = inv;
    q.norm = nu;
    if (NJ == 0) {
      q.g[0] = nu;
      q.resid = nu;
    } else {
      double hc[NJ + 1];
      for (int i = 0; i < NJ; ++i) hc[i] = sa[i] + sv[i];
      hc[NJ] = nu;
      for (int i = 0; i <= NJ; ++i) sHu[(NJ - 1) * (NJ + 1) + i] = hc[i];
      for (int i = 0; i + 1 < NJ; ++i) {
        const double a = hc[i], b = hc[i + 1];
        hc[i] = scs[i] * a + ssn[i] * b;
        hc[i + 1] = -ssn[i] * a + scs[i] * b;
      }
      const double a = hc[NJ - 1], b = hc[NJ];
      const double rad = hypot(a, b);
      const double cr = rad > 0.0 ? a / rad : 1.0, sr = rad > 0.0 ? b / rad : 0.0;
      q.cs[NJ - 1] = cr;
      q.sn[NJ - 1] = sr;
      hc[NJ - 1] = rad;
      hc[NJ] = 0.0;
      double* Hc = q.H + (size_t)(NJ - 1) * ld;
      for (int i = 0; i <= NJ; ++i) Hc[i] = hc[i];
      q.g[NJ - 1] = cr * sgj;
      q.g[NJ] = -sr * sgj;
      q.resid = fabs(sr * sgj);
    }
    q.k = NJ;
    if (HZ && NJ > 0 && (q.resid <= q.tol_abs || nu == 0.0)) q.active = 0;
    if (HZ) atomicAdd(nactive, q.active);  // integer count: order-independent
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (NJ > 0 && lane <= NJ) q.Hu[(size_t)(NJ - 1) * ld + lane] = sHu[(NJ - 1) * (NJ + 1) + lane];
  if (!HZ) return;
  if (lane <= NJ) {
    double acc = 0.0;
    for (int i = 0; i < NJ; ++i) acc += sHu[i * (NJ + 1) + lane] * sv[i];  // zero below the subdiagonal
    sHb[lane] = acc;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const double inv = scx[1];
  double e = 0.0;
  if (lane == 0) {
    double bc = 0.0;
    for (int i = 0; i < NJ; ++i) bc += sv[i] * sv[NJ + i];
    const double aj = ((sv[2 * NJ + 1] - bc) * inv - sHb[NJ]) * inv;
    const double dj = sHb[NJ] * inv + aj;
    e = dj * inv;
    q.h1[NJ] = aj;
    q.e = e;
    q.inv_norm = inv;
  }
  e = __shfl(e, 0, 64);
  if (lane < NJ) {
    const double ai = (sv[NJ + lane] - sHb[lane]) * inv;
    const double di = sHb[lane] * inv + ai;
    q.h1[lane] = ai;
    q.h2[lane] = sv[lane];
    q.f[lane] = di - e * sv[lane];
  }
}

// Update sweep of step NJ for the active systems: q_NJ = (u - Q b) / nu
// over slot NJ, u_{NJ+1} = z / nu - e u - Q f into slot NJ+1; with DOTS the
// partials of the completion of column NJ (q_i . u_{NJ+1}, i <= NJ, and
// u_{NJ+1} . u_{NJ+1}).
template <int NJ, bool DOTS>
__global__ __launch_bounds__(kT) void km_dupdate(BlockMap bm, int64_t ld, double* V, const double* __restrict__ z,
                                                 const SysScalars* ss, double* partials) {
  const int sys = bm.seg[blockIdx.x];
  if (!ss[sys].active) return;
  const SysScalars& q = ss[sys];
  double bq[NJ > 0 ? NJ : 1], fq[NJ > 0 ? NJ : 1];
#pragma unroll
  for (int i = 0; i < NJ; ++i) { bq[i] = q.h2[i]; fq[i] = q.f[i]; }
  const double inv = q.inv_norm, e = q.e;
  const double* __restrict__ Q = V;
  double* __restrict__ u = V + (size_t)NJ * ld;
  double* __restrict__ un = V + (size_t)(NJ + 1) * ld;
  double acc[DOTS ? NJ + 2 : 1];
#pragma unroll
  for (int i = 0; i < (DOTS ? NJ + 2 : 1); ++i) acc[i] = 0.0;
  const int64_t end = bm.end[blockIdx.x];
  for (int64_t t = bm.beg[blockIdx.x] + threadIdx.x; t < end; t += kT) {
    double vi[NJ > 0 ? NJ : 1];
#pragma unroll
    for (int i = 0; i < NJ; ++i) vi[i] = Q[(size_t)i * ld + t];
    const double ut = u[t];
    double qv = ut, w = z[t] * inv - e * ut;
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
      qv -= bq[i] * vi[i];
      w -= fq[i] * vi[i];
    }
    qv *= inv;
    u[t] = qv;
    un[t] = w;
    if constexpr (DOTS) {
#pragma unroll
      for (int i = 0; i < NJ; ++i) acc[i] += vi[i] * w;
      acc[NJ] += qv * w;
      acc[NJ + 1] += w * w;
    }
  }
  if constexpr (DOTS) block_partials_to<NJ + 2>(acc, partials, bm.nblocks);
}

#define SDG_MNJ0_CASES(X)                                                                                       \
  X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) \
  X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)

enum class Dm { Multidot, Fin, FinU, Update, UpdateDots };

void launch_dm(Dm op, int nj, const MultiSys& m, const BlockMap& bm, hipStream_t s, double* V, const double* z) {
  require(nj < kMaxRestart || op == Dm::FinU, SDG_EINVAL, "Gram-Schmidt basis size out of range");
  const unsigned g = (unsigned)bm.nblocks;
  const unsigned gs = (unsigned)m.S;
  const int64_t ld = m.n_total;
  SysScalars* ss = m.d_ss.p;
  double* pt = m.d_partials.p;
  switch (nj) {
#define SDG_DM_Z(N) (N < kMaxRestart ? N : kMaxRestart - 1)
#define SDG_DM_CASE(N)                                                                                            \
  case N:                                                                                                         \
    if (op == Dm::Multidot) km_dmultidot<SDG_DM_Z(N)><<<g, kT, 0, s>>>(bm, ld, V, z, ss, pt, m.d_nactive.p);     \
    else if (op == Dm::Fin)                                                                                       \
      km_dfin<SDG_DM_Z(N), true><<<gs, kT, 0, s>>>(pt, bm.nblocks, m.d_seg_blk0.p, m.S, ss, m.d_nactive.p);       \
    else if (op == Dm::FinU)                                                                                      \
      km_dfin<N, false><<<gs, kT, 0, s>>>(pt, bm.nblocks, m.d_seg_blk0.p, m.S, ss, m.d_nactive.p);               \
    else if (op == Dm::UpdateDots) km_dupdate<SDG_DM_Z(N), true><<<g, kT, 0, s>>>(bm, ld, V, z, ss, pt);           \
    else km_dupdate<SDG_DM_Z(N), false><<<g, kT, 0, s>>>(bm, ld, V, z, ss, pt);                                 \
    break;
    SDG_MNJ0_CASES(SDG_DM_CASE)
#undef SDG_DM_CASE
#undef SDG_DM_Z
    default:
      throw Error(SDG_EINVAL, "Gram-Schmidt basis size out of range");
  }
  SDG_HIP(hipGetLastError());
}

#define SDG_MNJ_CASES(X)                                                                                   \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) \
  X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)

enum class Op { Multidot, Pass, Final, Update };

void launch_m(Op op, int nj, const BlockMap& bm, hipStream_t s, int64_t ld, const double* V, double* w,
              SysScalars* ss, double* partials) {
  const unsigned g = (unsigned)bm.nblocks;
  switch (nj) {
#define SDG_M_CASE(N)                                                                          \
  case N:                                                                                      \
    if (op == Op::Multidot) km_multidot<N><<<g, kT, 0, s>>>(bm, ld, V, w, ss, partials, 0);     \
    else if (op == Op::Pass) km_cgs_pass<N><<<g, kT, 0, s>>>(bm, ld, V, w, ss, partials);       \
    else if (op == Op::Final) km_cgs_final<N><<<g, kT, 0, s>>>(bm, ld, V, w, ss, partials);     \
    else km_update<N><<<g, kT, 0, s>>>(bm, ld, V, w, ss);                                       \
    break;
    SDG_MNJ_CASES(SDG_M_CASE)
#undef SDG_M_CASE
    default:
      throw Error(SDG_EINVAL, "Gram-Schmidt basis size out of range");
  }
  SDG_HIP(hipGetLastError());
}

BlockMap map_of(const MultiSys& m) {
  return BlockMap{m.d_blk_seg.p, m.d_blk_beg.p, m.d_blk_end.p, m.n_blocks};
}

void finalize(const MultiSys& m, int nslots, int dst, int all, hipStream_t s) {
  const int waves = m.S * nslots;
  const unsigned blocks = (unsigned)((waves * 64 + kT - 1) / kT);
  km_finalize<<<blocks, kT, 0, s>>>(m.d_partials.p, m.n_blocks, m.d_seg_blk0.p, m.S, nslots, m.d_ss.p, dst, all);
  SDG_HIP(hipGetLastError());
}

// per-system x . x into ss.dot (all systems)
void seg_norm2(const MultiSys& m, const double* x, hipStream_t s) {
  km_multidot<1><<<(unsigned)m.n_blocks, kT, 0, s>>>(map_of(m), m.n_total, x, x, m.d_ss.p, m.d_partials.p, 1);
  SDG_HIP(hipGetLastError());
  finalize(m, 1, kDot, 1, s);
}

unsigned sys_threads(int S) { return (unsigned)std::max(64, ((S + 63) / 64) * 64); }

int read_int(int* dev, int* pinned, hipStream_t s) {
  SDG_HIP(hipMemcpyAsync(pinned, dev, sizeof(int), hipMemcpyDeviceToHost, s));
  SDG_HIP(hipStreamSynchronize(s));
  return *pinned;
}

}  // namespace

const int* MultiSys::active_flags() const {
  return reinterpret_cast<const int*>(reinterpret_cast<const char*>(d_ss.p) + offsetof(SysScalars, active));
}
int MultiSys::mask_stride() {
  static_assert(sizeof(SysScalars) % sizeof(int) == 0, "system records must tile ints");
  return (int)(sizeof(SysScalars) / sizeof(int));
}

void MultiSys::build(const std::vector<int64_t>& offsets) {
  require(offsets.size() >= 2, SDG_EINVAL, "at least one system");
  S = (int)offsets.size() - 1;
  require(S <= kMaxSystems, SDG_EUNSUPPORTED, "too many independent systems in one solve");
  off = offsets;
  n_total = off[S];
  const int64_t rpb = std::max<int64_t>(4 * kT, (n_total + 2047) / 2048);
  std::vector<int> seg, blk0(S + 1);
  std::vector<int64_t> beg, end;
  for (int q = 0; q < S; ++q) {
    blk0[q] = (int)seg.size();
    const int64_t len = off[q + 1] - off[q];
    require(len >= 0, SDG_EINVAL, "system offsets must be non-decreasing");
    const int64_t nb = std::max<int64_t>(1, (len + rpb - 1) / rpb);
    for (int64_t b = 0; b < nb; ++b) {
      seg.push_back(q);
      beg.push_back(off[q] + std::min(len, b * rpb));
      end.push_back(off[q] + std::min(len, (b + 1) * rpb));
    }
  }
  blk0[S] = (int)seg.size();
  n_blocks = (int)seg.size();
  d_blk_seg.alloc(seg.size());
  SDG_HIP(hipMemcpy(d_blk_seg.p, seg.data(), seg.size() * sizeof(int), hipMemcpyHostToDevice));
  d_seg_blk0.alloc(blk0.size());
  SDG_HIP(hipMemcpy(d_seg_blk0.p, blk0.data(), blk0.size() * sizeof(int), hipMemcpyHostToDevice));
  d_blk_beg.alloc(beg.size());
  SDG_HIP(hipMemcpy(d_blk_beg.p, beg.data(), beg.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  d_blk_end.alloc(end.size());
  SDG_HIP(hipMemcpy(d_blk_end.p, end.data(), end.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  d_ss.alloc(S);
  SDG_HIP(hipMemset(d_ss.p, 0, S * sizeof(SysScalars)));
  d_partials.alloc((size_t)(2 * kMaxRestart + 2) * n_blocks);
  d_nactive.alloc(1);
  d_outer.alloc(2 * (size_t)S);
  d_nouter.alloc(1);
  if (!h_pinned) SDG_HIP(hipHostMalloc((void**)&h_pinned, 16 * sizeof(int), hipHostMallocDefault));
}

MultiSys::~MultiSys() {
  if (h_pinned) (void)hipHostFree(h_pinned);
}

void MultiSys::read_scalars(std::vector<SysScalars>& out, hipStream_t s) const {
  out.resize(S);
  SDG_HIP(hipMemcpyAsync(out.data(), d_ss.p, S * sizeof(SysScalars), hipMemcpyDeviceToHost, s));
  SDG_HIP(hipStreamSynchronize(s));
}

double multi_rel_residual(MultiSys& m, const double* b, const double* r, hipStream_t s, double* bnorm_max) {
  std::vector<SysScalars> h;
  seg_norm2(m, b, s);
  m.read_scalars(h, s);
  std::vector<double> bn(m.S);
  for (int q = 0; q < m.S; ++q) bn[q] = std::sqrt(h[q].dot);
  seg_norm2(m, r, s);
  m.read_scalars(h, s);
  double worst = 0.0, bmax = 0.0;
  for (int q = 0; q < m.S; ++q) {
    const double rn = std::sqrt(h[q].dot);
    worst = std::max(worst, bn[q] > 0.0 ? rn / bn[q] : rn);
    bmax = std::max(bmax, bn[q]);
  }
  if (bnorm_max) *bnorm_max = bmax;
  return worst;
}

void multi_setup(MultiSys& m, const double* b, double* x, double rtol, hipStream_t s) {
  seg_norm2(m, b, s);
  km_set_tol<<<1, sys_threads(m.S), 0, s>>>(m.S, m.d_ss.p, rtol);
  km_zero_null<<<(unsigned)m.n_blocks, kT, 0, s>>>(map_of(m), x, m.d_ss.p);
  SDG_HIP(hipGetLastError());
}

void multi_residual(MultiSys& m, const double* b, const double* x, hipStream_t s,
                    const MultiOp& op, double* r) {
  op(x, r, false);
  vec_axpby(m.n_total, 1.0, b, -1.0, r, s);
  seg_norm2(m, r, s);
  km_cycle_start<<<1, sys_threads(m.S), 0, s>>>(m.S, m.d_ss.p, m.d_nactive.p);
  SDG_HIP(hipGetLastError());
}

// One restart cycle with delayed reorthogonalisation for every system.  The
// residual r = b - A x goes straight into slot 0 of V as the first,
// unnormalised basis vector; step j completes each system's Hessenberg
// column j-1 and switches systems whose estimate has converged off; the last
// step's update sweep forms the dots that complete the last column.
static int multi_cycle_delayed(MultiSys& m, const double* b, double* x, const KrylovCfg& k, hipStream_t s,
                               const MultiOp& op,
                               const std::function<void(const double*, double*)>* pre, double* V, double* w,
                               double* t, bool poll, int max_steps, int* matvecs, bool* all_converged) {
  const int64_t n = m.n_total;
  const BlockMap bm = map_of(m);
  SysScalars* ss = m.d_ss.p;
  const int check_every = std::max(1, k.check_every);
  *all_converged = false;
  multi_residual(m, b, x, s, op, V);
  ++*matvecs;
  if (poll) {
    if (read_int(m.d_nactive.p, m.h_pinned, s) == 0) {
      *all_converged = true;
      return 0;
    }
    if (max_steps <= 0) return 0;
  }
  const int steps = std::min(k.restart, max_steps);
  int j = 0;
  bool done = false;
  for (; j < steps; ++j) {
    double* vj = V + (size_t)j * n;
    if (pre) {
      (*pre)(vj, t);
      op(t, w, true);
    } else {
      op(vj, w, true);
    }
    ++*matvecs;
    const bool last = j + 1 == steps;
    launch_dm(Dm::Multidot, j, m, bm, s, V, w);
    launch_dm(Dm::Fin, j, m, bm, s, V, w);
    launch_dm(last ? Dm::UpdateDots : Dm::Update, j, m, bm, s, V, w);
    if (poll && !last && (j + 1) % check_every == 0) {
      if (read_int(m.d_nactive.p, m.h_pinned, s) == 0) {
        done = true;
        ++j;
        break;
      }
    }
  }
  if (!done) launch_dm(Dm::FinU, j, m, bm, s, V, nullptr);
  km_trisolve<<<(unsigned)((m.S * 64 + 255) / 256), 256, 0, s>>>(m.S, ss);
  SDG_HIP(hipGetLastError());
  if (pre) {
    vec_fill(n, 0.0, t, s);
    launch_m(Op::Update, j, bm, s, n, V, t, ss, nullptr);
    (*pre)(t, w);
    vec_axpby(n, 1.0, w, 1.0, x, s);
  } else {
    launch_m(Op::Update, j, bm, s, n, V, x, ss, nullptr);
  }
  return j;
}

// Part of one delayed-GMRES restart cycle of `steps` Arnoldi steps, for
// recording in graphs: with j0 == 0 the cycle's start (r = b - A x into V[0]),
// then steps [j0, j1); with j1 == steps the cycle's end (last Hessenberg
// column, triangular solve, correction).  The steps are those of
// multi_cycle_delayed, split where it polls.
void multi_cycle_part(MultiSys& m, const double* b, double* x, const KrylovCfg& k, hipStream_t s,
                      const MultiOp& op,
                      const std::function<void(const double*, double*)>* pre, double* V, double* w, double* t,
                      int steps, int j0, int j1, int* matvecs) {
  require(k.delayed && 0 <= j0 && j0 < j1 && j1 <= steps && steps <= k.restart, SDG_EINVAL, "bad cycle part");
  const int64_t n = m.n_total;
  const BlockMap bm = map_of(m);
  if (j0 == 0) {
    multi_residual(m, b, x, s, op, V);
    ++*matvecs;
  }
  for (int j = j0; j < j1; ++j) {
    double* vj = V + (size_t)j * n;
    if (pre) {
      (*pre)(vj, t);
      op(t, w, true);
    } else {
      op(vj, w, true);
    }
    ++*matvecs;
    const bool last = j + 1 == steps;
    launch_dm(Dm::Multidot, j, m, bm, s, V, w);
    launch_dm(Dm::Fin, j, m, bm, s, V, w);
    launch_dm(last ? Dm::UpdateDots : Dm::Update, j, m, bm, s, V, w);
  }
  if (j1 == steps) {
    launch_dm(Dm::FinU, steps, m, bm, s, V, nullptr);
    multi_cycle_stop(m, x, k, s, pre, V, w, t, steps);
  }
}

// End of a cycle after its step j: triangular solve and correction (every
// system's column j-1 is complete; after an early stop the converged systems
// need no further column).
void multi_cycle_stop(MultiSys& m, double* x, const KrylovCfg& k, hipStream_t s,
                      const std::function<void(const double*, double*)>* pre, double* V, double* w, double* t,
                      int j) {
  (void)k;
  const int64_t n = m.n_total;
  const BlockMap bm = map_of(m);
  km_trisolve<<<(unsigned)((m.S * 64 + 255) / 256), 256, 0, s>>>(m.S, m.d_ss.p);
  SDG_HIP(hipGetLastError());
  if (pre) {
    vec_fill(n, 0.0, t, s);
    launch_m(Op::Update, j, bm, s, n, V, t, m.d_ss.p, nullptr);
    (*pre)(t, w);
    vec_axpby(n, 1.0, w, 1.0, x, s);
  } else {
    launch_m(Op::Update, j, bm, s, n, V, x, m.d_ss.p, nullptr);
  }
}

int multi_cycle(MultiSys& m, const double* b, double* x, const KrylovCfg& k, hipStream_t s,
                const MultiOp& op,
                const std::function<void(const double*, double*)>* pre, double* V, double* r, double* w, double* t,
                bool poll, int max_steps, int* matvecs, bool* all_converged) {
  if (k.delayed) return multi_cycle_delayed(m, b, x, k, s, op, pre, V, w, t, poll, max_steps, matvecs, all_converged);
  const int64_t n = m.n_total;
  const BlockMap bm = map_of(m);
  SysScalars* ss = m.d_ss.p;
  const unsigned st = sys_threads(m.S);
  const int check_every = std::max(1, k.check_every);
  *all_converged = false;
  multi_residual(m, b, x, s, op, r);
  ++*matvecs;
  if (poll) {
    if (read_int(m.d_nactive.p, m.h_pinned, s) == 0) {
      *all_converged = true;
      return 0;
    }
    if (max_steps <= 0) return 0;
  }
  km_scale<<<(unsigned)m.n_blocks, kT, 0, s>>>(bm, r, V, ss, 1);
  SDG_HIP(hipGetLastError());
  int kk = 0;
  for (int j = 0; j < k.restart && j < max_steps; ++j) {
    double* vj = V + (size_t)j * n;
    if (pre) {
      (*pre)(vj, t);
      op(t, w, true);
    } else {
      op(vj, w, true);
    }
    ++*matvecs;
    launch_m(Op::Multidot, j + 1, bm, s, n, V, w, ss, m.d_partials.p);
    finalize(m, j + 1, kH1, 0, s);
    launch_m(Op::Pass, j + 1, bm, s, n, V, w, ss, m.d_partials.p);
    finalize(m, j + 1, kH2, 0, s);
    launch_m(Op::Final, j + 1, bm, s, n, V, w, ss, m.d_partials.p);
    km_arnoldi_fin<<<1, 1024, 0, s>>>(m.d_partials.p, m.n_blocks, m.d_seg_blk0.p, m.S, j, ss, m.d_nactive.p);
    SDG_HIP(hipGetLastError());
    km_scale<<<(unsigned)m.n_blocks, kT, 0, s>>>(bm, w, V + (size_t)(j + 1) * n, ss, 1);
    SDG_HIP(hipGetLastError());
    kk = j + 1;
    if (poll && ((j + 1) % check_every == 0 || j + 1 == k.restart)) {
      if (read_int(m.d_nactive.p, m.h_pinned, s) == 0) break;
    }
  }
  km_trisolve<<<(unsigned)((m.S * 64 + 255) / 256), 256, 0, s>>>(m.S, ss);
  SDG_HIP(hipGetLastError());
  if (pre) {
    vec_fill(n, 0.0, t, s);
    launch_m(Op::Update, kk, bm, s, n, V, t, ss, nullptr);
    (*pre)(t, w);
    vec_axpby(n, 1.0, w, 1.0, x, s);
  } else {
    launch_m(Op::Update, kk, bm, s, n, V, x, ss, nullptr);
  }
  return kk;
}

int multi_nactive(MultiSys& m, hipStream_t s) { return read_int(m.d_nactive.p, m.h_pinned, s); }

void multi_outer_setup(MultiSys& m, const double* b, hipStream_t s) {
  seg_norm2(m, b, s);
  km_outer_bnorm<<<1, sys_threads(m.S), 0, s>>>(m.S, m.d_ss.p, m.d_outer.p);
  SDG_HIP(hipGetLastError());
}

void multi_refine_check(MultiSys& m, const double* d, double rtol, double inner_rtol, hipStream_t s) {
  seg_norm2(m, d, s);
  km_refine_check<<<1, sys_threads(m.S), 0, s>>>(m.S, m.d_ss.p, m.d_outer.p, rtol, inner_rtol, m.d_nouter.p);
  SDG_HIP(hipGetLastError());
}

int multi_nouter(MultiSys& m, hipStream_t s) { return read_int(m.d_nouter.p, m.h_pinned + 1, s); }

void multi_outer_result(MultiSys& m, hipStream_t s, SolveResult& res) {
  std::vector<double> h(2 * (size_t)m.S);
  SDG_HIP(hipMemcpyAsync(h.data(), m.d_outer.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  SDG_HIP(hipStreamSynchronize(s));
  double worst = 0.0, bmax = 0.0;
  for (int q = 0; q < m.S; ++q) {
    bmax = std::max(bmax, h[q]);
    worst = std::isfinite(h[m.S + q]) ? std::max(worst, h[m.S + q]) : h[m.S + q];
    require(std::isfinite(worst), SDG_ENONFINITE, "non-finite residual");
  }
  res.rel_res = worst;
  res.bnorm = bmax;
}

void multi_result(MultiSys& m, hipStream_t s, SolveResult& res) {
  std::vector<SysScalars> h;
  m.read_scalars(h, s);
  double worst = 0.0, bmax = 0.0;
  for (const SysScalars& q : h) {
    // std::max drops a NaN operand: test every system's residual itself
    require(std::isfinite(q.rnorm), SDG_ENONFINITE, "non-finite residual");
    if (q.bnorm > 0.0) worst = std::max(worst, q.rnorm / q.bnorm);
    bmax = std::max(bmax, q.bnorm);
  }
  res.rel_res = worst;
  res.bnorm = bmax;
  require(std::isfinite(worst), SDG_ENONFINITE, "non-finite residual");
}

SolveResult solve_gmres_multi(MultiSys& m, const double* b, double* x, const KrylovCfg& k, hipStream_t s,
                              const MultiOp& op,
                              const std::function<void(const double*, double*)>* pre, double* V, double* r,
                              double* w, double* t) {
  SolveResult res;
  if (!k.keep_targets) multi_setup(m, b, x, k.rtol, s);
  for (;;) {
    bool done = false;
    const int it = multi_cycle(m, b, x, k, s, op, pre, V, r, w, t, true, k.max_iter - res.iters, &res.matvecs, &done);
    res.iters += it;
    if (done) { res.converged = true; break; }
    if (it == 0 || res.iters >= k.max_iter) {
      // one more residual evaluation to report the final state
      bool d2 = false;
      multi_cycle(m, b, x, k, s, op, pre, V, r, w, t, true, 0, &res.matvecs, &d2);
      res.converged = d2;
      break;
    }
  }
  multi_result(m, s, res);
  return res;
}

}  // namespace sdg
