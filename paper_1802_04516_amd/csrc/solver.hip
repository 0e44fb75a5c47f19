// Krylov solvers and vector kernels for the velocity system (Section 4:
// conjugate gradients for the symmetric positive definite Crank-Nicolson
// system, matrix-free restarted GMRES for p_gamma > 0).
//
// All reductions are deterministic: each block writes a partial sum and a
// single-block finalize kernel adds the partials in a fixed order.
// Scalars (alpha, beta, Hessenberg column, Givens rotations) stay in device
// memory.  CG and the GMRES with SDG_SOLVE_CGS2 read one residual estimate
// every `check_every` iterations (a stream synchronisation); the default
// GMRES reads the estimate that its finalize kernel wrote into coherent
// pinned host memory, without draining the stream.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "context.hpp"
#include "reduce.hpp"

namespace sdg {

namespace {

constexpr int kThreads = 256;

__device__ inline double warp_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Sum of `v` over the block; result valid in thread 0.
__device__ inline double block_sum(double v, double* sh) {
  v = warp_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  __syncthreads();
  return r;
}

// Reductions are two launches: the producer kernel writes one partial sum
// per block and slot, and a single-block finalize kernel adds them.  One
// wavefront per slot: lane l adds blocks l, l+64, ..., then the wave adds the
// 64 lane sums with a fixed shuffle tree, so results are deterministic and no
// atomics are involved.
__device__ inline void reduce_slots(const double* partials, int nblocks, int nslots, double* out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int sl = wid; sl < nslots; sl += nw) {
    // slot-major layout: the wave's loads are contiguous and independent
    // all of the lane's loads (at most kRedBlocks / 64) in flight at once
    const double* ps = partials + (size_t)sl * kRedBlocks;
    constexpr int PER = kRedBlocks / 64;
    double pv[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) pv[q] = lane + 64 * q < nblocks ? ps[lane + 64 * q] : 0.0;
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q) v += pv[q];
    v = warp_sum(v);
    if (lane == 0) out[sl] = v;
  }
  __syncthreads();
}

// Sums of NS slots of partials (nblocks <= kRedBlocks per slot) by one
// workgroup of NW wavefronts, every load in flight at once: wave w adds the
// slots w, w + NW, ..., lane l the blocks l, l + 64, ... of each, then a
// fixed shuffle tree per slot.  Result in out[0..NS) (LDS), valid after the
// call.
template <int NS, int NW = 4>
__device__ inline void reduce_slots_wg(const double* partials, int nblocks, double* out) {
  constexpr int SPW = (NS + NW - 1) / NW, PER = kRedBlocks / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double v[SPW][PER];
#pragma unroll
  for (int i = 0; i < SPW; ++i) {
    const int sl = wid + NW * i;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int b = lane + 64 * q;
      v[i][q] = (sl < NS && b < nblocks) ? partials[(size_t)sl * kRedBlocks + b] : 0.0;
    }
  }
#pragma unroll
  for (int i = 0; i < SPW; ++i) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q) t += v[i][q];
    t = warp_sum(t);
    const int sl = wid + NW * i;
    if (lane == 0 && sl < NS) out[sl] = t;
  }
  __syncthreads();
}

unsigned red_grid(int64_t n) {
  int64_t b = (n + 4 * kThreads - 1) / (4 * kThreads);
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, kRedBlocks));
}

// out[0..nslots) = sum of the producer's partials
__global__ void k_finalize(const double* partials, int nblocks, int nslots, double* out) {
  reduce_slots(partials, nblocks, nslots, out);
}

__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

__global__ void k_fill(int64_t n, double v, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}

__global__ void k_copy(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i];
}

// out = x . y
__global__ void k_dot(int64_t n, const double* __restrict__ x, const double* __restrict__ y, double* partials) {
  __shared__ double sh[16];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    a0 += x[i] * y[i];
    a1 += x[i + stride] * y[i + stride];
    a2 += x[i + 2 * stride] * y[i + 2 * stride];
    a3 += x[i + 3 * stride] * y[i + 3 * stride];
  }
  for (; i < n; i += stride) a0 += x[i] * y[i];
  const double acc = block_sum((a0 + a1) + (a2 + a3), sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// ---------------------------------------------------------------- CG

// x += alpha p, r -= alpha q with alpha = rz / pq (sc->rr holds rz); the
// partials of r.r go to slot 0.
__global__ void k_cg_update(int64_t n, double* __restrict__ x, double* __restrict__ r,
                            const double* __restrict__ p, const double* __restrict__ q,
                            const DevScalars* sc, double* partials) {
  __shared__ double sh[16];
  const double alpha = sc->rr / sc->pq;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    acc += ri * ri;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// rr_new = sum partials; without a preconditioner also beta = rr_new / rz and
// rz = rr_new.
__global__ void k_cg_update_fin(const double* partials, int nblocks, DevScalars* sc, int finish_beta) {
  __shared__ double tot;
  reduce_slots(partials, nblocks, 1, &tot);
  if (threadIdx.x == 0) {
    sc->alpha = sc->rr / sc->pq;
    sc->rr_new = tot;
    if (finish_beta) {
      sc->beta = tot / sc->rr;
      sc->rr = tot;
    }
  }
}

// beta = (r . z)_new / rz and rz = (r . z)_new (preconditioned CG)
__global__ void k_dot_beta_fin(const double* partials, int nblocks, DevScalars* sc) {
  __shared__ double tot;
  reduce_slots(partials, nblocks, 1, &tot);
  if (threadIdx.x == 0) {
    sc->beta = tot / sc->rr;
    sc->rr = tot;
  }
}

// Factored element block inverse (several time nodes):
//   y_e = (I (x) Q_e) blockdiag_i(B_{e,i}) (I (x) Q_e^T) x_e
// (B^T for the transpose).  NV = NG*NS threads per element, several elements
// per workgroup, one element per thread group; every global load of the
// element (x, the column and the row of Q_e, the row of B_{e,i}) is issued
// first so that they are all in flight together, then x, u and w pass
// through LDS.
template <int NG, int NS>
__global__ __launch_bounds__(256) void k_block_apply_fact(int64_t n_elem, const float* __restrict__ Q,
                                                          const float* __restrict__ B, const double* __restrict__ x,
                                                          double* __restrict__ y, int transpose, int64_t cstride) {
  constexpr int NV = NG * NS;
  constexpr int EPB = 256 / NV;
  __shared__ double sx[EPB * NV], su[EPB * NV];
  x += blockIdx.y * cstride;
  y += blockIdx.y * cstride;
  const int le = threadIdx.x / NV, r = threadIdx.x % NV;
  const int a = r / NS, i = r % NS;
  const int64_t e = (int64_t)blockIdx.x * EPB + le;
  const bool act = le < EPB && e < n_elem;
  float qc[NS], qr[NS], bq[NG];
  double xv = 0.0;
  if (act) {
    const float* Qe = Q + (size_t)e * NS * NS;
    const float* Be = B + ((size_t)e * NS + i) * NG * NG;
    xv = x[e * NV + r];
#pragma unroll
    for (int ck = 0; ck < NS; ++ck) qc[ck] = Qe[ck * NS + i];
#pragma unroll
    for (int ii = 0; ii < NS; ++ii) qr[ii] = Qe[i * NS + ii];
#pragma unroll
    for (int b = 0; b < NG; ++b) bq[b] = transpose ? Be[b * NG + a] : Be[a * NG + b];
  }
  const int ls = le < EPB ? le : EPB - 1;
  double* sxe = sx + ls * NV;
  double* sue = su + ls * NV;
  if (act) sxe[r] = xv;
  __syncthreads();
  if (act) {  // u[a][i] = sum_ck Q[ck][i] x[a][ck]
    double acc = 0.0;
#pragma unroll
    for (int ck = 0; ck < NS; ++ck) acc += (double)qc[ck] * sxe[a * NS + ck];
    sue[r] = acc;
  }
  __syncthreads();
  double wv = 0.0;
  if (act) {  // w[a][i] = sum_b B_i[a][b] u[b][i]
#pragma unroll
    for (int b = 0; b < NG; ++b) wv += (double)bq[b] * sue[b * NS + i];
  }
  if (act) sxe[r] = wv;  // every read of x happened before the last barrier
  __syncthreads();
  if (act) {  // y[a][i] = sum_ii Q[i][ii] w[a][ii]
    double acc = 0.0;
#pragma unroll
    for (int ii = 0; ii < NS; ++ii) acc += (double)qr[ii] * sxe[a * NS + ii];
    y[e * NV + r] = acc;
  }
}

__global__ void k_cg_p(int64_t n, double* __restrict__ p, const double* __restrict__ r, const DevScalars* sc) {
  if (sc->cg_on == 0) return;
  const double beta = sc->beta;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = r[i] + beta * p[i];
}

// ---------------------------------------------------------------- GMRES

// The Gram-Schmidt kernels take the number of basis vectors NJ as a template
// parameter: every row's NJ loads are independent and unconditional, so a
// wavefront keeps them all in flight.

template <int NS>
__device__ inline void block_partials(const double (&acc)[NS], double* partials) {
  block_partials_to<NS>(acc, partials, kRedBlocks);
}

// h1[i] = V_i . w for i < NJ (classical Gram-Schmidt projections) and, in
// slot NJ, w . w
template <int NJ>
__global__ __launch_bounds__(256) void k_multidot(int64_t n, const double* __restrict__ V,
                                                  const double* __restrict__ w, double* partials) {
  double acc[NJ + 1];
#pragma unroll
  for (int i = 0; i <= NJ; ++i) acc[i] = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const double wt = w[t];
    double vi[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) vi[i] = V[(size_t)i * n + t];
#pragma unroll
    for (int i = 0; i < NJ; ++i) acc[i] += vi[i] * wt;
    acc[NJ] += wt * wt;
  }
  block_partials<NJ + 1>(acc, partials);
}

// ---- Arnoldi with delayed reorthogonalisation (one reduction per step).
// The low-synchronisation classical Gram-Schmidt with a lagged second
// projection of Swirydowicz, Langou, Ananthan, Yang and Thomas (2020) and
// Bielich, Langou, Thomas, Swirydowicz, Yamazaki and Boman (2022),
// restated here.  Step j holds the final orthonormal q_0..q_{j-1} (Q), the
// once-projected, unnormalised u_j in slot j of V and z = A P^-1 u_j.  One
// sweep forms b = Q^T u_j, c = Q^T z, u_j.u_j and u_j.z; then
//   nu = ||u_j - Q b|| = sqrt(u.u - b.b),  q_j = (u_j - Q b) / nu,
//   Hessenberg column j-1 = (a_{j-1} + b, nu)       (a: first projection),
//   w_j = A P^-1 q_j = (z - Q_j Hb) / nu,  Hb = H[0:j+1, 0:j] b
//         (the Arnoldi relation A P^-1 Q = Q_j H applied to b),
//   a_j = Q_j^T w_j:  a_j[i] = (c_i - Hb_i) / nu (i < j),
//                     a_j[j] = ((u.z - b.c) / nu - Hb_j) / nu,
// and one update sweep writes q_j over u_j and the next once-projected
//   u_{j+1} = w_j - Q_j a_j = z / nu - e u_j - Q f,
//   d = Hb / nu + a_j,  e = d_j / nu,  f_i = d_i - e b_i.
// The Hessenberg column of step j is complete one step later; the last
// column of a cycle is completed from dot products that the last step's
// update sweep forms.

// Slots [0, NJ) = Q^T u, [NJ, 2NJ) = Q^T z, 2NJ = u.u, 2NJ+1 = u.z, with
// Q = V[0..NJ), u = V[NJ].
template <int NJ>
__global__ __launch_bounds__(256) void k_dmultidot(int64_t n, const double* __restrict__ V,
                                                   const double* __restrict__ z, double* partials) {
  constexpr int NS = 2 * NJ + 2;
  double acc[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) acc[i] = 0.0;
  const double* __restrict__ u = V + (size_t)NJ * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const double ut = u[t];
    const double zt = z[t];
    double vi[NJ > 0 ? NJ : 1];
#pragma unroll
    for (int i = 0; i < NJ; ++i) vi[i] = V[(size_t)i * n + t];
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
      acc[i] += vi[i] * ut;
      acc[NJ + i] += vi[i] * zt;
    }
    acc[2 * NJ] += ut * ut;
    acc[2 * NJ + 1] += ut * zt;
  }
  block_partials<NS>(acc, partials);
}

// Finalize of step NJ (one 1024-thread block): nu, Hessenberg column NJ-1
// (unrotated in Hu, rotated in H), its Givens rotation, g and the residual
// estimate; with HZ (a step with z, partials of k_dmultidot) also a_NJ (into
// h1) and the update coefficients b (h2), f, e and 1/nu (inv_norm); without
// (the completion of a cycle's last column) the partials are Q^T u in slots
// [0, NJ) and u.u in slot NJ.  Step 0 sets g[0] = nu = ||r||.
template <int NJ, bool HZ>
__global__ __launch_bounds__(1024) void k_dfin(const double* partials, int nblocks, DevScalars* sc, double* poll,
                                               double stamp) {
  constexpr int NS = HZ ? 2 * NJ + 2 : NJ + 1, IA = HZ ? 2 * NJ : NJ, ld = kMaxRestart + 1,
                NC = NJ > 0 ? NJ : 1;
  __shared__ double sv[NS];
  __shared__ double sHu[(NJ + 1) * NC];  // columns 0..NJ-1, ld NJ+1
  __shared__ double sHb[NJ + 1];
  __shared__ double sa[NC], scs[NC], ssn[NC], sgj;
  __shared__ double sc_[4];  // nu, 1/nu, e
  const int tid = threadIdx.x;
  // everything the serial part reads, staged in LDS with parallel loads that
  // are in flight together with the partials' loads
  for (int i = tid; i < (NJ + 1) * NJ; i += blockDim.x) {
    const int col = i / (NJ + 1), row = i % (NJ + 1);
    sHu[i] = col + 1 < NJ && row <= col + 1 ? sc->Hu[(size_t)col * ld + row] : 0.0;
  }
  if (tid < NJ) {
    sa[tid] = sc->h1[tid];
    if (tid + 1 < NJ) {
      scs[tid] = sc->cs[tid];
      ssn[tid] = sc->sn[tid];
    }
  }
  if (NJ > 0 && tid == 64) sgj = sc->g[NJ > 0 ? NJ - 1 : 0];
  reduce_slots_wg<NS, 16>(partials, nblocks, sv);  // ends with a barrier
  if (tid == 0) {
    double bb = 0.0;
#pragma unroll
    for (int i = 0; i < NJ; ++i) bb += sv[i] * sv[i];
    const double nu2 = sv[IA] - bb;
    const double nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
    const double inv = nu > 0.0 ? 1.0 / nu : 0.0;
    sc_[0] = nu;
    sc_[1] = inv;
    sc->norm = nu;
    double est = nu;
    if (NJ == 0) {
      sc->g[0] = nu;
      sc->resid = nu;
    } else {
      // complete column NJ-1, then rotate it
      double hc[NJ + 1];
#pragma unroll
      for (int i = 0; i < NJ; ++i) hc[i] = sa[i] + sv[i];
      hc[NJ] = nu;
#pragma unroll
      for (int i = 0; i <= NJ; ++i) sHu[(NJ - 1) * (NJ + 1) + i] = hc[i];
#pragma unroll
      for (int i = 0; i + 1 < NJ; ++i) {
        const double a = hc[i], b = hc[i + 1];
        hc[i] = scs[i] * a + ssn[i] * b;
        hc[i + 1] = -ssn[i] * a + scs[i] * b;
      }
      const double a = hc[NJ - 1], b = hc[NJ];
      const double rad = hypot(a, b);
      const double cr = rad > 0.0 ? a / rad : 1.0, sr = rad > 0.0 ? b / rad : 0.0;
      sc->cs[NJ - 1] = cr;
      sc->sn[NJ - 1] = sr;
      hc[NJ - 1] = rad;
      hc[NJ] = 0.0;
      double* Hc = sc->H + (size_t)(NJ - 1) * ld;
#pragma unroll
      for (int i = 0; i <= NJ; ++i) Hc[i] = hc[i];
      sc->g[NJ - 1] = cr * sgj;
      sc->g[NJ] = -sr * sgj;
      est = fabs(sr * sgj);
      sc->resid = est;
    }
    if (poll) {
      // residual estimate of this step, then its stamp, to coherent pinned
      // host memory
      __hip_atomic_store(&poll[1 + NJ], est, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(&poll[0], stamp, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
  if (NJ == 0 && tid > 0 && tid <= kMaxRestart) sc->g[tid] = 0.0;
  __syncthreads();
  if (NJ > 0 && tid <= NJ) sc->Hu[(size_t)(NJ - 1) * ld + tid] = sHu[(NJ - 1) * (NJ + 1) + tid];
  if (!HZ) return;
  // Hb = H[0:NJ+1, 0:NJ] b
  if (tid <= NJ) {
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < NJ; ++i) acc += sHu[i * (NJ + 1) + tid] * sv[i];  // zero below the subdiagonal
    sHb[tid] = acc;
  }
  __syncthreads();
  if (tid == 0) {
    const double inv = sc_[1];
    double bc = 0.0;
#pragma unroll
    for (int i = 0; i < NJ; ++i) bc += sv[i] * sv[NJ + i];
    const double aj = ((sv[2 * NJ + 1] - bc) * inv - sHb[NJ]) * inv;
    const double dj = sHb[NJ] * inv + aj;
    const double e = dj * inv;
    sc->h1[NJ] = aj;
    sc->e = e;
    sc->inv_norm = inv;
    sc_[2] = e;
  }
  __syncthreads();
  if (tid < NJ) {
    const double inv = sc_[1], e = sc_[2];
    const double ai = (sv[NJ + tid] - sHb[tid]) * inv;
    const double di = sHb[tid] * inv + ai;
    sc->h1[tid] = ai;
    sc->h2[tid] = sv[tid];
    sc->f[tid] = di - e * sv[tid];
  }
}

// Update sweep of step NJ: q_NJ = (u - Q b) / nu over slot NJ of V, and the
// next once-projected vector u_{NJ+1} = z / nu - e u - Q f into slot NJ+1.
// With DOTS (the last step of a cycle) the sweep also forms the partials of
// the completion of column NJ: q_i . u_{NJ+1} for i <= NJ and
// u_{NJ+1} . u_{NJ+1}: slots [0, NJ] and NJ + 1.
template <int NJ, bool DOTS = false>
__global__ __launch_bounds__(256) void k_dupdate(int64_t n, double* V, const double* __restrict__ z,
                                                 const DevScalars* sc, double* partials) {
  double bq[NJ > 0 ? NJ : 1], fq[NJ > 0 ? NJ : 1];
#pragma unroll
  for (int i = 0; i < NJ; ++i) { bq[i] = sc->h2[i]; fq[i] = sc->f[i]; }
  const double inv = sc->inv_norm, e = sc->e;
  const double* __restrict__ Q = V;
  double* __restrict__ u = V + (size_t)NJ * n;
  double* __restrict__ un = V + (size_t)(NJ + 1) * n;
  double acc[DOTS ? NJ + 2 : 1];
#pragma unroll
  for (int i = 0; i < (DOTS ? NJ + 2 : 1); ++i) acc[i] = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double vi[NJ > 0 ? NJ : 1];
#pragma unroll
    for (int i = 0; i < NJ; ++i) vi[i] = Q[(size_t)i * n + t];
    const double ut = u[t];
    double q = ut, w = z[t] * inv - e * ut;
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
      q -= bq[i] * vi[i];
      w -= fq[i] * vi[i];
    }
    q *= inv;
    u[t] = q;
    un[t] = w;
    if constexpr (DOTS) {
#pragma unroll
      for (int i = 0; i < NJ; ++i) acc[i] += vi[i] * w;
      acc[NJ] += q * w;
      acc[NJ + 1] += w * w;
    }
  }
  if constexpr (DOTS) block_partials<NJ + 2>(acc, partials);
}

#define SDG_NJ0_CASES(X)                                                                                        \
  X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) \
  X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)

enum class Dg { Multidot, Fin, FinU, Update, UpdateDots };

// Launch a kernel of the delayed scheme for step nj (FinU: the completion
// of the last column of a cycle, from the partials of UpdateDots; Fin / FinU
// take the producer's grid size as `grid`).
void launch_dgs(Dg which, int nj, unsigned grid, hipStream_t s, int64_t n, double* V, const double* z,
                DevScalars* sc, double* partials, double* poll = nullptr, double stamp = 0.0) {
  // a step with z has at most kMaxRestart - 1 final vectors before it
  require(nj < kMaxRestart || which == Dg::FinU, SDG_EINVAL,
          "Gram-Schmidt basis size out of range");
  switch (nj) {
#define SDG_DG_Z(N) (N < kMaxRestart ? N : kMaxRestart - 1)
#define SDG_DG_CASE(N)                                                                                      \
  case N:                                                                                                   \
    if (which == Dg::Multidot) k_dmultidot<SDG_DG_Z(N)><<<grid, 256, 0, s>>>(n, V, z, partials);            \
    else if (which == Dg::Fin) k_dfin<SDG_DG_Z(N), true><<<1, 1024, 0, s>>>(partials, (int)grid, sc, poll, stamp); \
    else if (which == Dg::FinU) k_dfin<N, false><<<1, 1024, 0, s>>>(partials, (int)grid, sc, nullptr, 0.0); \
    else if (which == Dg::UpdateDots) k_dupdate<SDG_DG_Z(N), true><<<grid, 256, 0, s>>>(n, V, z, sc, partials); \
    else k_dupdate<SDG_DG_Z(N)><<<grid, 256, 0, s>>>(n, V, z, sc, nullptr);                                 \
    break;
    SDG_NJ0_CASES(SDG_DG_CASE)
#undef SDG_DG_CASE
#undef SDG_DG_Z
    default:
      throw Error(SDG_EINVAL, "Gram-Schmidt basis size out of range");
  }
}

// h1 from the first projection's partials, and the decision whether this
// step needs a second projection: the "twice is enough" test of Daniel,
// Gragg, Kaufman and Stewart (1976), reorthogonalise when
// ||w - V h1||^2 = ||w||^2 - ||h1||^2 < ||w||^2 / 2.  When the test passes,
// the Pythagorean value is accurate to rounding, so no loss of
// orthogonality is missed.  One 256-thread block.
template <int NJ>
__global__ __launch_bounds__(256) void k_h1_fin(const double* partials, int nblocks, DevScalars* sc) {
  __shared__ double hs[NJ + 1];
  reduce_slots_wg<NJ + 1>(partials, nblocks, hs);
  if (threadIdx.x <= NJ) sc->h1[threadIdx.x] = hs[threadIdx.x];
  if (threadIdx.x == 0) {
    const double ww = hs[NJ];
    double hh = 0.0;
    for (int i = 0; i < NJ; ++i) hh += hs[i] * hs[i];
    const double r = (ww - hh < 0.5 * ww) ? 1.0 : 0.0;
    sc->reorth = r;
    sc->n_reorth += r;
  }
}

// h2 from the second projection's partials, or zero without one.  One
// 256-thread block.
template <int NJ>
__global__ __launch_bounds__(256) void k_h2_fin(const double* partials, int nblocks, DevScalars* sc) {
  if (sc->reorth != 0.0) {
    __shared__ double hs[NJ];
    reduce_slots_wg<NJ>(partials, nblocks, hs);
    if (threadIdx.x < NJ) sc->h2[threadIdx.x] = hs[threadIdx.x];
  } else if (threadIdx.x < NJ) {
    sc->h2[threadIdx.x] = 0.0;
  }
}

// w -= V h1.  When the step needs a second projection (sc->reorth), the
// partials of h2 = V . w follow; otherwise the partials of w . w (slot 0).
template <int NJ>
__global__ __launch_bounds__(256) void k_cgs_pass(int64_t n, const double* __restrict__ V, double* __restrict__ w,
                                                  const DevScalars* sc, double* partials) {
  double h[NJ];
#pragma unroll
  for (int i = 0; i < NJ; ++i) h[i] = sc->h1[i];
  if (sc->reorth != 0.0) {
    double acc[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) acc[i] = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
      double vi[NJ];
#pragma unroll
      for (int i = 0; i < NJ; ++i) vi[i] = V[(size_t)i * n + t];
      double wt = w[t];
#pragma unroll
      for (int i = 0; i < NJ; ++i) wt -= h[i] * vi[i];
      w[t] = wt;
#pragma unroll
      for (int i = 0; i < NJ; ++i) acc[i] += vi[i] * wt;
    }
    block_partials<NJ>(acc, partials);
  } else {
    double acc[1] = {0.0};
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
      double vi[NJ];
#pragma unroll
      for (int i = 0; i < NJ; ++i) vi[i] = V[(size_t)i * n + t];
      double wt = w[t];
#pragma unroll
      for (int i = 0; i < NJ; ++i) wt -= h[i] * vi[i];
      w[t] = wt;
      acc[0] += wt * wt;
    }
    block_partials<1>(acc, partials);
  }
}

// Second projection (only when sc->reorth): w -= V h2 and partials of w.w.
template <int NJ>
__global__ __launch_bounds__(256) void k_cgs_final(int64_t n, const double* __restrict__ V, double* __restrict__ w,
                                                   const DevScalars* sc, double* partials) {
  if (sc->reorth == 0.0) return;
  double h[NJ];
#pragma unroll
  for (int i = 0; i < NJ; ++i) h[i] = sc->h2[i];
  double acc[1] = {0.0};
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double vi[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) vi[i] = V[(size_t)i * n + t];
    double wt = w[t];
#pragma unroll
    for (int i = 0; i < NJ; ++i) wt -= h[i] * vi[i];
    w[t] = wt;
    acc[0] += wt * wt;
  }
  block_partials<1>(acc, partials);
}

// x += sum_i y_i V_i, or x = sum_i y_i V_i (SET)
template <int NJ, bool SET = false>
__global__ __launch_bounds__(256) void k_gmres_update(int64_t n, const double* __restrict__ V, double* __restrict__ x,
                                                      const DevScalars* sc) {
  double ys[NJ];
#pragma unroll
  for (int i = 0; i < NJ; ++i) ys[i] = sc->y[i];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double vi[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) vi[i] = V[(size_t)i * n + t];
    double acc = SET ? 0.0 : x[t];
#pragma unroll
    for (int i = 0; i < NJ; ++i) acc += ys[i] * vi[i];
    x[t] = acc;
  }
}

#define SDG_NJ_CASES(X)                                                                                    \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) \
  X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)
static_assert(kMaxRestart == 32, "the Gram-Schmidt dispatch covers 1..32 basis vectors");

enum class Gs { Multidot, Pass, Final, Update, UpdateSet, H1Fin, H2Fin };

// Launch one of the Gram-Schmidt kernels for nj basis vectors (the
// finalize kernels H1Fin / H2Fin take the producer's grid size as `grid`).
void launch_gs(Gs which, int nj, unsigned grid, hipStream_t s, int64_t n, const double* V, double* w,
               DevScalars* sc, double* partials) {
  switch (nj) {
#define SDG_GS_CASE(N)                                                                       \
  case N:                                                                                    \
    if (which == Gs::Multidot) k_multidot<N><<<grid, 256, 0, s>>>(n, V, w, partials);         \
    else if (which == Gs::Pass) k_cgs_pass<N><<<grid, 256, 0, s>>>(n, V, w, sc, partials);    \
    else if (which == Gs::Final) k_cgs_final<N><<<grid, 256, 0, s>>>(n, V, w, sc, partials);  \
    else if (which == Gs::H1Fin) k_h1_fin<N><<<1, 256, 0, s>>>(partials, (int)grid, sc);       \
    else if (which == Gs::H2Fin) k_h2_fin<N><<<1, 256, 0, s>>>(partials, (int)grid, sc);       \
    else if (which == Gs::UpdateSet) k_gmres_update<N, true><<<grid, 256, 0, s>>>(n, V, w, sc); \
    else k_gmres_update<N><<<grid, 256, 0, s>>>(n, V, w, sc);                                 \
    break;
    SDG_NJ_CASES(SDG_GS_CASE)
#undef SDG_GS_CASE
    default:
      throw Error(SDG_EINVAL, "Gram-Schmidt basis size out of range");
  }
}

// Completes Arnoldi step j and writes the next basis vector:
//   every block adds the ||w||^2 partials (slot 0) in the same fixed order,
//   so all blocks hold the same norm, and scales its rows of w into v;
//   block 0 also completes the Hessenberg column j (h1 + h2 and the norm),
//   applies the previous Givens rotations, forms the new one and updates g.
// The partials are read by every block (nblocks doubles each) instead of
// being reduced by a separate single-block launch.
__global__ __launch_bounds__(256) void k_arnoldi_scale(int64_t n, const double* partials, int nblocks, int nj,
                                                       DevScalars* sc, const double* __restrict__ w,
                                                       double* __restrict__ v) {
  __shared__ double tot_sh;
  {
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 64) {
      constexpr int PER = kRedBlocks / 64;
      double pv[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) pv[q] = lane + 64 * q < nblocks ? partials[lane + 64 * q] : 0.0;
      double a = 0.0;
#pragma unroll
      for (int q = 0; q < PER; ++q) a += pv[q];
      const double t = warp_sum(a);
      if (lane == 0) tot_sh = t;
    }
    __syncthreads();
  }
  const double nrm = sqrt(tot_sh);
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v[i] = w[i] * inv;
  if (blockIdx.x == 0) {
    // Hessenberg column and rotations staged in LDS with parallel loads, so
    // the serial rotation loop runs from LDS
    __shared__ double hc[kMaxRestart + 1], cs[kMaxRestart], sn[kMaxRestart];
    const int j = nj - 1;
    for (int i = threadIdx.x; i < nj; i += blockDim.x) {
      hc[i] = sc->h1[i] + sc->h2[i];
      if (i < j) { cs[i] = sc->cs[i]; sn[i] = sc->sn[i]; }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      hc[j + 1] = nrm;
      sc->norm = nrm;
      sc->inv_norm = inv;
      for (int i = 0; i < j; ++i) {
        const double a = hc[i], b = hc[i + 1];
        hc[i] = cs[i] * a + sn[i] * b;
        hc[i + 1] = -sn[i] * a + cs[i] * b;
      }
      const double a = hc[j], b = hc[j + 1];
      const double rad = hypot(a, b);
      const double c = rad > 0.0 ? a / rad : 1.0, s = rad > 0.0 ? b / rad : 0.0;
      sc->cs[j] = c;
      sc->sn[j] = s;
      hc[j] = rad;
      hc[j + 1] = 0.0;
      const double gj = sc->g[j];
      sc->g[j] = c * gj;
      sc->g[j + 1] = -s * gj;
      sc->resid = fabs(sc->g[j + 1]);
    }
    __syncthreads();
    double* Hc = sc->H + (size_t)j * (kMaxRestart + 1);
    for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) Hc[i] = hc[i];
  }
}

__global__ void k_scale_into(int64_t n, const double* __restrict__ w, double* __restrict__ v, const double* scale) {
  const double s = *scale;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v[i] = w[i] * s;
}

// Start of a cycle: g = (beta, 0, ...), V_0 = r / beta.
__global__ void k_gmres_start(DevScalars* sc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double beta = sqrt(sc->dots[0]);
    for (int i = 0; i <= kMaxRestart; ++i) sc->g[i] = 0.0;
    sc->g[0] = beta;
    sc->norm = beta;
    sc->inv_norm = beta > 0.0 ? 1.0 / beta : 0.0;
    sc->resid = beta;
  }
}

// Back substitution R y = g for the leading k x k triangle.
// y = R^-1 g for the k x k upper triangle R of the rotated Hessenberg
// matrix, one wavefront: lane l holds row l of R and the running right-hand
// side r_l; column by column from the last, y_i = r_i / R_ii is broadcast
// and the lanes above subtract R_li y_i.
__global__ __launch_bounds__(64) void k_gmres_trisolve(DevScalars* sc, int k) {
  constexpr int ld = kMaxRestart + 1;
  const int l = threadIdx.x;
  double hrow[kMaxRestart];
#pragma unroll
  for (int i = 0; i < kMaxRestart; ++i) hrow[i] = (l < k && i < k) ? sc->H[(size_t)i * ld + l] : 0.0;
  double r = l < k ? sc->g[l] : 0.0, y = 0.0;
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
  if (l < k) sc->y[l] = y;
}

bool debug_krylov() {
  static const bool on = std::getenv("SDG_DEBUG_KRYLOV") != nullptr;
  return on;
}

unsigned vgrid(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

void check_launch() { SDG_HIP(hipGetLastError()); }

double read_scalar(Ctx& c, const double* dev, hipStream_t s) {
  SDG_HIP(hipMemcpyAsync(c.h_pinned, dev, sizeof(double), hipMemcpyDeviceToHost, s));
  SDG_HIP(hipStreamSynchronize(s));
  return c.h_pinned[0];
}

// r.r of the last iteration the fused CG update ran, and their count (one
// read-back of cg_stat)
static double read_cg_stat(Ctx& c, const DevScalars* sc, hipStream_t s, int& iters) {
  SDG_HIP(hipMemcpyAsync(c.h_pinned, sc->cg_stat, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  SDG_HIP(hipStreamSynchronize(s));
  iters = (int)c.h_pinned[1];
  return c.h_pinned[0];
}

}  // namespace

// ---------------------------------------------------------------- public helpers

void vec_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  k_axpby<<<vgrid(n), kThreads, 0, s>>>(n, a, x, b, y);
  check_launch();
}

void vec_fill(int64_t n, double value, double* y, hipStream_t s) {
  k_fill<<<vgrid(n), kThreads, 0, s>>>(n, value, y);
  check_launch();
}

void vec_copy(int64_t n, const double* x, double* y, hipStream_t s) {
  k_copy<<<vgrid(n), kThreads, 0, s>>>(n, x, y);
  check_launch();
}

static void dev_dot(Ctx& c, int64_t n, const double* x, const double* y, double* out, hipStream_t s) {
  const unsigned g = red_grid(n);
  k_dot<<<g, kThreads, 0, s>>>(n, x, y, c.d_partials.p);
  check_launch();
  k_finalize<<<1, 512, 0, s>>>(c.d_partials.p, (int)g, 1, out);
  check_launch();
}

double vec_dot_host(Ctx& c, int64_t n, const double* x, const double* y, hipStream_t s) {
  dev_dot(c, n, x, y, &c.d_sc.p->dots[0], s);
  return read_scalar(c, &c.d_sc.p->dots[0], s);
}

static double read_scalar_dot(Ctx& c, int64_t n, const double* r, hipStream_t s) {
  return vec_dot_host(c, n, r, r, s);
}

// Explicit element block inverse y_e = P_e x_e for a compile-time block size
// NV.  P_e is symmetric and stored as its packed upper triangle (entry (r, c),
// r <= c, at c (c + 1) / 2 + r, FP32), so the transpose is the same product.
// The packed blocks of a workgroup's elements are contiguous: they are
// copied to LDS with coalesced loads (issued together with the x loads),
// then one thread per row forms y from LDS.  Launched with EPB * NV threads.
template <int NV>
__global__ __launch_bounds__(256) void k_block_apply_sym(int64_t n_elem, const float* __restrict__ P,
                                                         const double* __restrict__ x, double* __restrict__ y,
                                                         int64_t cstride) {
  constexpr int EPB = 256 / NV, NP = NV * (NV + 1) / 2, NT = EPB * NV;  // NT threads per workgroup
  constexpr int PPT = (EPB * NP + NT - 1) / NT;  // packed values copied per thread
  __shared__ double sx[EPB * NV];
  __shared__ float sP[EPB * NP];
  x += blockIdx.y * cstride;
  y += blockIdx.y * cstride;
  const int le = threadIdx.x / NV, r = threadIdx.x % NV;
  const int64_t e0 = (int64_t)blockIdx.x * EPB;
  const int ne = (int)min((int64_t)EPB, n_elem - e0);
  const int64_t e = e0 + le;
  const bool act = le < ne;
  {
    const float* Pg = P + (size_t)e0 * NP;
    float pv[PPT];
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      const int i = threadIdx.x + u * NT;
      pv[u] = i < ne * NP ? Pg[i] : 0.0f;
    }
    const double xv = act ? x[e * NV + r] : 0.0;
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      const int i = threadIdx.x + u * NT;
      if (i < ne * NP) sP[i] = pv[u];
    }
    if (act) sx[le * NV + r] = xv;
  }
  __syncthreads();
  if (act) {
    const float* Pe = sP + le * NP;
    const int rr = r * (r + 1) / 2;
    double acc = 0.0;
#pragma unroll
    for (int col = 0; col < NV; ++col)
      acc += (double)Pe[r <= col ? col * (col + 1) / 2 + r : rr + col] * sx[le * NV + col];
    y[e * NV + r] = acc;
  }
}

void launch_block_apply(int64_t n_elem, int nv, const float* P, const double* x, double* y, bool transpose,
                        hipStream_t s, int ncols, int64_t cstride) {
  (void)transpose;  // symmetric blocks
  const unsigned gy = (unsigned)std::max(1, ncols);
  // d N_phi for 2D p = 1..4 and 3D p = 1..4 (one time node)
#define SDG_BLK_NV(NV_)                                                                                      \
  if (nv == NV_) {                                                                                           \
    constexpr int epb = 256 / NV_;                                                                           \
    const int64_t groups = (n_elem + epb - 1) / epb;                                                         \
    require(groups <= 0x7fffffff, SDG_EINVAL, "too many elements for the block preconditioner grid");        \
    k_block_apply_sym<NV_><<<dim3((unsigned)std::max<int64_t>(1, groups), gy), epb * NV_, 0, s>>>(            \
        n_elem, P, x, y, cstride);                                                                           \
    check_launch();                                                                                          \
    return;                                                                                                  \
  }
  SDG_BLK_NV(6) SDG_BLK_NV(12) SDG_BLK_NV(20) SDG_BLK_NV(30) SDG_BLK_NV(60) SDG_BLK_NV(105)
#undef SDG_BLK_NV
  throw Error(SDG_EUNSUPPORTED, "no block-preconditioner kernel for this element size");
}

// Update sweep of a delayed-GMRES step fused with the factored block
// preconditioner of the next basis vector: per element (NV = NG*NS rows,
// several elements per workgroup) q_nj = (u - Q b) / nu over slot nj of V and
// u_{nj+1} = z / nu - e u - Q f into slot nj+1, as k_dupdate, then
// t = P^-1 u_{nj+1} from LDS, as k_block_apply_fact, with the same
// arithmetic in the same order.  nj is a runtime count; the basis loads go
// in chunks of 8 with every load of a chunk in flight.
template <int NG, int NS>
__global__ __launch_bounds__(256) void k_dupdate_pre(int64_t n_elem, int nj, int64_t n, double* V,
                                                     const double* __restrict__ z, const DevScalars* sc,
                                                     const float* __restrict__ Qf, const float* __restrict__ Bf,
                                                     double* __restrict__ tout, int transpose) {
  constexpr int NV = NG * NS;
  constexpr int EPB = 256 / NV;
  __shared__ double sb[kMaxRestart], sf[kMaxRestart];
  __shared__ double sx[EPB * NV], su[EPB * NV];
  const int le = threadIdx.x / NV, r = threadIdx.x % NV;
  const int a = r / NS, i = r % NS;
  const int64_t e = (int64_t)blockIdx.x * EPB + le;
  const bool act = le < EPB && e < n_elem;
  const int64_t row = e * NV + r;
  if (threadIdx.x < nj) {
    sb[threadIdx.x] = sc->h2[threadIdx.x];
    sf[threadIdx.x] = sc->f[threadIdx.x];
  }
  const double inv = sc->inv_norm, ee = sc->e;
  float qc[NS], qr[NS], bq[NG];
  double ut = 0.0, zt = 0.0;
  if (act) {
    const float* Qe = Qf + (size_t)e * NS * NS;
    const float* Be = Bf + ((size_t)e * NS + i) * NG * NG;
    ut = V[(size_t)nj * n + row];
    zt = z[row];
#pragma unroll
    for (int ck = 0; ck < NS; ++ck) qc[ck] = Qe[ck * NS + i];
#pragma unroll
    for (int ii = 0; ii < NS; ++ii) qr[ii] = Qe[i * NS + ii];
#pragma unroll
    for (int b = 0; b < NG; ++b) bq[b] = transpose ? Be[b * NG + a] : Be[a * NG + b];
  }
  __syncthreads();
  double w = 0.0;
  if (act) {
    double q = ut;
    w = zt * inv - ee * ut;
    for (int i0 = 0; i0 < nj; i0 += 8) {
      double vi[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) vi[k] = i0 + k < nj ? V[(size_t)(i0 + k) * n + row] : 0.0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (i0 + k < nj) {
          q -= sb[i0 + k] * vi[k];
          w -= sf[i0 + k] * vi[k];
        }
      }
    }
    V[(size_t)nj * n + row] = q * inv;
    V[(size_t)(nj + 1) * n + row] = w;
  }
  const int ls = le < EPB ? le : EPB - 1;
  double* sxe = sx + ls * NV;
  double* sue = su + ls * NV;
  if (act) sxe[r] = w;
  __syncthreads();
  if (act) {  // u[a][i] = sum_ck Q[ck][i] x[a][ck]
    double acc = 0.0;
#pragma unroll
    for (int ck = 0; ck < NS; ++ck) acc += (double)qc[ck] * sxe[a * NS + ck];
    sue[r] = acc;
  }
  __syncthreads();
  double wv = 0.0;
  if (act) {  // w[a][i] = sum_b B_i[a][b] u[b][i]
#pragma unroll
    for (int b = 0; b < NG; ++b) wv += (double)bq[b] * sue[b * NS + i];
  }
  if (act) sxe[r] = wv;
  __syncthreads();
  if (act) {  // y[a][i] = sum_ii Q[i][ii] w[a][ii]
    double acc = 0.0;
#pragma unroll
    for (int ii = 0; ii < NS; ++ii) acc += (double)qr[ii] * sxe[a * NS + ii];
    tout[row] = acc;
  }
}

// The fused update + preconditioner above for (ng, ns); false where no
// factored kernel exists for the element size.
bool launch_dupdate_pre(int64_t n_elem, int ng, int ns, int nj, int64_t n, double* V, const double* z,
                        const DevScalars* sc, const float* Q, const float* B, double* t, bool transpose,
                        hipStream_t s) {
  auto go = [&](auto kernel, int nv) {
    const int epb = 256 / nv;
    const int64_t groups = (n_elem + epb - 1) / epb;
    require(groups <= 0x7fffffff, SDG_EINVAL, "too many elements for the block preconditioner grid");
    kernel<<<(unsigned)std::max<int64_t>(1, groups), epb * nv, 0, s>>>(n_elem, nj, n, V, z, sc, Q, B, t,
                                                                      transpose ? 1 : 0);
    check_launch();
  };
#define SDG_DPRE(NG_, NS_) \
  if (ng == NG_ && ns == NS_) { go(k_dupdate_pre<NG_, NS_>, NG_ * NS_); return true; }
#define SDG_DPRE_NS(NS_) SDG_DPRE(2, NS_) SDG_DPRE(3, NS_) SDG_DPRE(4, NS_)
  SDG_DPRE_NS(6) SDG_DPRE_NS(12) SDG_DPRE_NS(20) SDG_DPRE_NS(30) SDG_DPRE_NS(60)
#undef SDG_DPRE_NS
#undef SDG_DPRE
  return false;
}

void launch_block_apply_fact(int64_t n_elem, int ng, int ns, const float* Q, const float* B, const double* x,
                             double* y, bool transpose, hipStream_t s, int ncols, int64_t cstride) {
  const unsigned gy = (unsigned)std::max(1, ncols);
  auto go = [&](auto kernel, int nv) {
    const int epb = 256 / nv;
    const int64_t groups = (n_elem + epb - 1) / epb;
    require(groups <= 0x7fffffff, SDG_EINVAL, "too many elements for the block preconditioner grid");
    kernel<<<dim3((unsigned)std::max<int64_t>(1, groups), gy), epb * nv, 0, s>>>(n_elem, Q, B, x, y,
                                                                                transpose ? 1 : 0, cstride);
  };
#define SDG_FACT(NG_, NS_) \
  if (ng == NG_ && ns == NS_) { go(k_block_apply_fact<NG_, NS_>, NG_ * NS_); check_launch(); return; }
#define SDG_FACT_NS(NS_) SDG_FACT(2, NS_) SDG_FACT(3, NS_) SDG_FACT(4, NS_)
  // d N_phi for 2D p = 1..4 and 3D p = 1..3
  SDG_FACT_NS(6) SDG_FACT_NS(12) SDG_FACT_NS(20) SDG_FACT_NS(30) SDG_FACT_NS(60)
#undef SDG_FACT_NS
#undef SDG_FACT
  throw Error(SDG_EUNSUPPORTED, "no factored block-preconditioner kernel for this element size");
}

// CG update fused with the explicit element block preconditioner and the
// reductions of the two inner products that follow it.  One workgroup per
// group of EPB elements (NV rows each): alpha = rz / pq, x += alpha p,
// r -= alpha q, z_e = P_e r_e (packed symmetric block, as in
// k_block_apply_sym), and the group's partial sums of r.r and r.z, written
// to partials[block] and partials[ngroups + block].  (One group per
// workgroup rather than a loop over groups: a loop would wait for each
// group's stores before the next group's loads could be used, since one
// counter retires both in issue order.)  Launched with 256 threads (whole
// wavefronts for the block reduction; rows past EPB * NV idle).
template <int NV, typename VT = double>
__global__ __launch_bounds__(256) void k_cg_update_blk(int64_t n_elem, const float* __restrict__ P,
                                                       VT* __restrict__ x, VT* __restrict__ r,
                                                       const VT* __restrict__ p, const VT* __restrict__ q,
                                                       VT* __restrict__ z, const DevScalars* sc,
                                                       double* partials, int ngroups) {
  if (sc->cg_on == 0) return;  // converged: an iteration queued past the stop
  constexpr int EPB = 256 / NV, NP = NV * (NV + 1) / 2;
  constexpr int PPT = (EPB * NP + 255) / 256;
  __shared__ double sx[EPB * NV];
  __shared__ float sP[EPB * NP];
  const int le = threadIdx.x / NV, row = threadIdx.x % NV;
  const int64_t e0 = (int64_t)blockIdx.x * EPB;
  const int ne = (int)min((int64_t)EPB, n_elem - e0);
  const bool act = le < ne;
  const int64_t i = (e0 + le) * NV + row;
  const float* Pg = P + (size_t)e0 * NP;
  float pv[PPT];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int j = threadIdx.x + u * 256;
    pv[u] = j < ne * NP ? __builtin_nontemporal_load(&Pg[j]) : 0.0f;  // read once: non-temporal
  }
  double xi = 0.0, pi = 0.0, ri = 0.0, qi = 0.0;
  if (act) {
    xi = (double)x[i];
    pi = (double)p[i];
    ri = (double)r[i];
    qi = (double)q[i];
  }
  const double alpha = sc->rr / sc->pq;
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int j = threadIdx.x + u * 256;
    if (j < ne * NP) sP[j] = pv[u];
  }
  double acc[2] = {0.0, 0.0};
  if (act) {
    x[i] = (VT)(xi + alpha * pi);
    ri = (double)(VT)(ri - alpha * qi);  // the stored residual
    r[i] = (VT)ri;
    sx[le * NV + row] = ri;
    acc[0] = ri * ri;
  }
  __syncthreads();
  if (act) {
    const float* Pe = sP + le * NP;
    const int rr = row * (row + 1) / 2;
    double zi = 0.0;
#pragma unroll
    for (int col = 0; col < NV; ++col)
      zi += (double)Pe[row <= col ? col * (col + 1) / 2 + row : rr + col] * sx[le * NV + col];
    zi = (double)(VT)zi;  // the stored preconditioned residual
    z[i] = (VT)zi;
    acc[1] = ri * zi;
  }
  block_partials_to<2>(acc, partials, ngroups);
}

// Start of the FP32-vector CG (x = 0): r = (FP32) b, z = P_e r, p = z, and
// per element group the partial sums of r.r (slot 0) and r.z (slot 1), as
// in k_cg_update_blk.
template <int NV>
__global__ __launch_bounds__(256) void k_cg_init_blk(int64_t n_elem, const float* __restrict__ P,
                                                     const double* __restrict__ b, float* __restrict__ r,
                                                     float* __restrict__ z, float* __restrict__ p,
                                                     double* partials, int ngroups) {
  constexpr int EPB = 256 / NV, NP = NV * (NV + 1) / 2;
  constexpr int PPT = (EPB * NP + 255) / 256;
  __shared__ double sx[EPB * NV];
  __shared__ float sP[EPB * NP];
  const int le = threadIdx.x / NV, row = threadIdx.x % NV;
  const int64_t e0 = (int64_t)blockIdx.x * EPB;
  const int ne = (int)min((int64_t)EPB, n_elem - e0);
  const bool act = le < ne;
  const int64_t i = (e0 + le) * NV + row;
  const float* Pg = P + (size_t)e0 * NP;
  float pv[PPT];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int j = threadIdx.x + u * 256;
    pv[u] = j < ne * NP ? __builtin_nontemporal_load(&Pg[j]) : 0.0f;  // read once: non-temporal
  }
  const double ri = act ? (double)(float)b[i] : 0.0;
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int j = threadIdx.x + u * 256;
    if (j < ne * NP) sP[j] = pv[u];
  }
  double acc[2] = {0.0, 0.0};
  if (act) {
    r[i] = (float)ri;
    sx[le * NV + row] = ri;
    acc[0] = ri * ri;
  }
  __syncthreads();
  if (act) {
    const float* Pe = sP + le * NP;
    const int rr = row * (row + 1) / 2;
    double zi = 0.0;
#pragma unroll
    for (int col = 0; col < NV; ++col)
      zi += (double)Pe[row <= col ? col * (col + 1) / 2 + row : rr + col] * sx[le * NV + col];
    const float zf = (float)zi;
    z[i] = zf;
    p[i] = zf;
    acc[1] = ri * (double)zf;
  }
  block_partials_to<2>(acc, partials, ngroups);
}

// rz = (r.z) and rr_new = (r.r) from the init kernel's partials
__global__ __launch_bounds__(1024) void k_cg_init_blk_fin(const double* partials, int nblocks, DevScalars* sc) {
  __shared__ double sh[2][16];
  double v[2] = {0.0, 0.0};
  for (int b0 = threadIdx.x; b0 < nblocks; b0 += 8 * 1024) {
    double t[2][8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int b = b0 + u * 1024;
      t[0][u] = b < nblocks ? partials[b] : 0.0;
      t[1][u] = b < nblocks ? partials[nblocks + b] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      v[0] += t[0][u];
      v[1] += t[1][u];
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    v[j] = warp_sum(v[j]);
    if (lane == 0) sh[j][wid] = v[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double rr = 0.0, rz = 0.0;
    for (int w = 0; w < 16; ++w) {
      rr += sh[0][w];
      rz += sh[1][w];
    }
    sc->rr_new = rr;
    sc->rr = rz;
  }
}

__global__ void k_cg_p32(int64_t n, float* __restrict__ p, const float* __restrict__ z, const DevScalars* sc) {
  if (sc->cg_on == 0) return;
  const double beta = sc->beta;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (float)((double)z[i] + beta * (double)p[i]);
}

__global__ void k_fill_f32(int64_t n, float* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = 0.0f;
}

__global__ void k_f32_to_f64(int64_t n, const float* __restrict__ x, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}

// alpha = rz / pq, rr_new = r.r, beta = (r.z)_new / rz, rz = (r.z)_new from
// the fused update's partials (one workgroup, fixed summation order); then
// the device-side stop: count the iteration, copy (r.r, count) to cg_stat
// and clear cg_on once sqrt(r.r) <= cg_tol (the host's own test).
__global__ __launch_bounds__(1024) void k_cg_update_blk_fin(const double* partials, int nblocks, DevScalars* sc) {
  if (sc->cg_on == 0) return;
  __shared__ double sh[2][16];
  double v[2] = {0.0, 0.0};
  // 8 blocks per thread and slot in flight at once, added in a fixed order
  for (int b0 = threadIdx.x; b0 < nblocks; b0 += 8 * 1024) {
    double t[2][8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int b = b0 + u * 1024;
      t[0][u] = b < nblocks ? partials[b] : 0.0;
      t[1][u] = b < nblocks ? partials[nblocks + b] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      v[0] += t[0][u];
      v[1] += t[1][u];
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    v[j] = warp_sum(v[j]);
    if (lane == 0) sh[j][wid] = v[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double rr = 0.0, rz = 0.0;
    for (int w = 0; w < 16; ++w) {
      rr += sh[0][w];
      rz += sh[1][w];
    }
    sc->alpha = sc->rr / sc->pq;
    sc->rr_new = rr;
    sc->beta = rz / sc->rr;
    sc->rr = rz;
    const int it = sc->cg_iters + 1;
    sc->cg_iters = it;
    sc->cg_stat[0] = rr;
    sc->cg_stat[1] = (double)it;
    if (sqrt(rr) <= sc->cg_tol) sc->cg_on = 0;
  }
}

// Arms the device-side stop of a CG solve: tol = rtol ||b|| (negative: never
// stop on the device, for the loops without the fused update).
__global__ void k_cg_arm(DevScalars* sc, double tol) {
  sc->cg_tol = tol;
  sc->cg_on = 1;
  sc->cg_iters = 0;
  sc->cg_stat[0] = 0.0;
  sc->cg_stat[1] = 0.0;
}

// *out = sum of partials[0 .. nblocks) (one workgroup, fixed order): the
// inner product p . A p from the element kernel's per-workgroup sums.
// run (null: always): nothing is written while *run is 0.
__global__ __launch_bounds__(1024) void k_sum_partials(const double* partials, int nblocks, double* out,
                                                       const int* run) {
  if (run != nullptr && *run == 0) return;
  __shared__ double sh[16];
  double v = 0.0;
  for (int b0 = threadIdx.x; b0 < nblocks; b0 += 8 * 1024) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int b = b0 + u * 1024;
      t[u] = b < nblocks ? partials[b] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) v += t[u];
  }
  v = warp_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < 16; ++w) tot += sh[w];
    *out = tot;
  }
}

// The fused update for the element block size nv; false when there is no
// instantiation for it (the caller then runs the separate kernels).
template <typename VT>
static bool launch_cg_update_blk(Ctx& c, int nv, VT* x, VT* r, const VT* p, const VT* q, VT* z, hipStream_t s) {
  const int64_t n_elem = c.hs.n_elem;
  auto go = [&](auto kernel, int epb) {
    const int64_t groups = (n_elem + epb - 1) / epb;
    require(groups <= 0x7fffffff && c.d_cg_partials.n >= (size_t)(2 * groups), SDG_EINVAL,
            "fused CG update: element grid exceeds its partials");
    kernel<<<(unsigned)groups, 256, 0, s>>>(n_elem, c.d_Pblk.p, x, r, p, q, z, c.d_sc.p, c.d_cg_partials.p,
                                           (int)groups);
    check_launch();
    k_cg_update_blk_fin<<<1, 1024, 0, s>>>(c.d_cg_partials.p, (int)groups, c.d_sc.p);
    check_launch();
  };
#define SDG_CGB(NV_) \
  if (nv == NV_) { go(k_cg_update_blk<NV_, VT>, 256 / NV_); return true; }
  SDG_CGB(6) SDG_CGB(12) SDG_CGB(20) SDG_CGB(30) SDG_CGB(60) SDG_CGB(105)
#undef SDG_CGB
  return false;
}

// Preconditioned CG on FP32 vectors for the inner solves of iterative
// refinement (x = 0 on entry, FP32 operator, explicit element block
// preconditioner; the caller tests the FP64 residual afterwards): the
// iteration of solve_cg with r, p, q, z, x stored in FP32, which halves the
// vector traffic of the operator's gather and of the update kernels.  Inner
// products and scalars stay FP64.  x (FP64) receives the FP32 iterate.
static SolveResult solve_cg_f32(Ctx& c, const double* b, double* x, const KrylovCfg& k, hipStream_t s) {
  SolveResult res;
  const int64_t n = c.n_slab;
  const int nv = c.hs.dim * c.hs.nphi;
  const int64_t egroups = (c.hs.n_elem + 256 / nv - 1) / (256 / nv);
  if (c.d_cg32.n < (size_t)(5 * n)) c.d_cg32.alloc((size_t)(5 * n));
  if (c.d_cg_partials.n < (size_t)(2 * egroups)) c.d_cg_partials.alloc((size_t)(2 * egroups));
  float* r = c.d_cg32.p;
  float* pv = r + n;
  float* q = pv + n;
  float* z = q + n;
  float* x32 = z + n;
  DevScalars* sc = c.d_sc.p;
  const int check_every = std::max(1, k.check_every);
  res.bnorm = std::sqrt(vec_dot_host(c, n, b, b, s));
  require(std::isfinite(res.bnorm), SDG_ENONFINITE, "non-finite right-hand side");
  if (res.bnorm == 0.0) {
    vec_fill(n, 0.0, x, s);
    res.converged = true;
    return res;
  }
  k_fill_f32<<<vgrid(n), kThreads, 0, s>>>(n, x32);
  check_launch();
  bool started = false;
  auto go_init = [&](auto kernel) {
    kernel<<<(unsigned)egroups, 256, 0, s>>>(c.hs.n_elem, c.d_Pblk.p, b, r, z, pv, c.d_cg_partials.p,
                                            (int)egroups);
    check_launch();
    k_cg_init_blk_fin<<<1, 1024, 0, s>>>(c.d_cg_partials.p, (int)egroups, sc);
    check_launch();
    started = true;
  };
#define SDG_CGI(NV_) \
  if (nv == NV_) go_init(k_cg_init_blk<NV_>);
  SDG_CGI(6) SDG_CGI(12) SDG_CGI(20) SDG_CGI(30) SDG_CGI(60) SDG_CGI(105)
#undef SDG_CGI
  require(started, SDG_EUNSUPPORTED, "no FP32-vector CG kernel for this element size");
  double rr = read_scalar(c, &sc->rr_new, s);
  require(std::isfinite(rr), SDG_ENONFINITE, "non-finite residual");
  if (std::sqrt(rr) <= k.rtol * res.bnorm) {
    vec_fill(n, 0.0, x, s);
    res.converged = true;
    res.rel_res = std::sqrt(rr) / res.bnorm;
    return res;
  }
  // device_stop: the iterations queued past convergence (up to
  // check_every - 1) return at entry; res counts the ones that ran
  const int* run = k.device_stop ? &sc->cg_on : nullptr;
  k_cg_arm<<<1, 1, 0, s>>>(sc, k.device_stop ? k.rtol * res.bnorm : -1.0);
  check_launch();
  for (int it = 0; it < k.max_iter; ++it) {
    apply_op_f32v(c, pv, q, s, c.d_cg_partials.p, run);
    k_sum_partials<<<1, 1024, 0, s>>>(c.d_cg_partials.p, (int)egroups, &sc->pq, run);
    check_launch();
    launch_cg_update_blk<float>(c, nv, x32, r, pv, q, z, s);
    k_cg_p32<<<vgrid(n), kThreads, 0, s>>>(n, pv, z, sc);
    check_launch();
    if ((it + 1) % check_every == 0 || it + 1 == k.max_iter) {
      int ran = 0;
      rr = read_cg_stat(c, sc, s, ran);
      res.iters = ran;
      res.matvecs = ran;
      require(std::isfinite(rr), SDG_ENONFINITE, "non-finite residual");
      // fewer iterations ran than were queued: the device has stopped
      if (std::sqrt(rr) <= k.rtol * res.bnorm || ran < it + 1) break;
    }
  }
  k_f32_to_f64<<<vgrid(n), kThreads, 0, s>>>(n, x32, x);
  check_launch();
  res.rel_res = std::sqrt(rr) / res.bnorm;
  res.converged = res.rel_res <= k.rtol;
  return res;
}

// ---------------------------------------------------------------- CG

// Preconditioned conjugate gradients (P = I for SDG_PRECOND_NONE):
//   z = P^-1 r, p = z, rz = r.z;  per iteration
//   q = A p; alpha = rz / p.q; x += alpha p; r -= alpha q; z = P^-1 r;
//   beta = r.z_new / rz; p = z + beta p.
SolveResult solve_cg(Ctx& c, const double* b, double* x, const KrylovCfg& k, hipStream_t s) {
  // inner FP32 solves of iterative refinement on FP32 vectors
  if (k.prec == SDG_PREC_F32 && k.x_zero && k.recurrence_only && !k.transpose && k.precond == SDG_PRECOND_BLOCK &&
      !c.pblk_factored && c.d_Pblk.p != nullptr && c.n_slab == c.hs.n_elem * (int64_t)(c.hs.dim * c.hs.nphi) &&
      fp32_vectors_ok(c))
    return solve_cg_f32(c, b, x, k, s);
  SolveResult res;
  const int64_t n = c.n_slab;
  double* r = c.d_r.p;
  double* pv = c.d_w.p;
  double* q = c.d_t.p;
  double* z = c.d_V.p;  // first basis vector (always allocated) holds z = P^-1 r
  DevScalars* sc = c.d_sc.p;
  const bool pre = k.precond != SDG_PRECOND_NONE;
  // the explicit element block preconditioner (one time node, symmetric
  // blocks) is applied inside the fused update kernel
  const int nv = c.hs.ng * c.hs.dim * c.hs.nphi;
  // p . A p is summed by the operator's element kernel (one partial per
  // workgroup of 256 / nv elements) when the velocity is one time node
  const bool dotfused = n == c.hs.n_elem * (int64_t)nv && nv <= 256 && c.hs.ng == 1;
  const bool fused = dotfused && k.precond == SDG_PRECOND_BLOCK && !c.pblk_factored && c.d_Pblk.p != nullptr;
  const int64_t egroups = (c.hs.n_elem + 256 / nv - 1) / (256 / nv);
  if (dotfused) {  // partial sums per element group (two for the fused update)
    const size_t need = 2 * (size_t)egroups;
    if (c.d_cg_partials.n < need) c.d_cg_partials.alloc(need);
  }
  const int check_every = std::max(1, k.check_every);
  res.bnorm = std::sqrt(vec_dot_host(c, n, b, b, s));
  require(std::isfinite(res.bnorm), SDG_ENONFINITE, "non-finite right-hand side");
  if (res.bnorm == 0.0) {
    vec_fill(n, 0.0, x, s);
    res.converged = true;
    return res;
  }
  vec_copy(n, b, r, s);
  if (!k.x_zero) {  // with x = 0 the residual is b exactly
    apply_op(c, x, q, k.prec, k.transpose, s);
    ++res.matvecs;
    vec_axpby(n, -1.0, q, 1.0, r, s);
  }
  if (pre) {
    apply_precond(c, k.precond, r, z, k.transpose, s);
  } else {
    z = r;
  }
  vec_copy(n, z, pv, s);
  dev_dot(c, n, r, z, &sc->rr, s);  // rz
  double rr = read_scalar_dot(c, n, r, s);
  require(std::isfinite(rr), SDG_ENONFINITE, "non-finite residual");
  if (std::sqrt(rr) <= k.rtol * res.bnorm) {
    res.converged = true;
    res.rel_res = std::sqrt(rr) / res.bnorm;
    return res;
  }
  // device_stop with the fused update: the device stops the iteration, the
  // iterations queued past convergence (up to check_every - 1) return at
  // entry, and res counts the ones that ran.  Otherwise the host stops it.
  const bool dstop = fused && k.device_stop;
  const int* run = dstop ? &sc->cg_on : nullptr;
  const int matvecs0 = res.matvecs;
  k_cg_arm<<<1, 1, 0, s>>>(sc, dstop ? k.rtol * res.bnorm : -1.0);
  check_launch();
  for (int it = 0; it < k.max_iter; ++it) {
    if (dotfused) {
      apply_op(c, pv, q, k.prec, k.transpose, s, 1, nullptr, nullptr, c.d_cg_partials.p, run);
      k_sum_partials<<<1, 1024, 0, s>>>(c.d_cg_partials.p, (int)egroups, &sc->pq, run);
      check_launch();
    } else {
      apply_op(c, pv, q, k.prec, k.transpose, s);
      dev_dot(c, n, pv, q, &sc->pq, s);
    }
    ++res.matvecs;
    if (!(fused && launch_cg_update_blk(c, nv, x, r, pv, q, z, s))) {
      const unsigned g = red_grid(n);
      k_cg_update<<<g, kThreads, 0, s>>>(n, x, r, pv, q, sc, c.d_partials.p);
      check_launch();
      k_cg_update_fin<<<1, kThreads, 0, s>>>(c.d_partials.p, (int)g, sc, pre ? 0 : 1);
      check_launch();
      if (pre) {
        apply_precond(c, k.precond, r, z, k.transpose, s);
        k_dot<<<g, kThreads, 0, s>>>(n, r, z, c.d_partials.p);
        check_launch();
        k_dot_beta_fin<<<1, kThreads, 0, s>>>(c.d_partials.p, (int)g, sc);
        check_launch();
      }
    }
    k_cg_p<<<vgrid(n), kThreads, 0, s>>>(n, pv, z, sc);
    check_launch();
    ++res.iters;
    if ((it + 1) % check_every == 0 || it + 1 == k.max_iter) {
      bool stopped = false;  // fewer iterations ran than were queued
      if (fused) {
        int ran = 0;
        rr = read_cg_stat(c, sc, s, ran);
        res.iters = ran;
        res.matvecs = matvecs0 + ran;
        stopped = ran < it + 1;
      } else {
        rr = read_scalar(c, &sc->rr_new, s);
      }
      require(std::isfinite(rr), SDG_ENONFINITE, "non-finite residual");
      if (std::sqrt(rr) <= k.rtol * res.bnorm || stopped) break;
    }
  }
  if (k.recurrence_only) {  // rr: the last residual read (the start's without iterations)
    res.rel_res = std::sqrt(rr) / res.bnorm;
    res.converged = res.rel_res <= k.rtol;
    return res;
  }
  // true residual
  apply_op(c, x, q, k.prec, k.transpose, s);
  ++res.matvecs;
  vec_copy(n, b, r, s);
  vec_axpby(n, -1.0, q, 1.0, r, s);
  double tr = vec_dot_host(c, n, r, r, s);
  require(std::isfinite(tr), SDG_ENONFINITE, "non-finite residual");
  res.rel_res = std::sqrt(tr) / res.bnorm;
  res.converged = res.rel_res <= k.rtol;
  return res;
}

// ---------------------------------------------------------------- GMRES

// x += P^-1 V[0..kk) y after the triangular solve of a restart cycle.
static void gmres_correction(Ctx& c, int kk, double* x, const KrylovCfg& k, hipStream_t s) {
  const int64_t n = c.n_slab;
  const unsigned vg = vgrid(n);
  double* V = c.d_V.p;
  double* w = c.d_w.p;
  double* t = c.d_t.p;
  DevScalars* sc = c.d_sc.p;
  k_gmres_trisolve<<<1, 64, 0, s>>>(sc, kk);
  check_launch();
  if (k.precond != SDG_PRECOND_NONE) {
    if (kk > 0) launch_gs(Gs::UpdateSet, kk, vg, s, n, V, t, sc, nullptr);
    else vec_fill(n, 0.0, t, s);
    check_launch();
    apply_precond(c, k.precond, t, w, k.transpose, s);
    vec_axpby(n, 1.0, w, 1.0, x, s);
  } else {
    if (kk > 0) launch_gs(Gs::Update, kk, vg, s, n, V, x, sc, nullptr);
    check_launch();
  }
}

// Residual estimate of step j of the current delayed-GMRES cycle, whose
// finalize carried `stamp`: the device writes the estimate of step j into
// slot 1 + j and then the stamp into slot 0 of coherent pinned memory, so the
// host waits for that step without draining the stream and decides on that
// step's value alone (the same decision on every run).  Device errors end
// the wait.
static double load_acquire(const double* p) {
  const uint64_t bits = __atomic_load_n(reinterpret_cast<const uint64_t*>(p), __ATOMIC_ACQUIRE);
  double d;
  std::memcpy(&d, &bits, sizeof d);
  return d;
}

static double wait_poll(Ctx& c, int j, double stamp, hipStream_t s) {
  for (long spin = 1;; ++spin) {
    if (load_acquire(&c.h_poll[0]) >= stamp) return load_acquire(&c.h_poll[1 + j]);
    if (spin % 4096 == 0) {
      const hipError_t e = hipStreamQuery(s);
      if (e == hipSuccess) {
        require(load_acquire(&c.h_poll[0]) >= stamp, SDG_EDEVICE, "convergence poll: estimate not written");
        return load_acquire(&c.h_poll[1 + j]);
      }
      if (e != hipErrorNotReady) SDG_HIP(e);
    }
  }
}

// Restarted GMRES with right preconditioning and delayed
// reorthogonalisation (one reduction and two sweeps over the basis per
// step; see k_dmultidot).  Step j completes Hessenberg column j-1.  Every
// `check_every` steps the host reads the residual estimate of the step two
// steps back (wait_poll), so the device always has queued work while the
// host decides; a converged cycle ends with all columns complete so far.
static SolveResult solve_gmres_delayed(Ctx& c, const double* b, double* x, const KrylovCfg& k, hipStream_t s) {
  SolveResult res;
  const int64_t n = c.n_slab;
  const int m = std::max(1, std::min(k.restart, kMaxRestart));
  double* V = c.d_V.p;
  double* w = c.d_w.p;
  double* t = c.d_t.p;
  DevScalars* sc = c.d_sc.p;
  const bool pre = k.precond != SDG_PRECOND_NONE;
  const int check_every = std::max(1, k.check_every);
  res.bnorm = std::sqrt(vec_dot_host(c, n, b, b, s));
  require(std::isfinite(res.bnorm), SDG_ENONFINITE, "non-finite right-hand side");
  if (res.bnorm == 0.0) {
    vec_fill(n, 0.0, x, s);
    res.converged = true;
    return res;
  }
  const unsigned rg = red_grid(n), vg = vgrid(n);
  // the factored block preconditioner is fused into the update sweep
  const bool fuse_pre = k.precond == SDG_PRECOND_BLOCK && c.pblk_factored && c.d_Pq.p != nullptr;
  int total = 0;
  bool x_zero = k.x_zero;
  for (;;) {
    // r = b - A x is the first (unnormalised) basis vector of the cycle (b
    // itself while x is still the zero initial guess)
    if (x_zero) {
      vec_copy(n, b, V, s);
      x_zero = false;
    } else {
      apply_op(c, x, V, k.prec, k.transpose, s);
      ++res.matvecs;
      vec_axpby(n, 1.0, b, -1.0, V, s);
    }
    dev_dot(c, n, V, V, &sc->dots[0], s);
    double rr = read_scalar(c, &sc->dots[0], s);
    require(std::isfinite(rr), SDG_ENONFINITE, "non-finite residual");
    res.rel_res = std::sqrt(rr) / res.bnorm;
    if (debug_krylov()) std::fprintf(stderr, "[gmres] restart at it %d: true rel res %.3e\n", total, res.rel_res);
    if (res.rel_res <= k.rtol) { res.converged = true; break; }
    if (total >= k.max_iter) break;
    int j = 0, kk = -1;
    double stamps[kMaxRestart];
    bool t_ready = false;  // t already holds P^-1 of slot j (fused into the previous update)
    for (; j < m && total < k.max_iter; ++j) {
      double* uj = V + (size_t)j * n;
      if (pre) {
        if (!t_ready) apply_precond(c, k.precond, uj, t, k.transpose, s);
        apply_op(c, t, w, k.prec, k.transpose, s);
      } else {
        apply_op(c, uj, w, k.prec, k.transpose, s);
      }
      t_ready = false;
      ++res.matvecs;
      launch_dgs(Dg::Multidot, j, rg, s, n, V, w, sc, c.d_partials.p);
      check_launch();
      stamps[j] = ++c.poll_seq;
      launch_dgs(Dg::Fin, j, rg, s, n, V, w, sc, c.d_partials.p, c.d_poll, stamps[j]);
      check_launch();
      // the last step of a cycle also forms the partials that complete its column
      const bool last = j + 1 == m || total + 1 >= k.max_iter;
      if (last) {
        launch_dgs(Dg::UpdateDots, j, rg, s, n, V, w, sc, c.d_partials.p);
      } else if (fuse_pre) {
        // the next basis vector and its preconditioned image in one pass
        t_ready = launch_dupdate_pre(c.hs.n_elem, c.hs.ng, c.hs.dim * c.hs.nphi, j, n, V, w, sc, c.d_Pq.p,
                                     c.d_Pb.p, t, k.transpose, s);
        if (!t_ready) launch_dgs(Dg::Update, j, vg, s, n, V, w, sc, c.d_partials.p);
      } else {
        launch_dgs(Dg::Update, j, vg, s, n, V, w, sc, c.d_partials.p);
      }
      check_launch();
      ++total;
      ++res.iters;
      if (j >= 2 && j % check_every == 0) {
        // estimate of step j-2; after this step columns 0..j-1 are complete
        const double est = wait_poll(c, j - 2, stamps[j - 2], s);
        if (debug_krylov()) std::fprintf(stderr, "[gmres]   it %d est rel res %.3e\n", total, est / res.bnorm);
        require(std::isfinite(est), SDG_ENONFINITE, "non-finite residual estimate");
        if (est <= k.rtol * res.bnorm) { kk = j; break; }
      }
    }
    if (kk < 0) {
      // j steps taken: complete column j-1 from u_j (slot j), whose partials
      // the last step's update sweep formed
      launch_dgs(Dg::FinU, j, rg, s, n, V, nullptr, sc, c.d_partials.p);
      check_launch();
      kk = j;
    }
    gmres_correction(c, kk, x, k, s);
  }
  return res;
}

// Restarted GMRES with right preconditioning (A P^-1 u = b, x = P^-1 u), so
// the Arnoldi residual estimate is the true residual of the unpreconditioned
// system.  By default the delayed scheme above; otherwise classical
// Gram-Schmidt with a second projection in the same step when the DGKS test
// asks for it.
SolveResult solve_gmres(Ctx& c, const double* b, double* x, const KrylovCfg& k, hipStream_t s) {
  if (k.delayed) return solve_gmres_delayed(c, b, x, k, s);
  SolveResult res;
  const int64_t n = c.n_slab;
  const int m = std::max(1, std::min(k.restart, kMaxRestart));
  double* V = c.d_V.p;
  double* r = c.d_r.p;
  double* w = c.d_w.p;
  double* t = c.d_t.p;
  DevScalars* sc = c.d_sc.p;
  const bool pre = k.precond != SDG_PRECOND_NONE;
  const int check_every = std::max(1, k.check_every);
  res.bnorm = std::sqrt(vec_dot_host(c, n, b, b, s));
  require(std::isfinite(res.bnorm), SDG_ENONFINITE, "non-finite right-hand side");
  if (res.bnorm == 0.0) {
    vec_fill(n, 0.0, x, s);
    res.converged = true;
    return res;
  }
  const unsigned rg = red_grid(n), vg = vgrid(n);
  int total = 0;
  bool x_zero = k.x_zero;
  for (;;) {
    if (x_zero) {  // b - A 0 = b
      vec_copy(n, b, r, s);
      x_zero = false;
    } else {
      apply_op(c, x, r, k.prec, k.transpose, s);
      ++res.matvecs;
      vec_axpby(n, 1.0, b, -1.0, r, s);
    }
    dev_dot(c, n, r, r, &sc->dots[0], s);
    double rr = read_scalar(c, &sc->dots[0], s);
    require(std::isfinite(rr), SDG_ENONFINITE, "non-finite residual");
    res.rel_res = std::sqrt(rr) / res.bnorm;
    if (debug_krylov()) std::fprintf(stderr, "[gmres] restart at it %d: true rel res %.3e\n", total, res.rel_res);
    if (res.rel_res <= k.rtol) { res.converged = true; break; }
    if (total >= k.max_iter) break;
    k_gmres_start<<<1, 64, 0, s>>>(sc);
    check_launch();
    k_scale_into<<<vg, kThreads, 0, s>>>(n, r, V, &sc->inv_norm);
    check_launch();
    int kk = 0;
    for (int j = 0; j < m && total < k.max_iter; ++j) {
      double* vj = V + (size_t)j * n;
      if (pre) {
        apply_precond(c, k.precond, vj, t, k.transpose, s);
        apply_op(c, t, w, k.prec, k.transpose, s);
      } else {
        apply_op(c, vj, w, k.prec, k.transpose, s);
      }
      ++res.matvecs;
      launch_gs(Gs::Multidot, j + 1, rg, s, n, V, w, sc, c.d_partials.p);
      check_launch();
      launch_gs(Gs::H1Fin, j + 1, rg, s, n, V, w, sc, c.d_partials.p);
      check_launch();
      launch_gs(Gs::Pass, j + 1, rg, s, n, V, w, sc, c.d_partials.p);
      check_launch();
      launch_gs(Gs::H2Fin, j + 1, rg, s, n, V, w, sc, c.d_partials.p);
      check_launch();
      launch_gs(Gs::Final, j + 1, rg, s, n, V, w, sc, c.d_partials.p);
      check_launch();
      k_arnoldi_scale<<<rg, kThreads, 0, s>>>(n, c.d_partials.p, (int)rg, j + 1, sc, w, V + (size_t)(j + 1) * n);
      check_launch();
      ++total;
      ++res.iters;
      kk = j + 1;
      if ((j + 1) % check_every == 0 || j + 1 == m) {
        double est = read_scalar(c, &sc->resid, s);
        if (debug_krylov()) std::fprintf(stderr, "[gmres]   it %d est rel res %.3e\n", total, est / res.bnorm);
        require(std::isfinite(est), SDG_ENONFINITE, "non-finite residual estimate");
        if (est <= k.rtol * res.bnorm) break;
      }
    }
    gmres_correction(c, kk, x, k, s);
  }
  if (debug_krylov()) {
    double nr = 0.0;
    SDG_HIP(hipMemcpyAsync(&nr, &c.d_sc.p->n_reorth, sizeof(double), hipMemcpyDeviceToHost, s));
    SDG_HIP(hipStreamSynchronize(s));
    std::fprintf(stderr, "[gmres] second projections so far: %.0f\n", nr);
  }
  return res;
}

}  // namespace sdg
