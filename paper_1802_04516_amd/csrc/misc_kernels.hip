// Per-step kernels around the Krylov solve: initial guess, end-of-slab
// values, point sources (eq. MD_5_2), the energy of Section 5.2, point
// evaluation of velocity and stress, and the element-level pieces of the
// discrete adjoint (density gradient, face-to-element gradient gather,
// transpose of the receiver sampling).
#include "context.hpp"

namespace sdg {

namespace {
constexpr int kT = 256;
unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kT - 1) / kT, 65535)); }

// slab[e][a][q] = state[e][q] for every time node a
__global__ void k_broadcast(int64_t n_elem, int ng, int nvs, const double* __restrict__ st, double* __restrict__ sl) {
  const int64_t n = n_elem * ng * nvs;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i / (ng * nvs);
    const int q = (int)(i % nvs);
    sl[i] = st[e * nvs + q];
  }
}

// out[e][a][q] = sum_b Mt[a][b] in[e][b][q] (time-node mixing of a slab)
struct TimeMat { double m[kMaxGamma * kMaxGamma]; };
__global__ void k_time_map(int64_t n_elem, int ng, int nvs, TimeMat Mt, const double* __restrict__ in,
                           double* __restrict__ out) {
  const int64_t n = n_elem * ng * nvs;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i / (ng * nvs);
    const int r = (int)(i % (ng * nvs)), a = r / nvs, q = r % nvs;
    const double* ib = in + e * ng * nvs + q;
    double acc = 0.0;
    for (int b = 0; b < ng; ++b) acc += Mt.m[a * ng + b] * ib[b * nvs];
    out[i] = acc;
  }
}

// state[e][q] = sum_a w[a] slab[e][a][q]
__global__ void k_end(int64_t n_elem, int ng, int nvs, const double* __restrict__ w, const double* __restrict__ sl,
                      double* __restrict__ st) {
  const int64_t n = n_elem * nvs;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i / nvs;
    const int q = (int)(i % nvs);
    double acc = 0.0;
    for (int a = 0; a < ng; ++a) acc += w[a] * sl[(e * ng + a) * nvs + q];
    st[i] = acc;
  }
}

// b[e][a][c][k] += dt w_a amp[s][a] dir[s][c] phi[s][k]; one thread per
// (a, c, k) of each source, sources applied in order by one thread to keep
// the sum deterministic.
__global__ void k_sources(int64_t n_src, int ng, int dim, int nphi, double dt, const double* __restrict__ wq,
                          const int64_t* __restrict__ elem, const double* __restrict__ phi,
                          const double* __restrict__ dir, const double* __restrict__ amp, double* __restrict__ b) {
  const int per = ng * dim * nphi;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= per) return;
  const int k = t % nphi, c = (t / nphi) % dim, a = t / (nphi * dim);
  for (int64_t s = 0; s < n_src; ++s) {
    const int64_t e = elem[s];
    b[((e * ng + a) * dim + c) * nphi + k] += dt * wq[a] * amp[s * ng + a] * dir[s * dim + c] * phi[s * nphi + k];
  }
}

// Batched right-hand sides: column r (grid y) carries source r % n_src only.
__global__ void k_sources_cols(int64_t n_src, int ng, int dim, int nphi, double dt, const double* __restrict__ wq,
                               const int64_t* __restrict__ elem, const double* __restrict__ phi,
                               const double* __restrict__ dir, const double* __restrict__ amp, double* __restrict__ b,
                               int64_t cstride) {
  const int per = ng * dim * nphi;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= per) return;
  const int64_t r = blockIdx.y;
  const int64_t s = r % n_src;
  const int k = t % nphi, c = (t / nphi) % dim, a = t / (nphi * dim);
  const int64_t e = elem[s];
  b[r * cstride + ((e * ng + a) * dim + c) * nphi + k] +=
      dt * wq[a] * amp[s * ng + a] * dir[s * dim + c] * phi[s * nphi + k];
}

__device__ inline double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Partial energies per block -> partials[block]; k_energy_fin adds them.
template <int D>
__global__ void k_energy(int64_t n_elem, int64_t n_face, int nphi, int npsi, const double* __restrict__ Mref,
                         const int32_t* __restrict__ cidx, const double* __restrict__ cM,
                         const double* __restrict__ ew, const double* __restrict__ flm,
                         const double* __restrict__ fcw, const double* __restrict__ v,
                         const double* __restrict__ sig, double* partials) {
  constexpr int NS = D * (D + 1) / 2;
  __shared__ double sh[16];
  double acc = 0.0;
  const int64_t nk = n_elem * D;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nk + n_face; i += (int64_t)gridDim.x * blockDim.x) {
    if (i < nk) {
      const int64_t e = i / D;
      const double* vb = v + i * nphi;
      // a curved element's own mass matrix (Section 3 maps), else Mref
      const double* M = (cidx != nullptr && cidx[e] >= 0) ? cM + (int64_t)cidx[e] * nphi * nphi : Mref;
      double q = 0.0;
      for (int k = 0; k < nphi; ++k) {
        double mv = 0.0;
        for (int kk = 0; kk < nphi; ++kk) mv += M[k * nphi + kk] * vb[kk];
        q += vb[k] * mv;
      }
      acc += 0.5 * ew[e] * q;
    } else {
      const int64_t j = i - nk;
      const double lam = flm[2 * j], mu = flm[2 * j + 1];
      const double* sb = sig + j * NS * npsi;
      double q = 0.0;
      for (int m = 0; m < npsi; ++m) {
        double s[NS];
        for (int c = 0; c < NS; ++c) s[c] = sb[c * npsi + m];
        if (fcw != nullptr) {
          // anisotropic: s^T (W E~^-1) s with the face's compliance form
          const double* C = fcw + j * NS * NS;
          for (int a = 0; a < NS; ++a) {
            double t = 0.0;
            for (int b = 0; b < NS; ++b) t += C[a * NS + b] * s[b];
            q += s[a] * t;
          }
        } else if (D == 2) {
          const double den = 4.0 * mu * (lam + mu);
          const double a = (lam + 2.0 * mu) / den, b = -lam / den;
          q += a * (s[0] * s[0] + s[1] * s[1]) + 2.0 * b * s[0] * s[1] + s[2] * s[2] / mu;
        } else {
          const double alpha = 3.0 * lam + 2.0 * mu;
          const double f = 1.0 / (2.0 * mu * alpha);
          const double dg = 2.0 * (lam + mu) * f, off = -lam * f;
          q += dg * (s[0] * s[0] + s[1] * s[1] + s[2] * s[2]) +
               2.0 * off * (s[0] * s[1] + s[0] * s[2] + s[1] * s[2]) +
               (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]) / mu;
        }
      }
      acc += 0.5 * q;
    }
  }
  acc = wsum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    partials[blockIdx.x] = s;
  }
}

__global__ void k_energy_fin(const double* partials, int nblocks, double* out) {
  if (threadIdx.x < 64) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 64) v += partials[b];
    v = wsum(v);
    if (threadIdx.x == 0) *out = v;
  }
}

__global__ void k_sample(int64_t n, int nphi, int dim, const int64_t* __restrict__ elem, const double* __restrict__ phi,
                         const double* __restrict__ v, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * dim) return;
  const int64_t pt = t / dim;
  const int c = (int)(t % dim);
  const double* vb = v + (elem[pt] * dim + c) * nphi;
  double acc = 0.0;
  for (int k = 0; k < nphi; ++k) acc += phi[pt * nphi + k] * vb[k];
  out[t] = acc;
}

__global__ void k_eval_stress(int64_t n, int npsi, int nsig, const int64_t* __restrict__ face,
                              const double* __restrict__ psi, const double* __restrict__ sig, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nsig) return;
  const int64_t pt = t / nsig;
  const int s = (int)(t % nsig);
  const double* sb = sig + (face[pt] * nsig + s) * npsi;
  double acc = 0.0;
  for (int m = 0; m < npsi; ++m) acc += psi[pt * npsi + m] * sb[m];
  out[t] = acc;
}
// g[e] += |J_e| sum_{a,c,k} L[e][a][c][k] (Mref u_a)[c][k], with
// u_a = sum_b Bq[a][b] X[e][b] + Bo[a] vold[e]: the derivative of the slab
// system residual with respect to rho_e, contracted with the adjoint
// multipliers.  One thread per element.
__global__ void k_grad_rho(int64_t n_elem, int ng, int dim, int nphi, RhoCoefs tc, const double* __restrict__ Mref,
                           const double* __restrict__ detJ, const double* __restrict__ L,
                           const double* __restrict__ X, const double* __restrict__ vold, double* __restrict__ g) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_elem) return;
  const int nvs = dim * nphi;
  double acc = 0.0;
  for (int a = 0; a < ng; ++a)
    for (int c = 0; c < dim; ++c)
      for (int kk = 0; kk < nphi; ++kk) {
        // u_a[c][kk]
        double u = tc.Bo[a] * vold[e * nvs + c * nphi + kk];
        for (int b = 0; b < ng; ++b) u += tc.Bq[a * ng + b] * X[(e * ng + b) * nvs + c * nphi + kk];
        double lm = 0.0;
        const double* Lb = L + (e * ng + a) * nvs + c * nphi;
        for (int k = 0; k < nphi; ++k) lm += Lb[k] * Mref[k * nphi + kk];
        acc += lm * u;
      }
  g[e] += detJ[e] * acc;
}

// Per element: g_lam[e] += sum_f wt[e][f] fg[2 j(e,f)], g_mu likewise with
// fg[2 j + 1]; the face gradients of the dual-cell Lame parameters are
// distributed with the volume fractions that define them.
__global__ void k_face_to_elem(int64_t n_elem, int nfe, const int32_t* __restrict__ ef, const double* __restrict__ wt,
                               const double* __restrict__ fg, double* __restrict__ g_lam, double* __restrict__ g_mu) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_elem) return;
  double sl = 0.0, sm = 0.0;
  for (int f = 0; f < nfe; ++f) {
    const int64_t j = ef[e * nfe + f];
    const double w = wt[e * nfe + f];
    sl += w * fg[2 * j];
    sm += w * fg[2 * j + 1];
  }
  g_lam[e] += sl;
  g_mu[e] += sm;
}

// Transpose of point sampling: vbar[e_q][c][k] += phi_q[k] obar[q][c], the
// points taken in order so that the sum is deterministic.
__global__ void k_sample_adjoint(int64_t n, int nphi, int dim, const int64_t* __restrict__ elem,
                                 const double* __restrict__ phi, const double* __restrict__ obar,
                                 double* __restrict__ vbar) {
  const int t = threadIdx.x;
  if (t >= dim * nphi) return;
  const int c = t / nphi, k = t % nphi;
  for (int64_t q = 0; q < n; ++q) vbar[elem[q] * dim * nphi + t] += phi[q * nphi + k] * obar[q * dim + c];
}

}  // namespace

void launch_grad_rho(int64_t n_elem, int ng, int dim, int nphi, const RhoCoefs& tc, const double* Mref,
                     const double* detJ, const double* L, const double* X, const double* vold, double* g,
                     hipStream_t s) {
  k_grad_rho<<<(unsigned)((n_elem + kT - 1) / kT), kT, 0, s>>>(n_elem, ng, dim, nphi, tc, Mref, detJ, L, X, vold, g);
}

void launch_face_to_elem(int64_t n_elem, int nfe, const int32_t* ef, const double* wt, const double* fg,
                         double* g_lam, double* g_mu, hipStream_t s) {
  k_face_to_elem<<<(unsigned)((n_elem + kT - 1) / kT), kT, 0, s>>>(n_elem, nfe, ef, wt, fg, g_lam, g_mu);
}

void launch_sample_adjoint(int64_t n, int nphi, int dim, const int64_t* elem, const double* phi,
                           const double* obar, double* vbar, hipStream_t s) {
  k_sample_adjoint<<<1, 256, 0, s>>>(n, nphi, dim, elem, phi, obar, vbar);
}

void launch_time_map(int64_t n_elem, int ng, int nvs, const double* Mt, const double* in, double* out,
                     hipStream_t s) {
  TimeMat t{};
  for (int i = 0; i < ng * ng; ++i) t.m[i] = Mt[i];
  const int64_t n = n_elem * ng * nvs;
  k_time_map<<<grid_for(n), kT, 0, s>>>(n_elem, ng, nvs, t, in, out);
  SDG_HIP(hipGetLastError());
}

void launch_broadcast_time(int64_t n_elem, int ng, int nvs, const double* state, double* slab, hipStream_t s) {
  k_broadcast<<<grid_for(n_elem * ng * nvs), kT, 0, s>>>(n_elem, ng, nvs, state, slab);
  SDG_HIP(hipGetLastError());
}

void launch_end_of_slab(int64_t n_elem, int ng, int nvs, const double* w, const double* slab, double* state,
                        hipStream_t s) {
  k_end<<<grid_for(n_elem * nvs), kT, 0, s>>>(n_elem, ng, nvs, w, slab, state);
  SDG_HIP(hipGetLastError());
}

void launch_add_sources(Ctx& c, double* b, const double* amp_dev, hipStream_t s, int ncols) {
  if (c.n_src == 0) return;
  const HostSetup& hs = c.hs;
  require(c.p_src == c.p && (int64_t)c.src_elem.size() == c.n_src &&
              c.src_phi.size() == (size_t)c.n_src * hs.nphi,
          SDG_ESTATE, "sources were located for another mesh or degree; set them again");
  for (int64_t e : c.src_elem)
    require(e >= 0 && e < hs.n_elem, SDG_ESTATE, "source element outside the mesh; set the sources again");
  const int per = hs.ng * hs.dim * hs.nphi;
  if (ncols > 1) {
    k_sources_cols<<<dim3((per + kT - 1) / kT, ncols), kT, 0, s>>>(c.n_src, hs.ng, hs.dim, hs.nphi, hs.dt, c.d_tw.p,
                                                                   c.d_src_elem.p, c.d_src_phi.p, c.d_src_dir.p,
                                                                   amp_dev, b, c.n_slab);
    SDG_HIP(hipGetLastError());
    return;
  }
  // quadrature weights of the slab's time nodes (Crank-Nicolson: midpoint, weight 1)
  k_sources<<<(per + kT - 1) / kT, kT, 0, s>>>(c.n_src, hs.ng, hs.dim, hs.nphi, hs.dt, c.d_tw.p,
                                              c.d_src_elem.p, c.d_src_phi.p, c.d_src_dir.p, amp_dev, b);
  SDG_HIP(hipGetLastError());
}

void launch_energy(Ctx& c, const double* v, const double* sig, double* out_dev, hipStream_t s, int64_t e0,
                   int64_t ne, int64_t f0, int64_t nf) {
  const HostSetup& hs = c.hs;
  if (ne < 0) ne = hs.n_elem - e0;
  if (nf < 0) nf = hs.n_face - f0;
  const int64_t n = ne * hs.dim + nf;
  unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kT - 1) / kT, kRedBlocks));
  const double* vv = v + e0 * hs.dim * hs.nphi;
  const double* ss = sig + f0 * hs.nsig * hs.npsi;
  if (hs.dim == 2)
    k_energy<2><<<g, kT, 0, s>>>(ne, nf, hs.nphi, hs.npsi, c.d_Mref.p, c.d_curved_idx.p ? c.d_curved_idx.p + e0 : nullptr,
                                 c.d_curved_M.p, c.d_elem_w.p + e0, c.d_face_lm.p + 2 * f0,
                                 c.d_face_Cw.p ? c.d_face_Cw.p + f0 * hs.nsig * hs.nsig : nullptr, vv,
                                 ss, c.d_partials.p);
  else
    k_energy<3><<<g, kT, 0, s>>>(ne, nf, hs.nphi, hs.npsi, c.d_Mref.p, nullptr, nullptr, c.d_elem_w.p + e0,
                                 c.d_face_lm.p + 2 * f0,
                                 c.d_face_Cw.p ? c.d_face_Cw.p + f0 * hs.nsig * hs.nsig : nullptr, vv,
                                 ss, c.d_partials.p);
  SDG_HIP(hipGetLastError());
  k_energy_fin<<<1, 64, 0, s>>>(c.d_partials.p, (int)g, out_dev);
  SDG_HIP(hipGetLastError());
}

void launch_sample(int64_t n, int nphi, int dim, const int64_t* elem, const double* phi, const double* v,
                   double* out, hipStream_t s) {
  if (n == 0) return;
  k_sample<<<(unsigned)((n * dim + kT - 1) / kT), kT, 0, s>>>(n, nphi, dim, elem, phi, v, out);
  SDG_HIP(hipGetLastError());
}

void launch_eval_stress(int64_t n, int npsi, int nsig, const int64_t* face, const double* psi, const double* sig,
                        double* out, hipStream_t s) {
  if (n == 0) return;
  k_eval_stress<<<(unsigned)((n * nsig + kT - 1) / kT), kT, 0, s>>>(n, npsi, nsig, face, psi, sig, out);
  SDG_HIP(hipGetLastError());
}

}  // namespace sdg
