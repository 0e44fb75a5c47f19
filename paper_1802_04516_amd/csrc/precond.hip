// Patch preconditioner Pre2 (Appendix A, eqs. APPRE1, APPRE2) on the GPU:
// y_i = sum_e A_i^-1(0, e) x_g(e), the stored first block row of the inverse
// of the velocity operator restricted to element i and its face neighbours.
#include "context.hpp"

namespace sdg {

namespace {

constexpr int kPatchThreads = 128;

// One workgroup per (element, column).  The stencil's velocity blocks are
// staged in LDS; thread r forms output row r from the element's block row,
// stored column-major (P[i][e][q][r]) so that the workgroup's loads of one
// column (e, q) are contiguous.
__global__ __launch_bounds__(kPatchThreads) void k_patch_apply(int64_t n_elem, int nb, int slots,
                                                             const float* __restrict__ P,
                                                             const int32_t* __restrict__ nbr,
                                                             const double* __restrict__ x, double* __restrict__ y,
                                                             int64_t cstride) {
  extern __shared__ double xs[];  // [slot][q]
  const int64_t i = blockIdx.x;
  const int64_t col = blockIdx.y;
  x += col * cstride;
  y += col * cstride;
  const int n = slots * nb;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const int e = t / nb, q = t % nb;
    const int32_t g = nbr[i * slots + e];
    xs[t] = g >= 0 ? x[(int64_t)g * nb + q] : 0.0;
  }
  __syncthreads();
  const float* __restrict__ Pi = P + i * (int64_t)n * nb;
  for (int r = threadIdx.x; r < nb; r += blockDim.x) {
    double acc = 0.0;
    for (int t = 0; t < n; ++t) acc += (double)Pi[(int64_t)t * nb + r] * xs[t];
    y[i * nb + r] = acc;
  }
}

}  // namespace

void launch_patch_apply(int64_t n_elem, int nb, int slots, const float* P, const int32_t* nbr, const double* x,
                        double* y, hipStream_t s, int ncols, int64_t cstride) {
  if (n_elem == 0) return;
  const size_t lds = (size_t)slots * nb * sizeof(double);
  k_patch_apply<<<dim3((unsigned)n_elem, (unsigned)ncols), kPatchThreads, lds, s>>>(n_elem, nb, slots, P, nbr, x, y,
                                                                                 cstride);
  SDG_HIP(hipGetLastError());
}

}  // namespace sdg
