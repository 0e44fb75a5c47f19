// Wavefront and workgroup reductions shared by the Krylov kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace sdg {

constexpr int pow2ceil(int x) { return x <= 1 ? 1 : 2 * pow2ceil((x + 1) / 2); }

// One butterfly exchange of a wavefront reduce-scatter (offset O, CNT
// accumulators left): a lane keeps one half of its accumulators, sends the
// other half to lane ^ O and adds what it receives; lanes with bit O set
// keep the upper half (their slot base moves up by CNT / 2).  With one
// accumulator left the exchange is a plain butterfly sum.
template <int CNT, int O>
__device__ inline void bfly(double* v, int lane, int& base) {
  if constexpr (O > 0) {
    if constexpr (CNT > 1) {
      constexpr int H = CNT / 2;
      const bool up = (lane & O) != 0;
#pragma unroll
      for (int i = 0; i < H; ++i) {
        const double send = up ? v[i] : v[i + H];
        const double keep = up ? v[i + H] : v[i];
        v[i] = keep + __shfl_xor(send, O, 64);
      }
      if (up) base += H;
      bfly<H, O / 2>(v, lane, base);
    } else {
      v[0] += __shfl_xor(v[0], O, 64);
      bfly<1, O / 2>(v, lane, base);
    }
  }
}

// Wavefront sums of NS (<= 64) accumulators by a butterfly reduce-scatter
// over the six lane offsets 32 .. 1: about NSP values move per lane (NSP =
// NS rounded up to a power of two) instead of 6 NS for one shuffle tree per
// accumulator.  Afterwards lane l holds the sum of accumulator `slot` =
// l / (64 / NSP) in v[0] and `first` tells whether it is the lowest lane
// holding that slot.
template <int NS>
__device__ inline double wave_reduce_scatter(const double (&acc)[NS], int lane, int& slot, bool& first) {
  constexpr int NSP = pow2ceil(NS), REP = 64 / NSP;
  static_assert(NSP <= 64, "at most 64 accumulators per wavefront reduction");
  double v[NSP];
#pragma unroll
  for (int i = 0; i < NSP; ++i) v[i] = i < NS ? acc[i] : 0.0;
  slot = 0;
  bfly<NSP, 32>(v, lane, slot);
  first = lane % REP == 0 && slot < NS;
  return v[0];
}

// Per-block sums of NS (<= 64) accumulators -> partials[i * stride + block]
// (slot-major): the wavefront reduce-scatter above, then the waves' sums
// added in wave order, so the result is deterministic.
template <int NS>
__device__ inline void block_partials_to(const double (&acc)[NS], double* partials, int stride) {
  constexpr int NSP = pow2ceil(NS);
  __shared__ double shp[16 * NSP];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int slot;
  bool first;
  const double v = wave_reduce_scatter<NS>(acc, lane, slot, first);
  if (first) shp[wid * NSP + slot] = v;
  __syncthreads();
  if (threadIdx.x < NS) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += shp[w * NSP + threadIdx.x];
    partials[(size_t)threadIdx.x * stride + blockIdx.x] = t;
  }
}

}  // namespace sdg
