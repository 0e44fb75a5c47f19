// Compile-time sizes of the operator blocks for (dimension, degree).
#pragma once

namespace sdg {

template <int D, int P>
struct Shape {
  static constexpr int NPHI = D == 2 ? (P + 1) * (P + 2) / 2 : (P + 1) * (P + 2) * (P + 3) / 6;
  static constexpr int NPSI = D == 2 ? (P + 1) * (P + 1) : NPHI;
  static constexpr int NSIG = D * (D + 1) / 2;
  static constexpr int BLK = NPHI * D * NPSI;  // one side's block [k][l][m]
};

// Voigt index of the symmetric tensor entry (c, l): 2D (xx, yy, xy),
// 3D (xx, yy, zz, yz, xz, xy).
template <int D>
__host__ __device__ constexpr int voigt(int c, int l) {
  if (c == l) return c;
  if (D == 2) return 2;
  return 6 - c - l;  // (1,2)->3, (0,2)->4, (0,1)->5
}
template <int D>
__host__ __device__ inline void voigt_pair(int sv, int& c, int& l) {
  if (sv < D) { c = l = sv; return; }
  if (D == 2) { c = 0; l = 1; return; }
  if (sv == 3) { c = 1; l = 2; } else if (sv == 4) { c = 0; l = 2; } else { c = 0; l = 1; }
}

// Faces staged per workgroup of the LDS face kernel (<= 48 KiB of LDS).
template <int D, int P, int NG, typename TD>
struct FacesPerBlock {
  using S = Shape<D, P>;
  static constexpr int per_face =
      (int)sizeof(TD) * (2 * S::BLK + 2 * NG * D * S::NPHI + 2 * NG * D * D * S::NPSI) + 24;
  static constexpr int raw = (48 * 1024) / per_face;
  static constexpr int value = raw < 1 ? 1 : (raw > 16 ? 16 : raw);
};

}  // namespace sdg
