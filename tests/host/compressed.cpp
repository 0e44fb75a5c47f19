// Host-side check of the compressed 3D operator (no GPU): builds the host
// set-up of a mesh and the compressed operator, rebuilds every face side's
// block of eq. (MD_3) from it,
//   Dt[k][l][m] = sum_m' C[m][m'] (a_l F_f[k][m'] - sum_a B[a][l] G_f[k][a][m']),
// and prints the largest difference to the stored blocks relative to the
// largest block entry.
//
//   compressed MESH        (MESH as for dual_basis.cpp, dim 3)
#include "../../paper_1802_04516_amd/csrc/setup.cpp"

#include <cstdio>

using namespace sdg;

static bool read_all(FILE* f, void* p, size_t bytes) { return std::fread(p, 1, bytes, f) == bytes; }

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  FILE* fm = std::fopen(argv[1], "rb");
  if (!fm) return 3;
  int64_t hdr[6];
  if (!read_all(fm, hdr, sizeof hdr)) return 3;
  const int dim = (int)hdr[0], p = (int)hdr[3], pg = (int)hdr[5];
  const int64_t nvert = hdr[1], nelem = hdr[2];
  std::vector<double> xyz((size_t)(nvert * dim));
  std::vector<int64_t> elem((size_t)(nelem * (dim + 1)));
  std::vector<double> lam((size_t)nelem), mu((size_t)nelem), rho((size_t)nelem);
  if (!read_all(fm, xyz.data(), xyz.size() * 8) || !read_all(fm, elem.data(), elem.size() * 8) ||
      !read_all(fm, lam.data(), lam.size() * 8) || !read_all(fm, mu.data(), mu.size() * 8) ||
      !read_all(fm, rho.data(), rho.size() * 8))
    return 3;
  std::fclose(fm);
  const double period[3] = {1.0, 1.0, 1.0};
  HostSetup hs;
  CompressedOp co;
  try {
    build_host_setup(hs, dim, nvert, xyz.data(), nelem, elem.data(), hdr[4] ? period : nullptr, p, pg,
                     pg == 0 ? SDG_SCHEME_CN : SDG_SCHEME_STDG, 0.01, lam.data(), mu.data(), rho.data());
    build_compressed(hs, elem.data(), co);
  } catch (const Error& e) {
    std::fprintf(stderr, "set-up failed: %s\n", e.what());
    return 4;
  }
  const int nphi = hs.nphi, npsi = hs.npsi, blk = nphi * 3 * npsi;
  double worst = 0.0, scale = 0.0;
  for (double v : hs.Dt) scale = std::max(scale, std::fabs(v));
  for (int64_t j = 0; j < hs.n_face; ++j) {
    const FaceRec& fr = hs.faces[j];
    for (int s = 0; s < (fr.right >= 0 ? 2 : 1); ++s) {
      const int f = s == 0 ? fr.lf : fr.rf;
      const int64_t e = s == 0 ? fr.left : fr.right;
      const double* C = &co.C[((size_t)j * 2 + s) * npsi * npsi];
      const double* a = &co.fa[((size_t)j * 2 + s) * 3];
      const double* B = &co.eB[(size_t)e * 9];
      const double* D = &hs.Dt[((size_t)j * 2 + s) * blk];
      for (int k = 0; k < nphi; ++k)
        for (int l = 0; l < 3; ++l)
          for (int m = 0; m < npsi; ++m) {
            double v = 0.0;
            for (int mm = 0; mm < npsi; ++mm) {
              double t = a[l] * co.F[((size_t)f * nphi + k) * npsi + mm];
              for (int aa = 0; aa < 3; ++aa) t -= B[aa * 3 + l] * co.G[(((size_t)f * nphi + k) * 3 + aa) * npsi + mm];
              v += C[m * npsi + mm] * t;
            }
            worst = std::max(worst, std::fabs(v - D[(k * 3 + l) * npsi + m]));
          }
    }
  }
  std::printf("%.3e\n", worst / scale);
  return 0;
}
