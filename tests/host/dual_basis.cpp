// Host-side check of the library's set-up code (no GPU): builds the host
// set-up of a mesh and writes the canonical dual basis of every face,
// evaluated at given points, so that a test can compare it with the
// oracle's Gram-Schmidt basis.
//
//   dual_basis MESH POINTS OUT [FACES BLOCKS DATA]
// MESH:   int64 dim, n_vert, n_elem, p, periodic, p_gamma; double xyz[n_vert][dim];
//         int64 elem[n_elem][dim + 1] (periodic: unit period in every axis);
//         double lambda[n_elem], mu[n_elem], rho[n_elem]
// POINTS: int64 K; double x[n_face][K][dim] (in the left element's frame)
// OUT:    double psi[n_face][K][n_psi]
// FACES:  int32 [n_face][4] = left, local face in left, right (-1 on the
//         boundary), local face in right
// BLOCKS: double Dt[n_face][2][N_phi][d][N_psi] (canonical dual basis; zero
//         for the missing side of a boundary face)
// DATA:   double face_lm[n_face][2], elem_w[n_elem], Mref[N_phi][N_phi],
//         tau[N_g], w[N_g], e0[N_g], e1[N_g], T[N_g][N_g]
#include "../../paper_1802_04516_amd/csrc/setup.cpp"

#include <cstdio>

using namespace sdg;

static bool read_all(FILE* f, void* p, size_t bytes) { return std::fread(p, 1, bytes, f) == bytes; }

int main(int argc, char** argv) {
  if (argc != 4 && argc != 7) {
    std::fprintf(stderr, "usage: dual_basis MESH POINTS OUT [FACES BLOCKS DATA]\n");
    return 2;
  }
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
  try {
    build_host_setup(hs, dim, nvert, xyz.data(), nelem, elem.data(), hdr[4] ? period : nullptr, p, pg,
                     pg == 0 ? SDG_SCHEME_CN : SDG_SCHEME_STDG, 0.01, lam.data(), mu.data(), rho.data());
  } catch (const Error& e) {
    std::fprintf(stderr, "set-up failed: %s\n", e.what());
    return 4;
  }
  FILE* fp = std::fopen(argv[2], "rb");
  if (!fp) return 3;
  int64_t K = 0;
  if (!read_all(fp, &K, 8)) return 3;
  std::vector<double> pts((size_t)(hs.n_face * K * dim));
  if (!read_all(fp, pts.data(), pts.size() * 8)) return 3;
  std::fclose(fp);
  std::vector<double> out((size_t)(hs.n_face * K * hs.npsi));
  for (int64_t j = 0; j < hs.n_face; ++j) {
    FaceGeom fg;
    face_geometry(hs, elem.data(), j, fg);
    DualBasis db(dim, p);
    double vol[2];
    build_dual(hs, j, fg, db, vol);
    for (int64_t q = 0; q < K; ++q) db.canonical(&pts[(size_t)((j * K + q) * dim)], &out[(size_t)((j * K + q) * hs.npsi)]);
  }
  FILE* fo = std::fopen(argv[3], "wb");
  if (!fo) return 3;
  bool ok = std::fwrite(out.data(), 8, out.size(), fo) == out.size();
  std::fclose(fo);
  if (ok && argc == 7) {
    FILE* ff = std::fopen(argv[4], "wb");
    if (!ff) return 3;
    for (const FaceRec& r : hs.faces) {
      const int32_t rec[4] = {r.left, r.lf, r.right, r.rf};
      ok = ok && std::fwrite(rec, 4, 4, ff) == 4;
    }
    std::fclose(ff);
    FILE* fb = std::fopen(argv[5], "wb");
    if (!fb) return 3;
    ok = ok && std::fwrite(hs.Dt.data(), 8, hs.Dt.size(), fb) == hs.Dt.size();
    std::fclose(fb);
    FILE* fd = std::fopen(argv[6], "wb");
    if (!fd) return 3;
    for (const std::vector<double>* v : {&hs.face_lm, &hs.elem_w, &hs.Mref, &hs.tau, &hs.w, &hs.e0, &hs.e1, &hs.T})
      ok = ok && std::fwrite(v->data(), 8, v->size(), fd) == v->size();
    std::fclose(fd);
  }
  return ok ? 0 : 3;
}
