// Host-side check of the library's L2 projection of initial data (no GPU):
// builds the host set-up of a mesh, then either writes the projection rule's
// points of every cell or projects values given at those points.
//
//   projection MESH 0 WHICH DEG OUT     OUT: int64 nq; double pts[n_cell][nq][dim], wts[n_cell][nq]
//   projection MESH 1 WHICH DEG IN OUT  IN: double values[n_cell][nq][comp];
//                                       OUT: double state[n_cell][comp][n_basis]
// MESH as for dual_basis.cpp; WHICH 0 = elements (comp = dim), 1 = dual
// elements (comp = n_sigma, canonical dual basis); DEG the rule's degree.
#include "../../paper_1802_04516_amd/csrc/setup.cpp"

#include <cstdio>
#include <cstdlib>

using namespace sdg;

static bool read_all(FILE* f, void* p, size_t bytes) { return std::fread(p, 1, bytes, f) == bytes; }

int main(int argc, char** argv) {
  if (argc < 6) {
    std::fprintf(stderr, "usage: projection MESH MODE WHICH DEG [IN] OUT\n");
    return 2;
  }
  const int mode = std::atoi(argv[2]), which = std::atoi(argv[3]), degree = std::atoi(argv[4]);
  if ((mode != 0 && mode != 1) || (which != 0 && which != 1) || argc != (mode == 0 ? 6 : 7)) return 2;
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
  const int64_t ncell = which == 0 ? hs.n_elem : hs.n_face;
  if (degree < projection_min_degree(hs, which)) return 2;
  const int64_t nq = projection_rule_size(hs, which, degree);
  bool ok = true;
  if (mode == 0) {
    std::vector<double> pts((size_t)(ncell * nq * dim)), wts((size_t)(ncell * nq));
    projection_points(hs, elem.data(), which, degree, pts.data(), wts.data());
    FILE* fo = std::fopen(argv[5], "wb");
    if (!fo) return 3;
    ok = std::fwrite(&nq, 8, 1, fo) == 1 && std::fwrite(pts.data(), 8, pts.size(), fo) == pts.size() &&
         std::fwrite(wts.data(), 8, wts.size(), fo) == wts.size();
    std::fclose(fo);
    return ok ? 0 : 3;
  }
  const int comp = which == 0 ? dim : hs.nsig;
  const int nb = which == 0 ? hs.nphi : hs.npsi;
  std::vector<double> vals((size_t)(ncell * nq * comp)), out((size_t)(ncell * comp * nb));
  FILE* fi = std::fopen(argv[5], "rb");
  if (!fi || !read_all(fi, vals.data(), vals.size() * 8)) return 3;
  std::fclose(fi);
  project_values(hs, elem.data(), which, degree, vals.data(), out.data());
  FILE* fo = std::fopen(argv[6], "wb");
  if (!fo) return 3;
  ok = std::fwrite(out.data(), 8, out.size(), fo) == out.size();
  std::fclose(fo);
  return ok ? 0 : 3;
}
