// Host-side setup: topology, geometry, bases, exact quadrature and the
// operator blocks of the staggered space-time DG scheme (Section 3 and
// eqs. (MD_2)-(MD_6) of Section 4).  Runs once per mesh / material / dt.
//
// Blocks are stored per face and side in the canonical orthonormal dual
// basis (Gram-Schmidt of the raw dual sequence over the dual element), so
// the dual mass matrices are the identity and the Schur complement needs no
// inverse mass:
//   Dt[j][side][k][l][m] = int_{Gamma_j} phi_k psi_m (n_{i,j})_l
//                          - int_{T_{i,j}} d_l phi_k psi_m,
// with the face term dropped on free-surface faces (sigma.n = 0).
#include <algorithm>
#include <atomic>
#include <mutex>
#include <thread>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "sdg_internal.hpp"

namespace sdg {
namespace {

// ---------------------------------------------------------------- 1D rules

// Gauss-Legendre nodes/weights on [0,1] by Newton iteration on the
// three-term recurrence of the Legendre polynomials.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
  }
  // ascending order
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return x[a] < x[b]; });
  std::vector<double> xs(n), ws(n);
  for (int i = 0; i < n; ++i) { xs[i] = x[idx[i]]; ws[i] = w[idx[i]]; }
  x = xs;
  w = ws;
}

// Rule on an affine k-simplex embedded in d-space (k = rows-1), exact for
// polynomials of total degree <= deg.  Collapsed (Duffy) coordinates with
// Gauss-Legendre factors and the Jacobian written out:
//   k=2: xi = u, eta = (1-u) v,                 J = (1-u)
//   k=3: xi = u, eta = (1-u) v, zeta = (1-u)(1-v) w,  J = (1-u)^2 (1-v)
struct Rule {
  std::vector<double> x;  // npts*d
  std::vector<double> w;
  int d = 0;
  int n() const { return (int)w.size(); }
};

Rule simplex_rule(const double* V, int k, int d, int deg) {
  Rule r;
  r.d = d;
  int n = deg / 2 + 2;  // handles the extra Jacobian degrees
  std::vector<double> gx, gw;
  gauss_legendre(n, gx, gw);
  // measure of the simplex relative to the reference one
  double J[9] = {0};
  for (int a = 0; a < k; ++a)
    for (int c = 0; c < d; ++c) J[c * k + a] = V[(a + 1) * d + c] - V[c];
  double vol;
  if (k == d) {
    if (d == 1) vol = std::fabs(J[0]);
    else if (d == 2) vol = std::fabs(J[0] * J[3] - J[1] * J[2]);
    else
      vol = std::fabs(J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                      J[2] * (J[3] * J[7] - J[4] * J[6]));
  } else if (k == 1) {
    double s = 0;
    for (int c = 0; c < d; ++c) s += J[c * k] * J[c * k];
    vol = std::sqrt(s);
  } else {  // k = 2 in 3D: |t1 x t2|
    double t1[3] = {J[0], J[2], J[4]}, t2[3] = {J[1], J[3], J[5]};
    double cx = t1[1] * t2[2] - t1[2] * t2[1], cy = t1[2] * t2[0] - t1[0] * t2[2],
           cz = t1[0] * t2[1] - t1[1] * t2[0];
    vol = std::sqrt(cx * cx + cy * cy + cz * cz);
  }
  auto push = [&](const double* ref, double wt) {
    for (int c = 0; c < d; ++c) {
      double s = V[c];
      for (int a = 0; a < k; ++a) s += J[c * k + a] * ref[a];
      r.x.push_back(s);
    }
    r.w.push_back(wt * vol);
  };
  if (k == 1) {
    for (int i = 0; i < n; ++i) push(&gx[i], gw[i]);
  } else if (k == 2) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double ref[2] = {gx[i], (1.0 - gx[i]) * gx[j]};
        push(ref, gw[i] * gw[j] * (1.0 - gx[i]));
      }
  } else {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        for (int l = 0; l < n; ++l) {
          double u = gx[i], v = gx[j], t = gx[l];
          double ref[3] = {u, (1.0 - u) * v, (1.0 - u) * (1.0 - v) * t};
          push(ref, gw[i] * gw[j] * gw[l] * (1.0 - u) * (1.0 - u) * (1.0 - v));
        }
  }
  return r;
}

// Dynamic parallel loop over [0, n) on the host cores.
template <class F>
void parallel_for(int64_t n, F&& fn) {
  unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  if (const char* omp = std::getenv("OMP_NUM_THREADS")) {
    const int k = std::atoi(omp);
    if (k > 0) nt = std::min(nt, (unsigned)k);
  }
  if (n < 256) nt = 1;
  std::atomic<int64_t> next{0};
  auto worker = [&]() {
    const int64_t chunk = 64;
    for (;;) {
      int64_t b = next.fetch_add(chunk);
      if (b >= n) break;
      int64_t e = std::min(n, b + chunk);
      for (int64_t i = b; i < e; ++i) fn(i);
    }
  };
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nt; ++t) th.emplace_back(worker);
  worker();
  for (auto& t : th) t.join();
}

// ---------------------------------------------------------------- velocity basis

// Equispaced Lagrange basis in Silvester's barycentric product form:
// phi_alpha = prod_a R_{alpha_a}(lambda_a), R_m(z) = prod_{s<m} (p z - s)/(s+1).
struct VelBasis {
  int dim, p, n;
  std::vector<std::array<int, 4>> alpha;  // barycentric multi-indices, pinned order

  VelBasis(int d, int pp) : dim(d), p(pp) {
    if (d == 2) {
      for (int j = 0; j <= p; ++j)
        for (int i = 0; i <= p - j; ++i) alpha.push_back({p - i - j, i, j, 0});
    } else {
      for (int kk = 0; kk <= p; ++kk)
        for (int j = 0; j <= p - kk; ++j)
          for (int i = 0; i <= p - kk - j; ++i) alpha.push_back({p - i - j - kk, i, j, kk});
    }
    n = (int)alpha.size();
  }

  static void R(int m, int p, double z, double& val, double& der) {
    val = 1.0;
    der = 0.0;
    for (int s = 0; s < m; ++s) {
      double f = (p * z - s) / (s + 1.0);
      double df = p / (s + 1.0);
      der = der * f + val * df;
      val *= f;
    }
  }

  // values (n) and reference gradients (n*dim, [k][b]) at reference point xi
  void eval(const double* xi, double* val, double* grad) const {
    double lam[4];
    lam[0] = 1.0;
    for (int b = 0; b < dim; ++b) { lam[b + 1] = xi[b]; lam[0] -= xi[b]; }
    for (int k = 0; k < n; ++k) {
      double rv[4], rd[4];
      for (int a = 0; a <= dim; ++a) R(alpha[k][a], p, lam[a], rv[a], rd[a]);
      double v = 1.0;
      for (int a = 0; a <= dim; ++a) v *= rv[a];
      val[k] = v;
      if (grad) {
        // d/dxi_b: lambda_0 decreases, lambda_{b+1} increases
        for (int b = 0; b < dim; ++b) {
          double t0 = rd[0], tb = rd[b + 1];
          for (int a = 0; a <= dim; ++a) {
            if (a != 0) t0 *= rv[a];
            if (a != b + 1) tb *= rv[a];
          }
          grad[k * dim + b] = tb - t0;
        }
      }
    }
  }
};

// ---------------------------------------------------------------- small linear algebra

// Solve A X = B in place (A n x n row-major, B n x m), partial pivoting.
void solve_dense(std::vector<double> A, std::vector<double>& B, int n, int m) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    require(std::fabs(A[piv * n + c]) > 0.0, SDG_EMESH, "singular matrix in setup");
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
      for (int k = 0; k < m; ++k) std::swap(B[c * m + k], B[piv * m + k]);
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = A[r * n + c] / A[c * n + c];
      if (f == 0.0) continue;
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      for (int k = 0; k < m; ++k) B[r * m + k] -= f * B[c * m + k];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int k = 0; k < m; ++k) B[r * m + k] /= A[r * n + r];
}

// Orthonormalisation of the raw dual sequence from its values: A (nq x n,
// row-major) holds sqrt(w_q) raw_k(x_q) for an exact rule, so A^T A is the
// Gram matrix.  Householder QR, A = Q R with diag(R) > 0, gives the
// canonical functions raw R^{-1}; returns Li = R^{-T} (lower triangular,
// canonical_i = sum_{k<=i} Li[i][k] raw_k).  Same result as Gram-Schmidt of
// the sequence (hence as the Cholesky factor of A^T A) in exact arithmetic,
// but the orthonormality error of the computed functions is eps cond(A)
// instead of eps cond(A)^2.
std::vector<double> orthonormaliser(std::vector<double> A, int nq, int n) {
  require(nq >= n, SDG_EMESH, "dual Gram rule has too few points");
  std::vector<double> v(nq);
  for (int j = 0; j < n; ++j) {
    double nrm = 0.0, scale = 0.0;
    for (int i = j; i < nq; ++i) scale = std::max(scale, std::fabs(A[i * n + j]));
    require(scale > 0.0, SDG_EMESH, "dual basis functions are linearly dependent");
    for (int i = j; i < nq; ++i) {
      double t = A[i * n + j] / scale;
      nrm += t * t;
    }
    nrm = scale * std::sqrt(nrm);
    const double alpha = A[j * n + j] > 0 ? -nrm : nrm;
    double vv = 0.0;
    for (int i = j; i < nq; ++i) {
      v[i] = A[i * n + j] - (i == j ? alpha : 0.0);
      vv += v[i] * v[i];
    }
    if (vv > 0.0) {
      for (int k = j; k < n; ++k) {
        double s = 0.0;
        for (int i = j; i < nq; ++i) s += v[i] * A[i * n + k];
        s *= 2.0 / vv;
        for (int i = j; i < nq; ++i) A[i * n + k] -= s * v[i];
      }
    }
  }
  // R = upper triangle of A with rows scaled to a positive diagonal
  std::vector<double> R(n * n, 0.0);
  double rmax = 0.0;
  for (int j = 0; j < n; ++j) rmax = std::max(rmax, std::fabs(A[j * n + j]));
  for (int j = 0; j < n; ++j) {
    const double sg = A[j * n + j] < 0 ? -1.0 : 1.0;
    require(std::fabs(A[j * n + j]) > 1e-14 * rmax, SDG_EMESH, "dual Gram matrix not positive definite");
    for (int k = j; k < n; ++k) R[j * n + k] = sg * A[j * n + k];
  }
  std::vector<double> Li(n * n, 0.0);
  for (int c = 0; c < n; ++c) {  // column c of R^{-1} by back substitution = row c of Li
    Li[c * n + c] = 1.0 / R[c * n + c];
    for (int i = c - 1; i >= 0; --i) {
      double s = 0.0;
      for (int k = i + 1; k <= c; ++k) s += R[i * n + k] * Li[c * n + k];
      Li[c * n + i] = -s / R[i * n + i];
    }
  }
  return Li;
}

double legendre(int n, double x) {
  double p0 = 1.0, p1 = x;
  if (n == 0) return 1.0;
  for (int k = 2; k <= n; ++k) {
    double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  return p1;
}

// ---------------------------------------------------------------- dual basis

// Raw dual basis of one face: 2D Legendre products in the quad frame
// (lexicographic, a major); 3D Legendre products in scaled physical
// coordinates ordered by total degree, then a, b descending.  Both share the
// nested spans of the monomial sequences that define the canonical basis.
struct DualBasis {
  int dim, p, n;
  std::vector<std::array<int, 3>> ex;
  double origin[3];
  double Ainv[9];  // frame coordinates = Ainv (x - origin)
  std::vector<double> Linv;  // canonical = Linv * raw

  DualBasis(int d, int pp) : dim(d), p(pp) {
    if (d == 2) {
      for (int a = 0; a <= p; ++a)
        for (int b = 0; b <= p; ++b) ex.push_back({a, b, 0});
    } else {
      for (int deg = 0; deg <= p; ++deg)
        for (int a = deg; a >= 0; --a)
          for (int b = deg - a; b >= 0; --b) ex.push_back({a, b, deg - a - b});
    }
    n = (int)ex.size();
  }

  void raw(const double* x, double* out) const {
    double y[3];
    for (int r = 0; r < dim; ++r) {
      double s = 0;
      for (int c = 0; c < dim; ++c) s += Ainv[r * dim + c] * (x[c] - origin[c]);
      y[r] = s;
    }
    if (dim == 2) { y[0] = 2.0 * y[0] - 1.0; y[1] = 2.0 * y[1] - 1.0; }
    double L[3][8];
    for (int r = 0; r < dim; ++r)
      for (int q = 0; q <= p; ++q) L[r][q] = legendre(q, y[r]);
    for (int m = 0; m < n; ++m) {
      double v = 1.0;
      for (int r = 0; r < dim; ++r) v *= L[r][ex[m][r]];
      out[m] = v;
    }
  }

  void canonical(const double* x, double* out) const {
    double r[64];
    raw(x, r);
    for (int i = 0; i < n; ++i) {
      double s = 0;
      for (int k = 0; k <= i; ++k) s += Linv[i * n + k] * r[k];
      out[i] = s;
    }
  }
};

// ---------------------------------------------------------------- helpers

double det_and_inverse(const double* V, int d, double* Jinv) {
  // J columns = V[a+1]-V[0]; returns det J and J^{-1} (row-major)
  double J[9];
  for (int c = 0; c < d; ++c)
    for (int a = 0; a < d; ++a) J[c * d + a] = V[(a + 1) * d + c] - V[c];
  if (d == 2) {
    double det = J[0] * J[3] - J[1] * J[2];
    Jinv[0] = J[3] / det; Jinv[1] = -J[1] / det;
    Jinv[2] = -J[2] / det; Jinv[3] = J[0] / det;
    return det;
  }
  double c00 = J[4] * J[8] - J[5] * J[7], c01 = J[5] * J[6] - J[3] * J[8], c02 = J[3] * J[7] - J[4] * J[6];
  double det = J[0] * c00 + J[1] * c01 + J[2] * c02;
  Jinv[0] = c00 / det; Jinv[1] = (J[2] * J[7] - J[1] * J[8]) / det; Jinv[2] = (J[1] * J[5] - J[2] * J[4]) / det;
  Jinv[3] = c01 / det; Jinv[4] = (J[0] * J[8] - J[2] * J[6]) / det; Jinv[5] = (J[2] * J[3] - J[0] * J[5]) / det;
  Jinv[6] = c02 / det; Jinv[7] = (J[1] * J[6] - J[0] * J[7]) / det; Jinv[8] = (J[0] * J[4] - J[1] * J[3]) / det;
  return det;
}

// Physical basis values and gradients of an element with vertices V at x.
void phys_eval(const VelBasis& vb, const double* V, const double* Jinv, const double* x,
               double* val, double* grad /* n*dim, [k][l] */) {
  int d = vb.dim;
  double xi[3];
  for (int b = 0; b < d; ++b) {
    double s = 0;
    for (int c = 0; c < d; ++c) s += Jinv[b * d + c] * (x[c] - V[c]);
    xi[b] = s;
  }
  double gref[64 * 3];
  vb.eval(xi, val, grad ? gref : nullptr);
  if (grad)
    for (int k = 0; k < vb.n; ++k)
      for (int l = 0; l < d; ++l) {
        double s = 0;
        for (int b = 0; b < d; ++b) s += Jinv[b * d + l] * gref[k * d + b];
        grad[k * d + l] = s;
      }
}

// Map of degree q of a curved element (Section 3, sub-/iso-parametric
// maps): x(xi) = sum_a X_a N_a(xi) with N_a the equispaced Lagrange basis of
// degree q (velocity node order) and X_a the element's geometry nodes.
struct CurvedGeom {
  int d, q;
  const double* X;  // nodes [a][c]
  VelBasis gb;
  CurvedGeom(int d_, int q_, const double* X_) : d(d_), q(q_), X(X_), gb(d_, q_) {}
  // x(xi) and J[c][b] = d x_c / d xi_b; returns det J
  double map(const double* xi, double* x, double* J) const {
    double val[64], grad[64 * 3];
    gb.eval(xi, val, grad);
    for (int c = 0; c < d; ++c) {
      double s = 0.0;
      for (int a = 0; a < gb.n; ++a) s += val[a] * X[a * d + c];
      x[c] = s;
      for (int b = 0; b < d; ++b) {
        double t = 0.0;
        for (int a = 0; a < gb.n; ++a) t += grad[a * d + b] * X[a * d + c];
        J[c * d + b] = t;
      }
    }
    return d == 2 ? J[0] * J[3] - J[1] * J[2]
                  : J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                        J[2] * (J[3] * J[7] - J[4] * J[6]);
  }
  // reference point of physical point x by Newton from the affine guess of
  // the corner nodes; false if it does not converge
  bool to_ref(const HostSetup& hs, int64_t e, const double* x, double* xi) const {
    const double* V = &hs.elem_xyz[e * (d + 1) * d];
    double Jinv[9];
    det_and_inverse(V, d, Jinv);
    for (int b = 0; b < d; ++b) {
      double s = 0;
      for (int c = 0; c < d; ++c) s += Jinv[b * d + c] * (x[c] - V[c]);
      xi[b] = s;
    }
    for (int it = 0; it < 60; ++it) {
      double xx[3], J[9], Ji[9];
      map(xi, xx, J);
      // invert J (2D here)
      const double det = J[0] * J[3] - J[1] * J[2];
      if (!(std::fabs(det) > 0.0)) return false;
      Ji[0] = J[3] / det; Ji[1] = -J[1] / det; Ji[2] = -J[2] / det; Ji[3] = J[0] / det;
      double step[2] = {Ji[0] * (xx[0] - x[0]) + Ji[1] * (xx[1] - x[1]),
                        Ji[2] * (xx[0] - x[0]) + Ji[3] * (xx[1] - x[1])};
      xi[0] -= step[0];
      xi[1] -= step[1];
      if (std::fabs(step[0]) + std::fabs(step[1]) <= 1e-15) return true;
    }
    return false;
  }
};

CurvedGeom curved_geom(const HostSetup& hs, int64_t e) {
  const int nq = (hs.curved_q + 1) * (hs.curved_q + 2) / 2;
  return CurvedGeom(hs.dim, hs.curved_q, &hs.curved_nodes[(size_t)hs.curved_idx[e] * nq * hs.dim]);
}

bool is_curved(const HostSetup& hs, int64_t e) {
  return e >= 0 && !hs.curved_idx.empty() && hs.curved_idx[e] >= 0;
}

// The element's barycentre: the image of the reference barycentre (the
// vertex mean for a straight element, left unchanged).
void curved_bary(const HostSetup& hs, int64_t e, double* b) {
  if (!is_curved(hs, e)) return;
  const double xi[3] = {1.0 / (hs.dim + 1), 1.0 / (hs.dim + 1), 1.0 / (hs.dim + 1)};
  double J[9];
  curved_geom(hs, e).map(xi, b, J);
}

// Rule over the sub-simplex T_{e,j} of a curved element e (local face f):
// the reference rule of the reference sub-simplex (face f's reference
// vertices and the reference barycentre), exact to total degree `deg` in
// the reference coordinates, mapped: physical points x, reference points
// xi, weights w |det J(xi)| (with the sub-simplex's volume factor).
struct MappedRule {
  std::vector<double> x, xi, w, J;  // J: d*d per point
  int n() const { return (int)w.size(); }
};
MappedRule curved_sub_rule(const HostSetup& hs, int64_t e, int f, int deg) {
  const int d = hs.dim;
  std::vector<double> T;
  for (int a = 0; a <= d; ++a) {
    if (a == f) continue;
    for (int b = 0; b < d; ++b) T.push_back(a > 0 && b == a - 1 ? 1.0 : 0.0);
  }
  for (int b = 0; b < d; ++b) T.push_back(1.0 / (d + 1));
  Rule r = simplex_rule(T.data(), d, d, deg);
  const CurvedGeom cg = curved_geom(hs, e);
  MappedRule m;
  m.x.resize((size_t)r.n() * d);
  m.J.resize((size_t)r.n() * d * d);
  m.xi = r.x;
  m.w.resize(r.n());
  for (int q = 0; q < r.n(); ++q) {
    const double det = cg.map(&r.x[q * d], &m.x[q * d], &m.J[(size_t)q * d * d]);
    m.w[q] = r.w[q] * std::fabs(det);
  }
  return m;
}

// Geometry of face j in the frame of its left element.
struct FaceGeom {
  double X[9];            // face vertices, ordered by global vertex index
  double Vl[12], Vr[12];  // left element, right element translated into the left frame
  double bl[3], br[3];    // barycentres (br mirrored through the face on the boundary)
  double nrm[3];          // unit normal from left to right
  double Tsub[2][12];     // sub-simplices T_{l,j}, T_{r,j}
};

void face_geometry(const HostSetup& hs, const int64_t* elem, int64_t j, FaceGeom& g) {
  const int d = hs.dim, nv = d + 1;
  const FaceRec& fr = hs.faces[j];
  const double* Vl = &hs.elem_xyz[(int64_t)fr.left * nv * d];
  for (int a = 0; a < nv * d; ++a) g.Vl[a] = Vl[a];
  int loc[3];
  int q = 0;
  for (int a = 0; a < nv; ++a)
    if (a != fr.lf) loc[q++] = a;
  std::sort(loc, loc + d, [&](int a, int b) {
    return elem[(int64_t)fr.left * nv + a] < elem[(int64_t)fr.left * nv + b];
  });
  for (int a = 0; a < d; ++a)
    for (int c = 0; c < d; ++c) g.X[a * d + c] = Vl[loc[a] * d + c];
  for (int c = 0; c < d; ++c) { g.bl[c] = 0; g.br[c] = 0; }
  for (int a = 0; a < nv; ++a)
    for (int c = 0; c < d; ++c) g.bl[c] += Vl[a * d + c] / nv;
  curved_bary(hs, fr.left, g.bl);
  const bool interior = fr.right >= 0;
  if (interior) {
    const double* Vr0 = &hs.elem_xyz[(int64_t)fr.right * nv * d];
    int64_t g0 = elem[(int64_t)fr.left * nv + loc[0]];
    int ar = -1;
    for (int a = 0; a < nv; ++a)
      if (elem[(int64_t)fr.right * nv + a] == g0) ar = a;
    require(ar >= 0, SDG_EMESH, "inconsistent face");
    double shift[3];
    for (int c = 0; c < d; ++c) shift[c] = g.X[c] - Vr0[ar * d + c];
    for (int a = 0; a < nv; ++a)
      for (int c = 0; c < d; ++c) g.Vr[a * d + c] = Vr0[a * d + c] + shift[c];
    for (int a = 0; a < d; ++a) {
      int64_t gv = elem[(int64_t)fr.left * nv + loc[a]];
      for (int b = 0; b < nv; ++b)
        if (elem[(int64_t)fr.right * nv + b] == gv)
          for (int c = 0; c < d; ++c)
            require(std::fabs(g.Vr[b * d + c] - g.X[a * d + c]) <= 1e-9 * (1.0 + std::fabs(g.X[a * d + c])),
                    SDG_EMESH, "unmatched periodic face");
    }
    for (int a = 0; a < nv; ++a)
      for (int c = 0; c < d; ++c) g.br[c] += g.Vr[a * d + c] / nv;
    curved_bary(hs, fr.right, g.br);  // curved meshes are not periodic: no shift
  } else {
    for (int c = 0; c < d; ++c) {
      double mid = 0;
      for (int a = 0; a < d; ++a) mid += g.X[a * d + c] / d;
      g.br[c] = 2.0 * mid - g.bl[c];
    }
  }
  if (d == 2) {
    double t0 = g.X[2] - g.X[0], t1 = g.X[3] - g.X[1];
    g.nrm[0] = t1; g.nrm[1] = -t0;
  } else {
    double t1[3] = {g.X[3] - g.X[0], g.X[4] - g.X[1], g.X[5] - g.X[2]};
    double t2[3] = {g.X[6] - g.X[0], g.X[7] - g.X[1], g.X[8] - g.X[2]};
    g.nrm[0] = t1[1] * t2[2] - t1[2] * t2[1];
    g.nrm[1] = t1[2] * t2[0] - t1[0] * t2[2];
    g.nrm[2] = t1[0] * t2[1] - t1[1] * t2[0];
  }
  double s = 0, dot = 0;
  for (int c = 0; c < d; ++c) s += g.nrm[c] * g.nrm[c];
  s = std::sqrt(s);
  for (int c = 0; c < d; ++c) {
    g.nrm[c] /= s;
    double fc = 0;
    for (int a = 0; a < d; ++a) fc += g.X[a * d + c] / d;
    dot += g.nrm[c] * (fc - g.bl[c]);
  }
  if (dot < 0)
    for (int c = 0; c < d; ++c) g.nrm[c] = -g.nrm[c];
  for (int sd = 0; sd < 2; ++sd) {
    for (int a = 0; a < d; ++a)
      for (int c = 0; c < d; ++c) g.Tsub[sd][a * d + c] = g.X[a * d + c];
    for (int c = 0; c < d; ++c) g.Tsub[sd][d * d + c] = sd == 0 ? g.bl[c] : g.br[c];
  }
}

// Frame and canonical orthonormalisation of the dual basis of
// one face; vol receives |T_{l,j}| and |T_{r,j}| (0 on the boundary).
void build_dual(const HostSetup& hs, int64_t j, const FaceGeom& g, DualBasis& db, double* vol) {
  const int d = hs.dim, npsi = hs.npsi;
  const int psi_deg = (d == 2) ? 2 * hs.p : hs.p;
  const bool interior = hs.faces[j].right >= 0;
  if (d == 2) {
    double d1[2] = {g.X[2] - g.X[0], g.X[3] - g.X[1]};
    double d2[2] = {g.br[0] - g.bl[0], g.br[1] - g.bl[1]};
    double e1[2] = {0.5 * (d1[0] - d2[0]), 0.5 * (d1[1] - d2[1])};
    double e2[2] = {0.5 * (d1[0] + d2[0]), 0.5 * (d1[1] + d2[1])};
    double det = e1[0] * e2[1] - e2[0] * e1[1];
    db.origin[0] = g.X[0];
    db.origin[1] = g.X[1];
    db.Ainv[0] = e2[1] / det; db.Ainv[1] = -e2[0] / det;
    db.Ainv[2] = -e1[1] / det; db.Ainv[3] = e1[0] / det;
  } else {
    double c[3] = {0, 0, 0};
    int cnt = 0;
    for (int a = 0; a < 3; ++a, ++cnt)
      for (int k = 0; k < 3; ++k) c[k] += g.X[a * 3 + k];
    for (int k = 0; k < 3; ++k) c[k] += g.bl[k];
    ++cnt;
    if (interior) { for (int k = 0; k < 3; ++k) c[k] += g.br[k]; ++cnt; }
    for (int k = 0; k < 3; ++k) c[k] /= cnt;
    double h = 0;
    for (int a = 0; a < 3; ++a) {
      double sq = 0;
      for (int k = 0; k < 3; ++k) sq += (g.X[a * 3 + k] - c[k]) * (g.X[a * 3 + k] - c[k]);
      h = std::max(h, std::sqrt(sq));
    }
    for (int k = 0; k < 3; ++k) db.origin[k] = c[k];
    for (int k = 0; k < 9; ++k) db.Ainv[k] = (k % 4 == 0) ? 1.0 / h : 0.0;
  }
  std::vector<double> A, raw(npsi);
  vol[0] = vol[1] = 0.0;
  int nq = 0;
  for (int s = 0; s < (interior ? 2 : 1); ++s) {
    const FaceRec& fr = hs.faces[j];
    const int64_t e = s == 0 ? fr.left : fr.right;
    Rule r;
    if (is_curved(hs, e)) {
      // psi_m psi_n |det J| in the reference coordinates
      MappedRule m = curved_sub_rule(hs, e, s == 0 ? fr.lf : fr.rf, 2 * psi_deg * hs.curved_q + d * (hs.curved_q - 1));
      r.x = m.x;
      r.w = m.w;
    } else {
      r = simplex_rule(g.Tsub[s], d, d, 2 * psi_deg);
    }
    for (int q = 0; q < r.n(); ++q, ++nq) {
      db.raw(&r.x[q * d], raw.data());
      vol[s] += r.w[q];
      const double sw = std::sqrt(r.w[q]);
      for (int a = 0; a < npsi; ++a) A.push_back(sw * raw[a]);
    }
  }
  db.Linv = orthonormaliser(std::move(A), nq, npsi);
}

}  // namespace

// ---------------------------------------------------------------- main builder

void build_host_setup(HostSetup& hs, int dim, int64_t n_vert, const double* xyz, int64_t n_elem,
                      const int64_t* elem, const double* period, int p, int pg, int scheme,
                      double dt, const double* lam, const double* mu, const double* rho,
                      const CurvedInput* curved) {
  require(dim == 2 || dim == 3, SDG_EINVAL, "dim must be 2 or 3");
  require(n_elem > 0 && n_vert > 0, SDG_EINVAL, "empty mesh");
  const int d = dim, nv = dim + 1;
  hs.dim = d;
  hs.p = p;
  hs.pg = pg;
  hs.scheme = scheme;
  hs.nphi = n_phi_of(d, p);
  hs.npsi = n_psi_of(d, p);
  hs.nsig = n_sig_of(d);
  hs.ng = pg + 1;
  hs.dt = dt;
  hs.n_elem = n_elem;

  // --- unwrapped element vertices
  hs.elem_xyz.assign(n_elem * nv * d, 0.0);
  for (int64_t e = 0; e < n_elem; ++e) {
    for (int a = 0; a < nv; ++a) {
      int64_t g = elem[e * nv + a];
      require(g >= 0 && g < n_vert, SDG_EMESH, "vertex index out of range");
      for (int c = 0; c < d; ++c) {
        double x = xyz[g * d + c];
        if (period && a > 0) {
          double x0 = hs.elem_xyz[(e * nv) * d + c];
          x += period[c] * std::nearbyint((x0 - x) / period[c]);
        }
        hs.elem_xyz[(e * nv + a) * d + c] = x;
      }
    }
  }
  hs.elem_detJ.assign(n_elem, 0.0);
  std::vector<double> Jinv_all(n_elem * d * d);
  for (int64_t e = 0; e < n_elem; ++e) {
    const double* V = &hs.elem_xyz[e * nv * d];
    double det = det_and_inverse(V, d, &Jinv_all[e * d * d]);
    double scale = 0;
    for (int a = 1; a < nv; ++a)
      for (int c = 0; c < d; ++c) scale = std::max(scale, std::fabs(V[a * d + c] - V[c]));
    require(std::isfinite(det) && std::fabs(det) > 1e-12 * std::pow(scale, d), SDG_EMESH,
            "degenerate element " + std::to_string(e));
    hs.elem_detJ[e] = std::fabs(det);
  }

  // --- curved elements: geometry nodes of degree q whose corner nodes are
  // the element's vertices
  hs.curved_q = 0;
  hs.curved_idx.clear();
  hs.curved_ids.clear();
  hs.curved_nodes.clear();
  hs.curved_M.clear();
  if (curved && curved->n > 0) {
    require(d == 2, SDG_EUNSUPPORTED, "curved elements are supported in 2D");
    require(!period, SDG_EUNSUPPORTED, "curved elements on a periodic mesh");
    require(curved->q >= 1 && curved->q <= 4, SDG_EINVAL, "geometry degree must be 1..4");
    require(curved->ids && curved->nodes, SDG_EINVAL, "null curved-element array");
    const int q = curved->q, nq = (q + 1) * (q + 2) / 2;
    hs.curved_q = q;
    hs.curved_idx.assign(n_elem, -1);
    const int corner[3] = {0, q, nq - 1};  // nodes at xi = (0,0), (1,0), (0,1)
    for (int64_t c = 0; c < curved->n; ++c) {
      const int64_t e = curved->ids[c];
      require(e >= 0 && e < n_elem, SDG_EINVAL, "curved element index out of range");
      require(hs.curved_idx[e] < 0, SDG_EINVAL, "curved element listed twice");
      const double* X = curved->nodes + (size_t)c * nq * d;
      const double* V = &hs.elem_xyz[e * nv * d];
      double scale = 1.0;
      for (int a = 0; a < nv * d; ++a) scale = std::max(scale, std::fabs(V[a]));
      for (int a = 0; a < nv; ++a)
        for (int k = 0; k < d; ++k) {
          require(std::isfinite(X[corner[a] * d + k]), SDG_EINVAL, "non-finite geometry node");
          require(std::fabs(X[corner[a] * d + k] - V[a * d + k]) <= 1e-12 * scale, SDG_EMESH,
                  "curved element " + std::to_string(e) + ": corner nodes differ from its vertices");
        }
      hs.curved_idx[e] = (int32_t)hs.curved_ids.size();
      hs.curved_ids.push_back(e);
      hs.curved_nodes.insert(hs.curved_nodes.end(), X, X + (size_t)nq * d);
    }
  }

  // --- faces: sort (sorted vertex key, elem, local face)
  struct Ent { int64_t k[3]; int64_t e; int f; };
  std::vector<Ent> ents;
  ents.reserve(n_elem * nv);
  for (int64_t e = 0; e < n_elem; ++e)
    for (int f = 0; f < nv; ++f) {
      Ent t{{-1, -1, -1}, e, f};
      int q = 0;
      for (int a = 0; a < nv; ++a)
        if (a != f) t.k[q++] = elem[e * nv + a];
      std::sort(t.k, t.k + d);
      ents.push_back(t);
    }
  std::sort(ents.begin(), ents.end(), [&](const Ent& a, const Ent& b) {
    for (int q = 0; q < 3; ++q)
      if (a.k[q] != b.k[q]) return a.k[q] < b.k[q];
    return a.e < b.e;
  });
  hs.faces.clear();
  for (size_t i = 0; i < ents.size();) {
    size_t j = i + 1;
    while (j < ents.size() && std::equal(ents[i].k, ents[i].k + 3, ents[j].k)) ++j;
    require(j - i <= 2, SDG_EMESH, "face shared by more than two elements");
    FaceRec r;
    r.left = (int32_t)ents[i].e;
    r.lf = ents[i].f;
    if (j - i == 2) {
      require(ents[i + 1].e != ents[i].e, SDG_EMESH, "element shares a face with itself");
      r.right = (int32_t)ents[i + 1].e;
      r.rf = ents[i + 1].f;
    } else {
      r.right = -1;
      r.rf = -1;
    }
    hs.faces.push_back(r);
    i = j;
  }
  std::sort(hs.faces.begin(), hs.faces.end(), [](const FaceRec& a, const FaceRec& b) {
    return a.left != b.left ? a.left < b.left : a.lf < b.lf;
  });
  const int64_t nf = (int64_t)hs.faces.size();
  hs.n_face = nf;
  hs.n_bface = 0;
  hs.elem_face.assign(n_elem * nv, -1);
  for (int64_t j = 0; j < nf; ++j) {
    const FaceRec& r = hs.faces[j];
    hs.elem_face[(int64_t)r.left * nv + r.lf] = (int32_t)j;
    if (r.right >= 0) hs.elem_face[(int64_t)r.right * nv + r.rf] = (int32_t)j;
    else ++hs.n_bface;
  }

  // a curved element's faces shared with another element must be straight:
  // their geometry nodes at the affine positions (a boundary face may curve)
  if (hs.curved_q > 0) {
    const int q = hs.curved_q, nq = (q + 1) * (q + 2) / 2;
    VelBasis gb(d, q);
    for (int64_t e : hs.curved_ids) {
      const double* X = &hs.curved_nodes[(size_t)hs.curved_idx[e] * nq * d];
      const double* V = &hs.elem_xyz[e * nv * d];
      double scale = 1.0;
      for (int a = 0; a < nv * d; ++a) scale = std::max(scale, std::fabs(V[a]));
      for (int f = 0; f < nv; ++f) {
        if (hs.faces[hs.elem_face[e * nv + f]].right < 0) continue;
        for (int k = 0; k < nq; ++k) {
          if (gb.alpha[k][f] != 0) continue;  // node not on local face f
          for (int c = 0; c < d; ++c) {
            double xa = 0.0;
            for (int a = 0; a < nv; ++a) xa += gb.alpha[k][a] / (double)q * V[a * d + c];
            require(std::fabs(X[k * d + c] - xa) <= 1e-12 * scale, SDG_EMESH,
                    "curved element " + std::to_string(e) + ": a face shared with another element is not straight");
          }
        }
      }
    }
  }

  // --- material and reference mass
  hs.elem_rho.assign(rho, rho + n_elem);
  hs.elem_w.resize(n_elem);
  for (int64_t e = 0; e < n_elem; ++e) {
    require(rho[e] > 0 && lam[e] >= 0 && mu[e] > 0, SDG_EINVAL, "material must be positive");
    // a curved element's mass is rho times its own matrix (curved_M)
    hs.elem_w[e] = is_curved(hs, e) ? rho[e] : rho[e] * hs.elem_detJ[e];
  }
  VelBasis vb(d, p);
  {
    std::vector<double> Vref(nv * d, 0.0);
    for (int a = 0; a < d; ++a) Vref[(a + 1) * d + a] = 1.0;
    Rule r = simplex_rule(Vref.data(), d, d, 2 * p);
    hs.Mref.assign(hs.nphi * hs.nphi, 0.0);
    std::vector<double> val(hs.nphi);
    for (int q = 0; q < r.n(); ++q) {
      vb.eval(&r.x[q * d], val.data(), nullptr);
      for (int k = 0; k < hs.nphi; ++k)
        for (int m = 0; m < hs.nphi; ++m) hs.Mref[k * hs.nphi + m] += r.w[q] * val[k] * val[m];
    }
    // curved elements: int phi_k phi_m |det J| on the reference element
    if (hs.curved_q > 0) {
      const int q = hs.curved_q, nq = (q + 1) * (q + 2) / 2;
      Rule rc = simplex_rule(Vref.data(), d, d, 2 * p + d * (q - 1));
      hs.curved_M.assign(hs.curved_ids.size() * hs.nphi * hs.nphi, 0.0);
      for (size_t c = 0; c < hs.curved_ids.size(); ++c) {
        CurvedGeom cg(d, q, &hs.curved_nodes[c * nq * d]);
        double* M = &hs.curved_M[c * hs.nphi * hs.nphi];
        for (int qq = 0; qq < rc.n(); ++qq) {
          double x[3], J[9];
          const double det = cg.map(&rc.x[qq * d], x, J);
          require(det > 0.0, SDG_EMESH, "curved element " + std::to_string(hs.curved_ids[c]) + " is folded");
          vb.eval(&rc.x[qq * d], val.data(), nullptr);
          for (int k = 0; k < hs.nphi; ++k)
            for (int m = 0; m < hs.nphi; ++m) M[k * hs.nphi + m] += rc.w[qq] * det * val[k] * val[m];
        }
      }
    }
  }

  // --- time basis: Lagrange through the Gauss-Legendre points of [0,1]
  {
    const int ng = hs.ng;
    gauss_legendre(ng, hs.tau, hs.w);
    auto lag = [&](int a, double t, double* dval) {
      double v = 1.0, dv = 0.0;
      for (int b = 0; b < ng; ++b) {
        if (b == a) continue;
        double f = (t - hs.tau[b]) / (hs.tau[a] - hs.tau[b]);
        dv = dv * f + v / (hs.tau[a] - hs.tau[b]);
        v *= f;
      }
      if (dval) *dval = dv;
      return v;
    };
    hs.e0.resize(ng);
    hs.e1.resize(ng);
    for (int a = 0; a < ng; ++a) { hs.e0[a] = lag(a, 0.0, nullptr); hs.e1[a] = lag(a, 1.0, nullptr); }
    // the slab polynomial continued to the next slab: Ext[a][b] = gamma_b(1 + tau_a)
    hs.Ext.assign(ng * ng, 0.0);
    for (int a = 0; a < ng; ++a)
      for (int b = 0; b < ng; ++b) hs.Ext[a * ng + b] = lag(b, 1.0 + hs.tau[a], nullptr);
    std::vector<double> qx, qw;
    gauss_legendre(ng + 1, qx, qw);
    hs.T.assign(ng * ng, 0.0);
    for (int a = 0; a < ng; ++a)
      for (int b = 0; b < ng; ++b) {
        double s = hs.e1[a] * hs.e1[b];
        for (int q = 0; q < (int)qx.size(); ++q) {
          double da;
          lag(a, qx[q], &da);
          s -= qw[q] * da * lag(b, qx[q], nullptr);
        }
        hs.T[a * ng + b] = s;
      }
  }

  // --- per-face blocks
  const int nphi = hs.nphi, npsi = hs.npsi;
  const int blk = nphi * d * npsi;
  hs.Dt.assign((size_t)nf * 2 * blk, 0.0);
  hs.face_lm.assign(nf * 2, 0.0);
  hs.face_wt.assign(nf * 2, 0.0);
  const int psi_deg = (d == 2) ? 2 * p : p;
  int err_code = 0;
  std::string err_msg;

  std::mutex err_mu;
  parallel_for(nf, [&](int64_t j) {
    std::vector<double> phi(nphi), gphi(nphi * d), psi(npsi);
      try {
        FaceGeom fg;
        face_geometry(hs, elem, j, fg);
        DualBasis db(d, p);
        double vol[2];
        build_dual(hs, j, fg, db, vol);
        const FaceRec& fr = hs.faces[j];
        const bool interior = fr.right >= 0;
        const int nsides = interior ? 2 : 1;
        for (int s = 0; s < nsides; ++s) {
          const double* Ve = s == 0 ? fg.Vl : fg.Vr;
          double Jinv[9];
          det_and_inverse(Ve, d, Jinv);
          double* out = &hs.Dt[((size_t)j * 2 + s) * blk];
          const int64_t es = s == 0 ? fr.left : fr.right;
          if (is_curved(hs, es)) {
            // -int d_l phi_k psi_m over the curved T_{i,j}: the reference
            // gradient through J(xi)^-T, times |det J| (together adj J)
            const int q = hs.curved_q;
            MappedRule m = curved_sub_rule(hs, es, s == 0 ? fr.lf : fr.rf,
                                           std::max(p - 1, 0) + psi_deg * q + (d - 1) * (q - 1));
            std::vector<double> gref(nphi * d);
            for (int qq = 0; qq < m.n(); ++qq) {
              const double* J = &m.J[(size_t)qq * d * d];
              const double det = J[0] * J[3] - J[1] * J[2];
              const double Ji[4] = {J[3] / det, -J[1] / det, -J[2] / det, J[0] / det};  // Ji[b][c]
              vb.eval(&m.xi[qq * d], phi.data(), gref.data());
              for (int k = 0; k < nphi; ++k)
                for (int l = 0; l < d; ++l) {
                  double sgl = 0.0;
                  for (int b = 0; b < d; ++b) sgl += Ji[b * d + l] * gref[k * d + b];
                  gphi[k * d + l] = sgl;
                }
              db.canonical(&m.x[qq * d], psi.data());
              for (int k = 0; k < nphi; ++k)
                for (int l = 0; l < d; ++l) {
                  double f = -m.w[qq] * gphi[k * d + l];
                  double* o = out + (k * d + l) * npsi;
                  for (int mm = 0; mm < npsi; ++mm) o[mm] += f * psi[mm];
                }
            }
          }
          Rule r = is_curved(hs, es) ? Rule() : simplex_rule(fg.Tsub[s], d, d, std::max(p - 1, 0) + psi_deg);
          for (int qq = 0; qq < r.n(); ++qq) {
            const double* x = &r.x[qq * d];
            phys_eval(vb, Ve, Jinv, x, phi.data(), gphi.data());
            db.canonical(x, psi.data());
            for (int k = 0; k < nphi; ++k)
              for (int l = 0; l < d; ++l) {
                double f = -r.w[qq] * gphi[k * d + l];
                double* o = out + (k * d + l) * npsi;
                for (int m = 0; m < npsi; ++m) o[m] += f * psi[m];
              }
          }
          if (interior) {
            double sgn = s == 0 ? 1.0 : -1.0;
            Rule rf = simplex_rule(fg.X, d - 1, d, p + psi_deg);
            for (int qq = 0; qq < rf.n(); ++qq) {
              const double* x = &rf.x[qq * d];
              phys_eval(vb, Ve, Jinv, x, phi.data(), nullptr);
              db.canonical(x, psi.data());
              for (int k = 0; k < nphi; ++k)
                for (int l = 0; l < d; ++l) {
                  double f = rf.w[qq] * phi[k] * sgn * fg.nrm[l];
                  double* o = out + (k * d + l) * npsi;
                  for (int m = 0; m < npsi; ++m) o[m] += f * psi[m];
                }
            }
          }
        }
        // dual material: volume-weighted Lame parameters
        if (interior) {
          double vt = vol[0] + vol[1];
          hs.face_lm[2 * j] = (vol[0] * lam[fr.left] + vol[1] * lam[fr.right]) / vt;
          hs.face_lm[2 * j + 1] = (vol[0] * mu[fr.left] + vol[1] * mu[fr.right]) / vt;
          hs.face_wt[2 * j] = vol[0] / vt;
          hs.face_wt[2 * j + 1] = vol[1] / vt;
        } else {
          hs.face_lm[2 * j] = lam[fr.left];
          hs.face_lm[2 * j + 1] = mu[fr.left];
          hs.face_wt[2 * j] = 1.0;
        }
      } catch (const Error& e) {
        std::lock_guard<std::mutex> lk(err_mu);
        if (!err_code) { err_code = e.code; err_msg = e.what(); }
      }
  });
  if (err_code) throw Error(err_code, err_msg);
}

double elem_mass(const HostSetup& hs, int64_t e, int k, int m) {
  const int n = hs.nphi;
  if (is_curved(hs, e)) return hs.elem_w[e] * hs.curved_M[((size_t)hs.curved_idx[e] * n + k) * n + m];
  return hs.elem_w[e] * hs.Mref[k * n + m];
}

bool eval_velocity_basis(const HostSetup& hs, int64_t e, const double* x, double* phi, double tol) {
  const int d = hs.dim, nv = d + 1;
  if (is_curved(hs, e)) {
    // reference point by Newton on the element's map (the affine guess first
    // rejects points far outside)
    double xi[3];
    if (!curved_geom(hs, e).to_ref(hs, e, x, xi)) return false;
    double lam0 = 1.0;
    for (int b = 0; b < d; ++b) {
      if (xi[b] < -tol) return false;
      lam0 -= xi[b];
    }
    if (lam0 < -tol) return false;
    if (phi) {
      VelBasis vb(d, hs.p);
      vb.eval(xi, phi, nullptr);
    }
    return true;
  }
  const double* V = &hs.elem_xyz[e * nv * d];
  double Jinv[9];
  det_and_inverse(V, d, Jinv);
  double xi[3], lam0 = 1.0;
  for (int b = 0; b < d; ++b) {
    double s = 0;
    for (int c = 0; c < d; ++c) s += Jinv[b * d + c] * (x[c] - V[c]);
    xi[b] = s;
    lam0 -= s;
    if (s < -tol) return false;
  }
  if (lam0 < -tol) return false;
  if (phi) {
    VelBasis vb(d, hs.p);
    vb.eval(xi, phi, nullptr);
  }
  return true;
}

int64_t locate_point(const HostSetup& hs, const double* x, int64_t e_begin, int64_t e_end) {
  if (e_end < 0) e_end = hs.n_elem;
  for (int64_t e = std::max<int64_t>(0, e_begin); e < std::min<int64_t>(e_end, hs.n_elem); ++e)
    if (eval_velocity_basis(hs, e, x, nullptr, 1e-12)) return e;
  return -1;
}

void eval_dual_canonical(const HostSetup& hs, const int64_t* elem, int64_t j, int64_t n,
                         const double* x, double* out) {
  FaceGeom fg;
  face_geometry(hs, elem, j, fg);
  DualBasis db(hs.dim, hs.p);
  double vol[2];
  build_dual(hs, j, fg, db, vol);
  for (int64_t q = 0; q < n; ++q) db.canonical(x + q * hs.dim, out + q * hs.npsi);
}

// ---------------------------------------------------------------- compressed 3D operator

// In 3D the dual functions are polynomials of degree p in physical
// coordinates (Section 3), so on the sub-simplex T_{i,j} each one is a
// polynomial of degree p in the reference coordinates xi of element i.  With
// a basis mu^(f) of P_p orthonormal over the reference sub-simplex T_f^ref
// (reference face f and the reference barycentre; f = local face of j in i):
//   psi_m(x(xi)) = sum_m' C_{i,j}[m][m'] mu^(f)_m'(xi),
// and the block of eq. (MD_3) factors into reference tables and a little
// geometry:
//   Dt[k][l][m] = sum_m' C[m][m'] (a_l F_f[k][m'] - sum_a B[a][l] G_f[k][a][m']),
//   F_f[k][m']    = int_{face f} phi_k mu_m' dS_ref,
//   G_f[k][a][m'] = int_{T_f^ref} d_{xi_a} phi_k mu_m' dxi,
//   a_l = (+1 left, -1 right) |Gamma_j| / |face f| n_l (0 on a free-surface face),
//   B[a][l] = |J_i| (J_i^-1)[a][l].
namespace {

// reference tetrahedron and its local face f (the face opposite vertex f)
const double kRefTet[12] = {0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1};

void ref_sub_simplex(int f, double* T) {  // face f's three vertices, then the barycentre
  int q = 0;
  for (int a = 0; a < 4; ++a) {
    if (a == f) continue;
    for (int c = 0; c < 3; ++c) T[q * 3 + c] = kRefTet[a * 3 + c];
    ++q;
  }
  for (int c = 0; c < 3; ++c) T[9 + c] = 0.25;
}

// Orthonormal basis mu^(f) of P_p over T_f^ref: Legendre products (ordered
// as the 3D dual sequence) times Li.
struct RefDual {
  DualBasis raw{3, 1};
  std::vector<double> Li;
  explicit RefDual(int p, int f) : raw(3, p) {
    // Legendre products in coordinates centred on T_f^ref and scaled by its
    // size, for a well-conditioned orthonormalisation
    double T[12];
    ref_sub_simplex(f, T);
    double h = 0.0;
    for (int c = 0; c < 3; ++c) raw.origin[c] = 0.25 * (T[c] + T[3 + c] + T[6 + c] + T[9 + c]);
    for (int a = 0; a < 4; ++a) {
      double sq = 0.0;
      for (int c = 0; c < 3; ++c) sq += (T[a * 3 + c] - raw.origin[c]) * (T[a * 3 + c] - raw.origin[c]);
      h = std::max(h, std::sqrt(sq));
    }
    for (int k = 0; k < 9; ++k) raw.Ainv[k] = (k % 4 == 0) ? 1.0 / h : 0.0;
    Rule r = simplex_rule(T, 3, 3, 2 * p);
    std::vector<double> A, v(raw.n);
    for (int q = 0; q < r.n(); ++q) {
      raw.raw(&r.x[q * 3], v.data());
      const double sw = std::sqrt(r.w[q]);
      for (int a = 0; a < raw.n; ++a) A.push_back(sw * v[a]);
    }
    Li = orthonormaliser(std::move(A), r.n(), raw.n);
  }
  void eval(const double* xi, double* out) const {
    double rv[64];
    raw.raw(xi, rv);
    for (int i = 0; i < raw.n; ++i) {
      double s = 0.0;
      for (int k = 0; k <= i; ++k) s += Li[i * raw.n + k] * rv[k];
      out[i] = s;
    }
  }
};

}  // namespace

void build_compressed(const HostSetup& hs, const int64_t* elem, CompressedOp& out) {
  require(hs.dim == 3, SDG_EUNSUPPORTED, "the compressed operator is built for tetrahedra");
  const int p = hs.p, nphi = hs.nphi, npsi = hs.npsi;
  out.npsi = npsi;
  VelBasis vb(3, p);
  std::vector<RefDual> mu;
  for (int f = 0; f < 4; ++f) mu.emplace_back(p, f);
  // reference tables
  out.F.assign((size_t)4 * nphi * npsi, 0.0);
  out.G.assign((size_t)4 * nphi * 3 * npsi, 0.0);
  out.face_area_ref.assign(4, 0.0);
  std::vector<double> phi(nphi), gphi(nphi * 3), m(npsi);
  for (int f = 0; f < 4; ++f) {
    double T[12];
    ref_sub_simplex(f, T);
    Rule rv = simplex_rule(T, 3, 3, std::max(p - 1, 0) + p);
    for (int q = 0; q < rv.n(); ++q) {
      vb.eval(&rv.x[q * 3], phi.data(), gphi.data());
      mu[f].eval(&rv.x[q * 3], m.data());
      for (int k = 0; k < nphi; ++k)
        for (int a = 0; a < 3; ++a)
          for (int mm = 0; mm < npsi; ++mm)
            out.G[(((size_t)f * nphi + k) * 3 + a) * npsi + mm] += rv.w[q] * gphi[k * 3 + a] * m[mm];
    }
    Rule rf = simplex_rule(T, 2, 3, 2 * p);
    for (int q = 0; q < rf.n(); ++q) {
      vb.eval(&rf.x[q * 3], phi.data(), nullptr);
      mu[f].eval(&rf.x[q * 3], m.data());
      out.face_area_ref[f] += rf.w[q];
      for (int k = 0; k < nphi; ++k)
        for (int mm = 0; mm < npsi; ++mm)
          out.F[((size_t)f * nphi + k) * npsi + mm] += rf.w[q] * phi[k] * m[mm];
    }
  }
  // per element: B = |J| J^-1
  out.eB.assign((size_t)hs.n_elem * 9, 0.0);
  parallel_for(hs.n_elem, [&](int64_t e) {
    double Jinv[9];
    const double det = det_and_inverse(&hs.elem_xyz[e * 12], 3, Jinv);
    for (int k = 0; k < 9; ++k) out.eB[e * 9 + k] = std::fabs(det) * Jinv[k];
  });
  // per face and side: C and the face-term coefficients
  out.C.assign((size_t)hs.n_face * 2 * npsi * npsi, 0.0);
  out.fa.assign((size_t)hs.n_face * 2 * 3, 0.0);
  int err_code = 0;
  std::string err_msg;
  std::mutex err_mu;
  parallel_for(hs.n_face, [&](int64_t j) {
    try {
      FaceGeom fg;
      face_geometry(hs, elem, j, fg);
      DualBasis db(3, p);
      double vol[2];
      build_dual(hs, j, fg, db, vol);
      const FaceRec& fr = hs.faces[j];
      const bool interior = fr.right >= 0;
      // |Gamma_j| from the face vertices
      const double t1[3] = {fg.X[3] - fg.X[0], fg.X[4] - fg.X[1], fg.X[5] - fg.X[2]};
      const double t2[3] = {fg.X[6] - fg.X[0], fg.X[7] - fg.X[1], fg.X[8] - fg.X[2]};
      const double cx = t1[1] * t2[2] - t1[2] * t2[1], cy = t1[2] * t2[0] - t1[0] * t2[2],
                   cz = t1[0] * t2[1] - t1[1] * t2[0];
      const double area = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
      std::vector<double> psi(npsi), mv(npsi);
      for (int s = 0; s < (interior ? 2 : 1); ++s) {
        const double* Ve = s == 0 ? fg.Vl : fg.Vr;
        const int f = s == 0 ? fr.lf : fr.rf;
        double T[12];
        ref_sub_simplex(f, T);
        Rule r = simplex_rule(T, 3, 3, 2 * p);
        double* Co = &out.C[((size_t)j * 2 + s) * npsi * npsi];
        for (int q = 0; q < r.n(); ++q) {
          const double* xi = &r.x[q * 3];
          double x[3];
          for (int c = 0; c < 3; ++c) {
            x[c] = Ve[c];
            for (int a = 0; a < 3; ++a) x[c] += (Ve[(a + 1) * 3 + c] - Ve[c]) * xi[a];
          }
          db.canonical(x, psi.data());
          mu[f].eval(xi, mv.data());
          for (int a = 0; a < npsi; ++a)
            for (int b = 0; b < npsi; ++b) Co[a * npsi + b] += r.w[q] * psi[a] * mv[b];
        }
        if (interior) {
          const double sgn = s == 0 ? 1.0 : -1.0;
          for (int l = 0; l < 3; ++l) out.fa[((size_t)j * 2 + s) * 3 + l] = sgn * area / out.face_area_ref[f] * fg.nrm[l];
        }
      }
    } catch (const Error& e) {
      std::lock_guard<std::mutex> lk(err_mu);
      if (!err_code) { err_code = e.code; err_msg = e.what(); }
    }
  });
  if (err_code) throw Error(err_code, err_msg);
}

// ---------------------------------------------------------------- projection of data

// Lowest rule degree of the L2 projection of initial data (the state at
// t^{0,-}) that integrates the mass of the discrete space exactly: velocity
// functions have degree p, dual functions degree psi_deg (2p for the 2D
// tensor products), and the projected data is at least of degree p.
int projection_min_degree(const HostSetup& hs, int which) {
  const int psi_deg = hs.dim == 2 ? 2 * hs.p : hs.p;
  if (hs.curved_q > 1) {
    // curved elements integrate in reference coordinates: phi phi |det J|,
    // and psi (degree psi_deg + p data) composed with the map, times |det J|
    const int q = hs.curved_q, jd = hs.dim * (q - 1);
    return which == 0 ? 2 * hs.p + jd : (psi_deg + hs.p) * q + jd;
  }
  return which == 0 ? 2 * hs.p : psi_deg + hs.p;
}

int projection_rule_size(const HostSetup& hs, int which, int degree) {
  std::vector<double> Vref((hs.dim + 1) * hs.dim, 0.0);
  for (int a = 0; a < hs.dim; ++a) Vref[(a + 1) * hs.dim + a] = 1.0;
  const int nq = simplex_rule(Vref.data(), hs.dim, hs.dim, degree).n();
  return which == 0 ? nq : 2 * nq;
}

void projection_points(const HostSetup& hs, const int64_t* elem, int which, int degree, double* pts,
                       double* wts) {
  const int d = hs.dim, nv = d + 1;
  const int nq = projection_rule_size(hs, which, degree);
  if (which == 0) {
    std::vector<double> Vref(nv * d, 0.0);
    for (int a = 0; a < d; ++a) Vref[(a + 1) * d + a] = 1.0;
    const Rule rref = simplex_rule(Vref.data(), d, d, degree);
    parallel_for(hs.n_elem, [&](int64_t e) {
      if (is_curved(hs, e)) {  // the reference rule mapped, weights times |det J|
        const CurvedGeom cg = curved_geom(hs, e);
        for (int q = 0; q < nq; ++q) {
          double J[9];
          const double det = cg.map(&rref.x[q * d], &pts[(e * nq + q) * d], J);
          if (wts) wts[e * nq + q] = rref.w[q] * std::fabs(det);
        }
        return;
      }
      Rule r = simplex_rule(&hs.elem_xyz[e * nv * d], d, d, degree);
      for (int q = 0; q < nq; ++q) {
        for (int c = 0; c < d; ++c) pts[(e * nq + q) * d + c] = r.x[q * d + c];
        if (wts) wts[e * nq + q] = r.w[q];
      }
    });
    return;
  }
  const int half = nq / 2;
  parallel_for(hs.n_face, [&](int64_t j) {
    FaceGeom fg;
    face_geometry(hs, elem, j, fg);
    const bool interior = hs.faces[j].right >= 0;
    for (int s = 0; s < 2; ++s) {
      // a free-surface dual element is T_{l,j} alone: its second half of
      // points repeats the first with zero weights
      const int sd = interior ? s : 0;
      const FaceRec& fr = hs.faces[j];
      const int64_t e = sd == 0 ? fr.left : fr.right;
      Rule r;
      if (is_curved(hs, e)) {
        MappedRule m = curved_sub_rule(hs, e, sd == 0 ? fr.lf : fr.rf, degree);
        r.x = m.x;
        r.w = m.w;
      } else {
        r = simplex_rule(fg.Tsub[sd], d, d, degree);
      }
      for (int q = 0; q < half; ++q) {
        const int64_t o = j * nq + s * half + q;
        for (int c = 0; c < d; ++c) pts[o * d + c] = r.x[q * d + c];
        if (wts) wts[o] = (interior || s == 0) ? r.w[q] : 0.0;
      }
    }
  });
}

void project_values(const HostSetup& hs, const int64_t* elem, int which, int degree, const double* values,
                    double* out) {
  const int d = hs.dim, nv = d + 1, nphi = hs.nphi, npsi = hs.npsi, nsig = hs.nsig;
  const int nq = projection_rule_size(hs, which, degree);
  if (which == 0) {
    // v_e = Mbar_e^-1 int_{T_e} phi f = Mref^-1 sum_q w_q phi(xi_q) f(x_q) / |J_e|, computed
    // on the reference element with the same points the caller evaluated f at
    std::vector<double> Vref(nv * d, 0.0);
    for (int a = 0; a < d; ++a) Vref[(a + 1) * d + a] = 1.0;
    Rule r = simplex_rule(Vref.data(), d, d, degree);
    VelBasis vb(d, hs.p);
    std::vector<double> Phi((size_t)nq * nphi);
    for (int q = 0; q < nq; ++q) vb.eval(&r.x[q * d], &Phi[(size_t)q * nphi], nullptr);
    parallel_for(hs.n_elem, [&](int64_t e) {
      std::vector<double> B((size_t)nphi * d, 0.0);  // [k][c]
      const bool cur = is_curved(hs, e);
      std::vector<double> wq(r.w);
      if (cur) {  // a curved element's integral carries |det J|, its mass is curved_M
        const CurvedGeom cg = curved_geom(hs, e);
        for (int q = 0; q < nq; ++q) {
          double x[3], J[9];
          wq[q] *= std::fabs(cg.map(&r.x[q * d], x, J));
        }
      }
      for (int q = 0; q < nq; ++q) {
        const double* f = values + (e * nq + q) * d;
        for (int k = 0; k < nphi; ++k)
          for (int c = 0; c < d; ++c) B[k * d + c] += wq[q] * Phi[(size_t)q * nphi + k] * f[c];
      }
      if (cur) {
        std::vector<double> Mc(&hs.curved_M[(size_t)hs.curved_idx[e] * nphi * nphi],
                               &hs.curved_M[(size_t)(hs.curved_idx[e] + 1) * nphi * nphi]);
        solve_dense(Mc, B, nphi, d);
        for (int c = 0; c < d; ++c)
          for (int k = 0; k < nphi; ++k) out[(e * d + c) * nphi + k] = B[k * d + c];
        return;
      }
      solve_dense(hs.Mref, B, nphi, d);
      for (int c = 0; c < d; ++c)
        for (int k = 0; k < nphi; ++k) out[(e * d + c) * nphi + k] = B[k * d + c];
    });
    return;
  }
  // sigma_j[s][m] = int_{R_j} psi_m f_s: the canonical dual basis is orthonormal
  std::vector<double> pts((size_t)hs.n_face * nq * d), wts((size_t)hs.n_face * nq);
  projection_points(hs, elem, 1, degree, pts.data(), wts.data());
  parallel_for(hs.n_face, [&](int64_t j) {
    FaceGeom fg;
    face_geometry(hs, elem, j, fg);
    DualBasis db(d, hs.p);
    double vol[2];
    build_dual(hs, j, fg, db, vol);
    std::vector<double> psi(npsi);
    double* o = out + j * nsig * npsi;
    for (int a = 0; a < nsig * npsi; ++a) o[a] = 0.0;
    for (int q = 0; q < nq; ++q) {
      const double w = wts[j * nq + q];
      if (w == 0.0) continue;
      db.canonical(&pts[(j * nq + q) * d], psi.data());
      const double* f = values + (j * nq + q) * nsig;
      for (int sv = 0; sv < nsig; ++sv)
        for (int m = 0; m < npsi; ++m) o[sv * npsi + m] += w * psi[m] * f[sv];
    }
  });
}

// Element diagonal blocks of the velocity operator (eq. pre1),
//   D_i = Tm (x) w_i Mref + Cg (x) K_ii,  K_ii = sum_f Dt_{i,f} E_j Dt_{i,f}^T,
// inverted on the host; returned in FP32, column-major per element.
namespace {

// Voigt index of the tensor entry (c, l): 2D (xx, yy, xy); 3D (xx, yy, zz,
// yz, xz, xy), Section 2.
int voigt_of(int d, int c, int l) {
  if (c == l) return c;
  if (d == 2) return 2;
  return 6 - c - l;
}

// E[c][l][c2][l2] of the dual material of face j: sigma_cl = sum E d_l2 v_c2.
// Isotropic (eq. 1.1b): lambda delta_cl delta_c2l2 + mu (delta_cc2 delta_ll2 +
// delta_cl2 delta_lc2).  Anisotropic: the Voigt stiffness acts on the strain
// rate with the shear components halved (Section 2), so
// E = E~[v(c,l)][v(c2,l2)] (1 if c2 == l2, else 1/2).
double hooke_entry(const HostSetup& hs, int64_t j, int c, int l, int c2, int l2) {
  const int d = hs.dim;
  if (!hs.face_E.empty()) {
    const int ns = hs.nsig;
    const double e = hs.face_E[(size_t)j * ns * ns + voigt_of(d, c, l) * ns + voigt_of(d, c2, l2)];
    return c2 == l2 ? e : 0.5 * e;
  }
  const double lam = hs.face_lm[2 * j], mu = hs.face_lm[2 * j + 1];
  return mu * ((c == c2 && l == l2) + (c == l2 && l == c2)) + lam * (c == l && c2 == l2);
}

// Element stiffness of the Schur operator restricted to element e (the
// diagonal block of K): K[(c,k),(c2,k2)] = sum over the faces of e of
// sum_{l,l2,m} Dt[k][l][m] E_{cl,c2l2} Dt[k2][l2][m].
void element_stiffness(const HostSetup& hs, int64_t e, std::vector<double>& K) {
  const int d = hs.dim, nphi = hs.nphi, npsi = hs.npsi;
  const int ns = d * nphi, blk = nphi * d * npsi;
  K.assign((size_t)ns * ns, 0.0);
  for (int f = 0; f <= d; ++f) {
    const int32_t j = hs.elem_face[e * (d + 1) + f];
    const FaceRec& fr = hs.faces[j];
    const int side = (fr.left == e && fr.lf == f) ? 0 : 1;
    const double* Db = &hs.Dt[((size_t)j * 2 + side) * blk];
    for (int c = 0; c < d; ++c)
      for (int l = 0; l < d; ++l)
        for (int c2 = 0; c2 < d; ++c2)
          for (int l2 = 0; l2 < d; ++l2) {
            const double E = hooke_entry(hs, j, c, l, c2, l2);
            if (E == 0.0) continue;
            for (int k = 0; k < nphi; ++k)
              for (int k2 = 0; k2 < nphi; ++k2) {
                double sacc = 0.0;
                const double* a1 = Db + (k * d + l) * npsi;
                const double* a2 = Db + (k2 * d + l2) * npsi;
                for (int m = 0; m < npsi; ++m) sacc += a1[m] * a2[m];
                K[(c * nphi + k) * ns + c2 * nphi + k2] += E * sacc;
              }
          }
  }
}

// Stiffness coupling of element sides sl and sm of face j (the face's part
// of the block of K between the two elements):
// K[(c,k),(c2,k2)] += sum_{l,l2,m} Dt_sl[k][l][m] E_{cl,c2l2} Dt_sm[k2][l2][m].
void face_coupling(const HostSetup& hs, int64_t j, int sl, int sm, std::vector<double>& K) {
  const int d = hs.dim, nphi = hs.nphi, npsi = hs.npsi;
  const int ns = d * nphi, blk = nphi * d * npsi;
  const double* D1 = &hs.Dt[((size_t)j * 2 + sl) * blk];
  const double* D2 = &hs.Dt[((size_t)j * 2 + sm) * blk];
  for (int c = 0; c < d; ++c)
    for (int l = 0; l < d; ++l)
      for (int c2 = 0; c2 < d; ++c2)
        for (int l2 = 0; l2 < d; ++l2) {
          const double E = hooke_entry(hs, j, c, l, c2, l2);
          if (E == 0.0) continue;
          for (int k = 0; k < nphi; ++k)
            for (int k2 = 0; k2 < nphi; ++k2) {
              double sacc = 0.0;
              const double* a1 = D1 + (k * d + l) * npsi;
              const double* a2 = D2 + (k2 * d + l2) * npsi;
              for (int m = 0; m < npsi; ++m) sacc += a1[m] * a2[m];
              K[(c * nphi + k) * ns + c2 * nphi + k2] += E * sacc;
            }
        }
}

// Solve A X = B in place with partial pivoting (A n x n row-major, destroyed;
// B n x m row-major); false if singular.
bool lu_solve(std::vector<double>& A, std::vector<double>& B, int n, int m) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[(size_t)r * n + c]) > std::fabs(A[(size_t)piv * n + c])) piv = r;
    if (A[(size_t)piv * n + c] == 0.0) return false;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(A[(size_t)c * n + k], A[(size_t)piv * n + k]);
      for (int k = 0; k < m; ++k) std::swap(B[(size_t)c * m + k], B[(size_t)piv * m + k]);
    }
    const double dinv = 1.0 / A[(size_t)c * n + c];
    for (int r = c + 1; r < n; ++r) {
      const double f = A[(size_t)r * n + c] * dinv;
      if (f == 0.0) continue;
      A[(size_t)r * n + c] = f;
      for (int k = c + 1; k < n; ++k) A[(size_t)r * n + k] -= f * A[(size_t)c * n + k];
      for (int k = 0; k < m; ++k) B[(size_t)r * m + k] -= f * B[(size_t)c * m + k];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    const double dinv = 1.0 / A[(size_t)c * n + c];
    for (int k = 0; k < m; ++k) {
      double v = B[(size_t)c * m + k];
      for (int r = c + 1; r < n; ++r) v -= A[(size_t)c * n + r] * B[(size_t)r * m + k];
      B[(size_t)c * m + k] = v * dinv;
    }
  }
  return true;
}

// Gauss-Jordan inverse with partial pivoting (row-major, n x n); false if singular.
bool gj_inverse(std::vector<double> M, int n, std::vector<double>& Inv) {
  Inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Inv[i * n + i] = 1.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(M[r * n + col]) > std::fabs(M[piv * n + col])) piv = r;
    if (M[piv * n + col] == 0.0) return false;
    if (piv != col)
      for (int k = 0; k < n; ++k) { std::swap(M[col * n + k], M[piv * n + k]); std::swap(Inv[col * n + k], Inv[piv * n + k]); }
    const double dinv = 1.0 / M[col * n + col];
    for (int k = 0; k < n; ++k) { M[col * n + k] *= dinv; Inv[col * n + k] *= dinv; }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double f = M[r * n + col];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) { M[r * n + k] -= f * M[col * n + k]; Inv[r * n + k] -= f * Inv[col * n + k]; }
    }
  }
  return true;
}

// Cyclic Jacobi eigenvalue iteration for a symmetric matrix A (n x n,
// row-major, destroyed): on return lam holds the eigenvalues and U (row-major,
// columns = eigenvectors) satisfies A = U diag(lam) U^T.  Each rotation zeroes
// one off-diagonal entry with the symmetric 2x2 Schur decomposition
// (Golub and Van Loan, Matrix Computations, Sec. 8.5).
void jacobi_eigen(std::vector<double>& A, int n, std::vector<double>& lam, std::vector<double>& U) {
  U.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) U[i * n + i] = 1.0;
  double scale = 0.0;
  for (double v : A) scale += v * v;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += 2.0 * A[p * n + q] * A[p * n + q];
    if (off <= 1e-30 * scale) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (apq == 0.0) continue;
        const double tau = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
        for (int k = 0; k < n; ++k) {  // A <- A J (columns p, q)
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - sn * akq;
          A[k * n + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- J^T A (rows p, q)
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - sn * aqk;
          A[q * n + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {  // U <- U J
          const double ukp = U[k * n + p], ukq = U[k * n + q];
          U[k * n + p] = c * ukp - sn * ukq;
          U[k * n + q] = sn * ukp + c * ukq;
        }
      }
  }
  lam.resize(n);
  for (int i = 0; i < n; ++i) lam[i] = A[i * n + i];
}

}  // namespace

BlockPrecond block_inverses(const HostSetup& hs, const Coefs& op) {
  const int d = hs.dim, nphi = hs.nphi, ng = hs.ng;
  const int ns = d * nphi, nv = ng * ns;
  BlockPrecond out;
  out.ns = ns;
  out.ng = ng;
  out.factored = ng > 1;
  std::atomic<int> err{0};
  if (!out.factored) {
    // one time node: explicit inverse of rho|J| Tm Mbar + Cg K.  The block is
    // symmetric (K and Mbar are), so only its upper triangle is kept,
    // packed column by column: entry (r, c), r <= c, at c (c + 1) / 2 + r,
    // symmetrised from the two computed entries
    const size_t np = (size_t)nv * (nv + 1) / 2;
    out.P.resize((size_t)hs.n_elem * np);
    parallel_for(hs.n_elem, [&](int64_t e) {
      std::vector<double> K, Dm((size_t)nv * nv), Inv;
      element_stiffness(hs, e, K);
      for (int i = 0; i < ns; ++i)
        for (int i2 = 0; i2 < ns; ++i2) {
          const int c = i / nphi, k = i % nphi, c2 = i2 / nphi, k2 = i2 % nphi;
          double v = op.Cg[0] * K[i * ns + i2];
          if (c == c2) v += op.Tm[0] * elem_mass(hs, e, k, k2);
          Dm[i * nv + i2] = v;
        }
      if (!gj_inverse(Dm, nv, Inv)) { err = 1; return; }
      float* o = &out.P[(size_t)e * np];
      for (int col = 0; col < nv; ++col)
        for (int r = 0; r <= col; ++r)
          o[(size_t)col * (col + 1) / 2 + r] = (float)(0.5 * (Inv[r * nv + col] + Inv[col * nv + r]));
    });
    require(!err, SDG_EMESH, "singular diagonal block");
    return out;
  }
  // Several time nodes: the diagonal block is Tm (x) M_e + Cg (x) K_e with
  // M_e = rho_e|J_e| (I (x) Mref) (rho_e (I (x) curved_M) on a curved element).  With the generalised eigenvectors
  // K_e Q = M_e Q Lambda, Q^T M_e Q = I, it factors as
  //   (I (x) Q^-T) (Tm (x) I + Cg (x) Lambda) (I (x) Q^-1),
  // whose inverse is (I (x) Q) blockdiag_i (Tm + lambda_i Cg)^-1 (I (x) Q^T).
  // Stored per element: Q (ns x ns, row-major [ck][i]) and the ns inverses
  // (ng x ng, row-major [a][b]).
  // inverse of the Cholesky factor of a mass matrix M (nphi x nphi)
  auto chol_inverse = [nphi](const double* M, std::vector<double>& Linv) {
    std::vector<double> L((size_t)nphi * nphi, 0.0);
    for (int i = 0; i < nphi; ++i)
      for (int j = 0; j <= i; ++j) {
        double s = M[i * nphi + j];
        for (int k = 0; k < j; ++k) s -= L[i * nphi + k] * L[j * nphi + k];
        if (i == j) {
          if (!(s > 0.0)) return false;
          L[i * nphi + i] = std::sqrt(s);
        } else {
          L[i * nphi + j] = s / L[j * nphi + j];
        }
      }
    return gj_inverse(L, nphi, Linv);
  };
  std::vector<double> Linv_ref;
  require(chol_inverse(hs.Mref.data(), Linv_ref), SDG_EMESH, "reference mass matrix is not positive definite");
  out.Q.resize((size_t)hs.n_elem * ns * ns);
  out.B.resize((size_t)hs.n_elem * ns * ng * ng);
  parallel_for(hs.n_elem, [&](int64_t e) {
    std::vector<double> K, C((size_t)ns * ns), lam, U, Bi((size_t)ng * ng), BiInv, Lc;
    element_stiffness(hs, e, K);
    const double w = hs.elem_w[e], sw = std::sqrt(w);
    const bool curved_e = is_curved(hs, e);
    if (curved_e && !chol_inverse(&hs.curved_M[(size_t)hs.curved_idx[e] * nphi * nphi], Lc)) { err = 1; return; }
    const std::vector<double>& Linv = curved_e ? Lc : Linv_ref;
    // C = L^-1 K L^-T with L = sqrt(w) (I (x) Lref)
    auto Li = [&](int r, int col) {  // (I (x) Linv)[r][col]
      const int c = r / nphi, k = r % nphi, c2 = col / nphi, k2 = col % nphi;
      return c == c2 ? Linv[k * nphi + k2] : 0.0;
    };
    std::vector<double> T((size_t)ns * ns, 0.0);
    for (int r = 0; r < ns; ++r)
      for (int col = 0; col < ns; ++col) {
        double s = 0.0;
        for (int k = 0; k < ns; ++k) s += Li(r, k) * K[k * ns + col];
        T[r * ns + col] = s;
      }
    for (int r = 0; r < ns; ++r)
      for (int col = 0; col < ns; ++col) {
        double s = 0.0;
        for (int k = 0; k < ns; ++k) s += T[r * ns + k] * Li(col, k);
        C[r * ns + col] = s / w;
      }
    for (int r = 0; r < ns; ++r)  // exact symmetry before the eigen-solve
      for (int col = r + 1; col < ns; ++col) {
        const double m = 0.5 * (C[r * ns + col] + C[col * ns + r]);
        C[r * ns + col] = C[col * ns + r] = m;
      }
    jacobi_eigen(C, ns, lam, U);
    // Q = L^-T U = (1/sqrt(w)) (I (x) Linv^T) U
    float* Qe = &out.Q[(size_t)e * ns * ns];
    for (int r = 0; r < ns; ++r)
      for (int i = 0; i < ns; ++i) {
        double s = 0.0;
        for (int k = 0; k < ns; ++k) s += Li(k, r) * U[k * ns + i];
        Qe[r * ns + i] = (float)(s / sw);
      }
    float* Be = &out.B[(size_t)e * ns * ng * ng];
    for (int i = 0; i < ns; ++i) {
      for (int a = 0; a < ng; ++a)
        for (int b = 0; b < ng; ++b) Bi[a * ng + b] = op.Tm[a * ng + b] + lam[i] * op.Cg[a * ng + b];
      if (!gj_inverse(Bi, ng, BiInv)) { err = 1; return; }
      for (int a = 0; a < ng * ng; ++a) Be[i * ng * ng + a] = (float)BiInv[a];
    }
  });
  require(!err, SDG_EMESH, "singular diagonal block");
  return out;
}

// Patch preconditioner Pre2 (Appendix A, eqs. APPRE1, APPRE2): for each
// element i the velocity operator restricted to the stencil S_i of i and its
// face neighbours (the diagonal blocks of eq. pre1 and the neighbour blocks
// N_{l,m}), inverted, and the first block row of the inverse kept.  Stored
// in FP32 per element as P[i][e][q][r] = A_i^-1[r][(e, q)] (r, q < nb =
// N_gamma d N_phi, e < d + 2 stencil slots, zero for missing neighbours),
// with the stencil's element indices (slot 0 = i, -1 = none).
PatchPrecond patch_inverses(const HostSetup& hs, const Coefs& op) {
  const int d = hs.dim, nphi = hs.nphi, ng = hs.ng, nfe = d + 1;
  const int ns = d * nphi, nb = ng * ns, slots = d + 2;
  PatchPrecond out;
  out.nb = nb;
  out.slots = slots;
  out.P.assign((size_t)hs.n_elem * slots * nb * nb, 0.0f);
  out.nbr.assign((size_t)hs.n_elem * slots, -1);
  std::atomic<int> err{0};
  parallel_for(hs.n_elem, [&](int64_t i) {
    // stencil: i, then its face neighbours in local face order (each once)
    int64_t st[8];
    int n_s = 0;
    st[n_s++] = i;
    for (int f = 0; f < nfe; ++f) {
      const FaceRec& fr = hs.faces[hs.elem_face[i * nfe + f]];
      const int64_t o = (fr.left == i && fr.lf == f) ? fr.right : fr.left;
      if (o < 0) continue;
      bool seen = false;
      for (int q = 0; q < n_s; ++q) seen |= st[q] == o;
      if (!seen) st[n_s++] = o;
    }
    const int n = n_s * nb;
    std::vector<double> A((size_t)n * n, 0.0), K;
    auto add_block = [&](int p, int q, const std::vector<double>& Ks, bool mass) {
      // rows (a, c, k) of slot p, columns (b, c2, k2) of slot q:
      // Tm[a][b] delta_{c c2} w Mref[k][k2] (mass, p == q) + Cg[a][b] Ks[(c,k),(c2,k2)]
      for (int a = 0; a < ng; ++a)
        for (int b = 0; b < ng; ++b) {
          const double cg = op.Cg[a * ng + b], tm = op.Tm[a * ng + b];
          for (int r = 0; r < ns; ++r)
            for (int cc = 0; cc < ns; ++cc) {
              double v = cg * Ks[(size_t)r * ns + cc];
              if (mass && r / nphi == cc / nphi)
                v += tm * elem_mass(hs, st[p], r % nphi, cc % nphi);
              A[(size_t)(p * nb + a * ns + r) * n + q * nb + b * ns + cc] += v;
            }
        }
    };
    for (int p = 0; p < n_s; ++p) {
      element_stiffness(hs, st[p], K);
      add_block(p, p, K, true);
    }
    // neighbour blocks N_{p,q}: every face shared by two stencil elements
    for (int p = 0; p < n_s; ++p)
      for (int f = 0; f < nfe; ++f) {
        const int64_t j = hs.elem_face[st[p] * nfe + f];
        const FaceRec& fr = hs.faces[j];
        const int sp = (fr.left == st[p] && fr.lf == f) ? 0 : 1;
        const int64_t o = sp == 0 ? fr.right : fr.left;
        if (o < 0) continue;
        for (int q = 0; q < n_s; ++q) {
          if (q == p || st[q] != o) continue;
          K.assign((size_t)ns * ns, 0.0);
          face_coupling(hs, j, sp, 1 - sp, K);
          add_block(p, q, K, false);
        }
      }
    // first block row of A^-1: rows of A^-T E_0, solved as A^T Y = E_0
    std::vector<double> At((size_t)n * n), Y((size_t)n * nb, 0.0);
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) At[(size_t)c * n + r] = A[(size_t)r * n + c];
    for (int r = 0; r < nb; ++r) Y[(size_t)r * nb + r] = 1.0;
    if (!lu_solve(At, Y, n, nb)) { err = 1; return; }
    // A^-1[r][col] = Y[col][r]
    float* Pi = &out.P[(size_t)i * slots * nb * nb];
    for (int e = 0; e < n_s; ++e) {
      out.nbr[(size_t)i * slots + e] = (int32_t)st[e];
      for (int q = 0; q < nb; ++q)
        for (int r = 0; r < nb; ++r) Pi[((size_t)e * nb + q) * nb + r] = (float)Y[(size_t)(e * nb + q) * nb + r];
    }
  });
  require(!err, SDG_EMESH, "singular patch block");
  return out;
}

void set_anisotropic_faces(HostSetup& hs, const double* E) {
  const int ns = hs.nsig;
  hs.face_E.assign((size_t)hs.n_face * ns * ns, 0.0);
  hs.face_Cw.assign((size_t)hs.n_face * ns * ns, 0.0);
  int bad = 0;
  for (int64_t j = 0; j < hs.n_face; ++j) {
    const FaceRec& fr = hs.faces[j];
    double* Ej = &hs.face_E[(size_t)j * ns * ns];
    for (int a = 0; a < ns * ns; ++a) {
      double v = hs.face_wt[2 * j] * E[(size_t)fr.left * ns * ns + a];
      if (fr.right >= 0) v += hs.face_wt[2 * j + 1] * E[(size_t)fr.right * ns * ns + a];
      Ej[a] = v;
    }
    // The strain energy density is 1/2 s~^T W E~^-1 s~ and W E~^-1 is the
    // inverse of the symmetric E^ = E~ W^-1 (the tensor entries E_ijkl);
    // it is taken by Cholesky, which is also the positive-definiteness check
    auto wt = [&](int k) { return k < hs.dim ? 1.0 : 2.0; };
    std::vector<double> Lc((size_t)ns * ns, 0.0);
    for (int i = 0; i < ns && !bad; ++i)
      for (int k = 0; k <= i; ++k) {
        double sum = Ej[i * ns + k] / wt(k);
        for (int q = 0; q < k; ++q) sum -= Lc[i * ns + q] * Lc[k * ns + q];
        if (i == k) {
          if (!(sum > 0.0)) { bad = 1; break; }
          Lc[i * ns + i] = std::sqrt(sum);
        } else {
          Lc[i * ns + k] = sum / Lc[k * ns + k];
        }
      }
    if (bad) break;
    std::vector<double> Inv((size_t)ns * ns);
    for (int col = 0; col < ns; ++col) {
      std::vector<double> y(ns, 0.0);
      for (int i = 0; i < ns; ++i) {  // L y = e_col
        double sum = i == col ? 1.0 : 0.0;
        for (int q = 0; q < i; ++q) sum -= Lc[i * ns + q] * y[q];
        y[i] = sum / Lc[i * ns + i];
      }
      for (int i = ns - 1; i >= 0; --i) {  // L^T x = y
        double sum = y[i];
        for (int q = i + 1; q < ns; ++q) sum -= Lc[q * ns + i] * y[q];
        y[i] = sum / Lc[i * ns + i];
      }
      for (int i = 0; i < ns; ++i) Inv[i * ns + col] = y[i];
    }
    for (int i = 0; i < ns * ns; ++i) hs.face_Cw[(size_t)j * ns * ns + i] = Inv[i];
  }
  require(!bad, SDG_EINVAL, "dual-element stiffness is not symmetric positive definite");
}

}  // namespace sdg
