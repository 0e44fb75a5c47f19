// Internal declarations shared by the host setup, the HIP kernels and the
// C-ABI layer of the staggered space-time DG elasticity library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/sdg.h"

namespace sdg {

// ---------------------------------------------------------------- errors

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define SDG_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      throw ::sdg::Error(SDG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline void require(bool ok, int code, const std::string& msg) {
  if (!ok) throw Error(code, msg);
}

// ---------------------------------------------------------------- sizes

constexpr int kNumVariants = 9;
constexpr int kMaxGamma = 4;   // N_gamma <= 4 (p_gamma <= 3)
constexpr int kMaxRhs = 64;

inline int n_phi_of(int dim, int p) {
  return dim == 2 ? (p + 1) * (p + 2) / 2 : (p + 1) * (p + 2) * (p + 3) / 6;
}
inline int n_psi_of(int dim, int p) { return dim == 2 ? (p + 1) * (p + 1) : n_phi_of(3, p); }
inline int n_sig_of(int dim) { return dim * (dim + 1) / 2; }

// Per-face record used by the kernels.  right < 0 marks a free-surface face.
struct FaceRec {
  int32_t left, right;
  int32_t lf, rf;   // local face index of the face in its left/right element
};

// ---------------------------------------------------------------- host setup products

struct HostSetup {
  int dim = 0, p = 0, pg = 0, scheme = SDG_SCHEME_STDG;
  int nphi = 0, npsi = 0, ng = 1, nsig = 0;
  int64_t n_elem = 0, n_face = 0, n_bface = 0;
  double dt = 0.0;

  std::vector<FaceRec> faces;           // n_face
  std::vector<int32_t> elem_face;       // n_elem*(dim+1): face id of local face f
  std::vector<double> Dt;               // n_face*2*nphi*dim*npsi, canonical dual basis
  std::vector<double> face_lm;          // n_face*2: lambda_j, mu_j
  // anisotropic material (empty when isotropic): the Voigt stiffness of the
  // dual element, n_face * n_sigma^2 (row-major), and its compliance form
  // W E^-1 (W = 1 on normal, 2 on shear components) for the energy
  std::vector<double> face_E, face_Cw;
  std::vector<double> face_wt;          // n_face*2: |T_{left,j}|/|R_j|, |T_{right,j}|/|R_j| (1, 0 on the boundary)
  std::vector<double> elem_w;           // n_elem: rho_i |det J_i| (rho_i for a curved element)
  std::vector<double> elem_detJ;        // n_elem
  std::vector<double> elem_rho;         // n_elem
  std::vector<double> Mref;             // nphi*nphi reference mass matrix
  // unwrapped element vertices (n_elem*(dim+1)*dim) for point location
  std::vector<double> elem_xyz;
  // curved elements (2D; Section 3, sub-/iso-parametric maps of degree
  // curved_q): index of each element in the curved list (-1: straight),
  // their geometry nodes [c][node][dim] in the velocity node order of degree
  // curved_q, and their mass int phi_k phi_m (without rho; a curved element's
  // mass is elem_w * curved_M, a straight one's elem_w * Mref)
  int curved_q = 0;
  std::vector<int32_t> curved_idx;
  std::vector<int64_t> curved_ids;
  std::vector<double> curved_nodes;
  std::vector<double> curved_M;
  // time basis
  std::vector<double> tau, w, e0, e1, T;  // T is ng*ng row-major
  std::vector<double> Ext;                 // ng*ng: time basis of the slab evaluated on the next slab
};

// Curved elements given to build_host_setup: n elements (ids), each with
// its (q+1)(q+2)/2 geometry nodes (nodes[c][node][2]).
struct CurvedInput {
  int q = 0;
  int64_t n = 0;
  const int64_t* ids = nullptr;
  const double* nodes = nullptr;
};

// Build topology, geometry, bases and blocks.  Throws Error.
void build_host_setup(HostSetup& hs, int dim, int64_t n_vert, const double* xyz, int64_t n_elem,
                      const int64_t* elem, const double* period, int p, int pg, int scheme,
                      double dt, const double* lam, const double* mu, const double* rho,
                      const CurvedInput* curved = nullptr);
// Mass of element e (rho included): elem_w[e] * (curved_M or Mref)[k][m].
double elem_mass(const HostSetup& hs, int64_t e, int k, int m);

// Nodal basis values of element e at physical point x (nphi values); returns
// false if x is not in the closed element (tolerance tol in barycentric units).
bool eval_velocity_basis(const HostSetup& hs, int64_t e, const double* x, double* phi, double tol);
// First element (in [e_begin, e_end), default all) containing x, or -1.
int64_t locate_point(const HostSetup& hs, const double* x, int64_t e_begin = 0, int64_t e_end = -1);
// Canonical dual basis functions of face j at n points x (n*dim) -> out (n*npsi).
void eval_dual_canonical(const HostSetup& hs, const int64_t* elem, int64_t j, int64_t n,
                         const double* x, double* out);

// Compressed 3D operator: each face side's block of eq. (MD_3) as
//   Dt[k][l][m] = sum_m' C[m][m'] (a_l F_f[k][m'] - sum_a B[a][l] G_f[k][a][m'])
// with reference tables F_f, G_f per local face f, the change of basis C of
// the side (N_psi x N_psi), the face-term coefficients a (3 per side, zero on
// free-surface faces) and B = |J| J^-1 per element.
struct CompressedOp {
  int npsi = 0;
  std::vector<double> C;   // [face][side][m][m'] (zero for the missing side)
  std::vector<double> fa;  // [face][side][l]
  std::vector<double> eB;  // [elem][a][l]
  std::vector<double> F;   // [f][k][m']
  std::vector<double> G;   // [f][k][a][m']
  std::vector<double> face_area_ref;  // areas of the reference faces
};
void build_compressed(const HostSetup& hs, const int64_t* elem, CompressedOp& out);

// Anisotropic dual material: E_j = (|T_{l,j}| E_l + |T_{r,j}| E_r) / |R_j|
// from per-element Voigt matrices E~ (n_elem * n_sigma^2, tensor shear
// strains, E~ W^-1 symmetric) and the volume fractions of hs.face_wt; fills
// hs.face_E (E~_j) and hs.face_Cw (the energy's compliance W E~_j^-1).
// SDG_EINVAL if some E~_j W^-1 is not positive definite.
void set_anisotropic_faces(HostSetup& hs, const double* E);

// L2 projection of initial data (the state at t^{0,-}) onto the velocity
// space (which = 0, per element) or the dual space (which = 1, per face, in
// the canonical dual basis) with a rule exact to total degree `degree`
// (>= projection_min_degree): the points of the rule per cell, their
// weights, and the projection of the caller's values at those points
// (values [cell][q][comp], comp = dim or n_sigma; out [cell][comp][basis]).
int projection_min_degree(const HostSetup& hs, int which);
int projection_rule_size(const HostSetup& hs, int which, int degree);
void projection_points(const HostSetup& hs, const int64_t* elem, int which, int degree, double* pts,
                       double* wts);
void project_values(const HostSetup& hs, const int64_t* elem, int which, int degree, const double* values,
                    double* out);

// ---------------------------------------------------------------- kernel interface

// Small coefficient matrices used by the operator kernels (row-major, N_gamma <= 4).
struct Coefs {
  double Tm[kMaxGamma * kMaxGamma];  // mass time matrix   [a][b]
  double Cg[kMaxGamma * kMaxGamma];  // stress-from-gradient time matrix [a][b]
  double Cs[kMaxGamma * kMaxGamma];  // stress-from-input-stress matrix [a][q], q < sig_in_ng
  double send[kMaxGamma];            // end-of-slab weights gamma_a(1) for the stress output
};

enum FaceMode : int {
  kScatter = 0,   // z = D s written to the element slots
  kWriteStress = 1  // s written out (slab and/or end-of-slab value)
};

struct OpArgs {
  int64_t n_face, n_elem;
  const FaceRec* faces;
  const void* Dt;          // double or float blocks
  const double* face_lm;
  const double* face_E;    // anisotropic Voigt stiffness per face (n_sigma^2), or null (isotropic)
  const double* elem_w;
  const double* v;         // [elem][ng_in][d][nphi] (ng_in = NG, or 1 when v_spatial)
  const double* sig_in;    // [face][nsig][npsi] or null
  double* z;               // [elem][d+1][NG][d][nphi]  (kScatter)
  double* s_out;           // [face][NG][nsig][npsi]    (kWriteStress, optional)
  double* s_end;           // [face][nsig][npsi]        (kWriteStress, optional)
  const double* y_add;     // element kernel: optional extra term added to y
  double* y;               // element kernel output [elem][NG][d][nphi]
  const double* Mref;      // nphi*nphi (device)
  int use_g;               // 0: skip the gradient term (Cg == 0)
  int vsum;                // 1: replace the Hooke law by the Voigt sum (g_pq + g_qp), the
                           //    transpose of the scatter's use of the stress
  int sig_in_ng;           // time slots of sig_in (1 or NG); layout [face][q][s][m]
  int sig_in_Et;           // 1: apply E^T (Voigt -> gradient space) to the input stress
  int mass_identity;       // element kernel: y = Tm[a] v instead of Tm (x) w Mref v
  int v_spatial;           // element kernel: v has no time axis (mass applied with Tm[:,0])
  double y_scale;          // element kernel: y = y_scale * (...) (reserved, 1.0)
  int variant;             // operator face kernel: 0 = LDS flat loops, 1 = register-tiled
                           // with the most faces per block, 2 = register-tiled, half of it,
                           // 3 = column-parallel, persistent and pipelined, 4 = column-parallel,
                           // 5 = column-parallel reading blocks from HBM into registers,
                           // 6 = the same with the scatter summed across the face's lanes,
                           // 7 = one face per wavefront on the FP64 matrix cores,
                           // 8 = compressed 3D operator (blocks rebuilt from factors)
  // Several independent columns (right-hand sides) of the same mesh: the
  // launch grid's y index is the column and every per-column array is offset
  // by column * its stride (0 = shared by all columns).
  int n_cols;
  int z_f32 = 0;           // face slots z in FP32 (written by the FP32 face kernels of the
                           // operator apply, read by its element kernel); else FP64
  int bvariant;            // batched FP64 operator: 0 = column grid of the variant above,
                           // 1, 2 = matrix-core kernel with 8 or 16 columns per workgroup
  int64_t cs_v, cs_y, cs_z, cs_sig_in, cs_s_out, cs_s_end, cs_y_add;
  Coefs c;
  // compressed 3D operator (variant 8): per face side C [face][side][m][m']
  // (double or float as Dt), face-term coefficients [face][side][3], per
  // element B = |J| J^-1 [elem][3][3], reference tables F [4][k][m'] and
  // G [4][k][a][m']; cmpC == nullptr when not assembled
  const void* cmpC = nullptr;
  const double* cmpA = nullptr;
  const double* cmpB = nullptr;
  const double* cmpF = nullptr;
  const double* cmpG = nullptr;
  // Inside multi-system Arnoldi steps the operator skips the work of
  // converged systems, whose rows are no longer read: mask_active[s *
  // mask_stride] is system s's activity flag (null: no mask).  Systems are
  // the columns (grid y) of a batched solve, or the meshes of a mesh batch,
  // given per face and per element by face_sys / elem_sys.
  const int* mask_active = nullptr;
  int mask_stride = 0;
  // run_flag (null: always run): while *run_flag is 0 every operator
  // kernel returns at entry, so the iterations a solver queued past its
  // convergence cost only their launches.
  const int* run_flag = nullptr;
  const int* face_sys = nullptr;
  const int* elem_sys = nullptr;
  // curved elements (Section 3, sub-/iso-parametric maps): the element
  // kernels take element e's mass matrix from curved_M + curved_idx[e] *
  // N_phi^2 instead of Mref when curved_idx[e] >= 0 (null: no curved element)
  const int32_t* curved_idx = nullptr;
  const double* curved_M = nullptr;
  // one right-hand side, no mask: the element kernel also writes each
  // workgroup's sum of v . y (the CG inner product p . A p) to dot_part
  // [blockIdx.x] (null: not formed)
  double* dot_part = nullptr;
  // v and y hold FP32 values (the FP32-vector CG inside iterative
  // refinement: the FP32 operator of variant 3 and the element-blocked
  // kernel, one column)
  int vy_f32 = 0;
};

// Launch the face kernel and/or the element kernel for (dim, p, NG).
// prec: SDG_PREC_F64 or SDG_PREC_F32.  Returns false if not compiled in.
bool launch_face(int dim, int p, int ng, int prec, int mode, const OpArgs& a, hipStream_t s);
bool launch_elem(int dim, int p, int ng, const OpArgs& a, hipStream_t s);
bool have_kernels(int dim, int p, int ng);

// Material-gradient pieces of the discrete adjoint (one time slab):
//   face_out[2j]   += coef * sum_{a,m} wq[a] tr(g_a) sum_p Lam_s[a][pp][m]
//   face_out[2j+1] += coef * sum_{a,m,s} wq[a] Lam_s[a][s][m] (g_pq + g_qp)_a[m]
// with g = sum_sides Dt^T v (v: slab velocities [elem][a][c][k]).
struct GradArgs {
  int64_t n_face, n_elem;
  const FaceRec* faces;
  const double* Dt;
  const double* v;        // forward slab velocity (or the CN sum v^n + v^{n+1})
  const double* lam_s;    // adjoint stress slab [face][a][s][m]
  double* face_out;       // [face][2]
  double coef;            // -dt (space-time) or -dt/2 (Crank-Nicolson)
  double wq[kMaxGamma];
};
bool launch_grad_face(int dim, int p, int ng, const GradArgs& a, hipStream_t s);

// Time coefficients of the density gradient (see launch_grad_rho).
struct RhoCoefs {
  double Bq[kMaxGamma * kMaxGamma];  // applied to the slab velocity
  double Bo[kMaxGamma];              // applied to the start-of-slab velocity
};

// Inverses of the element diagonal blocks of the velocity operator (eq. pre1)
// with time coefficients op, in FP32.  One time node: explicit inverses,
// column-major per element (P).  Several: the factored form
// (I (x) Q) blockdiag_i (Tm + lambda_i Cg)^-1 (I (x) Q^T) from the generalised
// eigenvectors Q of the element stiffness and mass (Q [e][ck][i], B
// [e][i][a][b]).
struct BlockPrecond {
  bool factored = false;
  int ns = 0, ng = 0;
  std::vector<float> P, Q, B;
};
BlockPrecond block_inverses(const HostSetup& hs, const Coefs& op);

// Patch preconditioner (Appendix A, eqs. APPRE1-APPRE2): the first block row
// of the inverse of the velocity operator restricted to each element and its
// face neighbours, FP32, P[i][e][q][r] (nb = N_gamma d N_phi rows r and
// columns q per stencil slot e < slots = d + 2), and the stencil's element
// indices nbr[i][e] (slot 0 = i, -1 = no neighbour).
struct PatchPrecond {
  int nb = 0, slots = 0;
  std::vector<float> P;
  std::vector<int32_t> nbr;
};
PatchPrecond patch_inverses(const HostSetup& hs, const Coefs& op);

}  // namespace sdg
