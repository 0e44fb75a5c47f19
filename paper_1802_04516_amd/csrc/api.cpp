// C-ABI entry points (include/sdg.h): context lifecycle, assembly, operator
// application, one implicit time step, energy and point evaluation.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>

#include "context.hpp"

namespace sdg {

bool dispatch_2d(int which, int dim, int p, int ng, int prec, int mode, const OpArgs& a, hipStream_t s,
                 const GradArgs* ga = nullptr);
bool dispatch_3d(int which, int dim, int p, int ng, int prec, int mode, const OpArgs& a, hipStream_t s,
                 const GradArgs* ga = nullptr);

bool launch_face(int dim, int p, int ng, int prec, int mode, const OpArgs& a, hipStream_t s) {
  return dim == 2 ? dispatch_2d(0, dim, p, ng, prec, mode, a, s) : dispatch_3d(0, dim, p, ng, prec, mode, a, s);
}
bool launch_elem(int dim, int p, int ng, const OpArgs& a, hipStream_t s) {
  return dim == 2 ? dispatch_2d(1, dim, p, ng, SDG_PREC_F64, 0, a, s)
                  : dispatch_3d(1, dim, p, ng, SDG_PREC_F64, 0, a, s);
}
bool launch_grad_face(int dim, int p, int ng, const GradArgs& g, hipStream_t s) {
  OpArgs a{};
  return dim == 2 ? dispatch_2d(3, dim, p, ng, SDG_PREC_F64, 0, a, s, &g) : dispatch_3d(3, dim, p, ng, SDG_PREC_F64, 0, a, s, &g);
}
bool have_kernels(int dim, int p, int ng) {
  OpArgs a{};
  return dim == 2 ? dispatch_2d(2, dim, p, ng, SDG_PREC_F64, 0, a, nullptr)
                  : dispatch_3d(2, dim, p, ng, SDG_PREC_F64, 0, a, nullptr);
}

namespace {

thread_local std::string g_err;

template <class F>
int guard(F&& f) {
  try {
    f();
    g_err.clear();
    return SDG_OK;
  } catch (const Error& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return SDG_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return SDG_EINVAL;
  }
}

Ctx& ctx_of(sdg_ctx* c) {
  require(c != nullptr, SDG_EINVAL, "null context");
  return *reinterpret_cast<Ctx*>(c);
}

// small dense helpers for the N_gamma x N_gamma time matrices
std::vector<double> inverse(const std::vector<double>& A, int n) {
  std::vector<double> M = A, I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(M[r * n + c]) > std::fabs(M[piv * n + c])) piv = r;
    for (int k = 0; k < n; ++k) { std::swap(M[c * n + k], M[piv * n + k]); std::swap(I[c * n + k], I[piv * n + k]); }
    const double d = M[c * n + c];
    for (int k = 0; k < n; ++k) { M[c * n + k] /= d; I[c * n + k] /= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = M[r * n + c];
      for (int k = 0; k < n; ++k) { M[r * n + k] -= f * M[c * n + k]; I[r * n + k] -= f * I[c * n + k]; }
    }
  }
  return I;
}

void set_sq(double* dst, const std::vector<double>& m, int n, bool transpose) {
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) dst[a * n + b] = transpose ? m[b * n + a] : m[a * n + b];
}

OpArgs base_args(Ctx& c, int prec) {
  OpArgs a{};
  a.n_face = c.hs.n_face;
  a.n_elem = c.hs.n_elem;
  a.faces = c.d_faces.p;
  a.Dt = prec == SDG_PREC_F32 ? (const void*)c.d_Dt32.p : (const void*)c.d_Dt64.p;
  a.face_lm = c.d_face_lm.p;
  a.face_E = c.d_face_E.p;
  a.elem_w = c.d_elem_w.p;
  a.Mref = c.d_Mref.p;
  a.curved_idx = c.d_curved_idx.p;
  a.curved_M = c.d_curved_M.p;
  a.y_scale = 1.0;
  a.sig_in_ng = 1;
  a.cmpC = prec == SDG_PREC_F32 ? (const void*)c.d_cmpC32.p : (const void*)c.d_cmpC64.p;
  a.cmpA = c.d_cmpA.p;
  a.cmpB = c.d_cmpB.p;
  a.cmpF = c.d_cmpF.p;
  a.cmpG = c.d_cmpG.p;
  return a;
}

void check_prec(Ctx& c, int prec) {
  require(prec == SDG_PREC_F64 || prec == SDG_PREC_F32, SDG_EINVAL, "precision must be SDG_PREC_F64 or SDG_PREC_F32");
  require((c.precisions & prec) != 0, SDG_ESTATE, "operator blocks of this precision were not assembled");
}

}  // namespace

void apply_op(Ctx& c, const double* v, double* y, int prec, bool transpose, hipStream_t s, int ncols, void* z,
              const int* mask_active, double* dot_part, const int* run_flag) {
  require(!dot_part || (ncols == 1 && !mask_active), SDG_EINVAL, "the fused inner product takes one unmasked column");
  OpArgs a = base_args(c, prec);
  a.dot_part = dot_part;
  a.run_flag = run_flag;
  if (mask_active) {
    a.mask_active = mask_active;
    a.mask_stride = MultiSys::mask_stride();
    a.face_sys = c.d_face_sys.p;
    a.elem_sys = c.d_elem_sys.p;
  }
  a.variant = prec == SDG_PREC_F32 ? c.variant32 : c.variant64;
  a.v = v;
  a.z = z ? static_cast<double*>(z) : c.d_z.p;
  a.y = y;
  a.use_g = 1;
  a.c = transpose ? c.adj : c.op;
  a.n_cols = ncols;
  a.bvariant = prec == SDG_PREC_F32 ? c.bvariant32 : c.bvariant;
  a.cs_v = a.cs_y = c.n_slab;
  a.cs_z = c.z_col;
  a.z_f32 = prec == SDG_PREC_F32;
  launch_face(c.hs.dim, c.hs.p, c.hs.ng, prec, kScatter, a, s);
  SDG_HIP(hipGetLastError());
  launch_elem(c.hs.dim, c.hs.p, c.hs.ng, a, s);
  SDG_HIP(hipGetLastError());
}

// y = A32 v with FP32 vectors (one column, forward operator, FP32 face
// slots), for the FP32-vector CG inside iterative refinement; dot_part and
// run_flag as in apply_op.  Only the persistent face kernel (variant 3) and the
// element-blocked kernel take FP32 vectors: the caller checks
// fp32_vectors_ok first.
void apply_op_f32v(Ctx& c, const float* v, float* y, hipStream_t s, double* dot_part, const int* run_flag) {
  require(fp32_vectors_ok(c), SDG_EUNSUPPORTED, "no FP32-vector operator for this configuration");
  OpArgs a = base_args(c, SDG_PREC_F32);
  a.dot_part = dot_part;
  a.run_flag = run_flag;
  a.variant = c.variant32;
  a.v = reinterpret_cast<const double*>(v);  // FP32 values (vy_f32)
  a.y = reinterpret_cast<double*>(y);
  a.vy_f32 = 1;
  a.z = c.d_z.p;
  a.use_g = 1;
  a.c = c.op;
  a.n_cols = 1;
  a.bvariant = c.bvariant32;
  a.cs_v = a.cs_y = c.n_slab;
  a.cs_z = c.z_col;
  a.z_f32 = true;
  launch_face(c.hs.dim, c.hs.p, c.hs.ng, SDG_PREC_F32, kScatter, a, s);
  SDG_HIP(hipGetLastError());
  launch_elem(c.hs.dim, c.hs.p, c.hs.ng, a, s);
  SDG_HIP(hipGetLastError());
}

// The FP32-vector operator exists: the FP32 operator tuned to variant 3
// (the persistent face kernel), isotropic material, one time node and at
// most 256 values per element (the element-blocked kernel).
bool fp32_vectors_ok(const Ctx& c) {
  return (c.precisions & SDG_PREC_F32) && c.variant32 == 3 && !c.aniso && c.hs.ng == 1 &&
         c.hs.dim * c.hs.nphi <= 256;
}

// The compressed 3D operator (variant 8) exists for this precision.
static bool compressed_available(const Ctx& c, int prec) {
  return prec == SDG_PREC_F32 ? c.d_cmpC32.p != nullptr : c.d_cmpC64.p != nullptr;
}

// Face-kernel variants that apply an anisotropic Hooke law: the
// column-parallel kernels (3, 4) and the compressed operator (8).
static bool aniso_variant(int v) { return v == 3 || v == 4 || v == 8; }

// Time every face-kernel variant on the assembled operator and keep the
// fastest per precision (the project's tile-shape autotuner).
static void autotune(Ctx& c) {
  hipStream_t s = nullptr;
  hipEvent_t e0, e1;
  SDG_HIP(hipEventCreate(&e0));
  SDG_HIP(hipEventCreate(&e1));
  vec_fill(c.n_slab, 1.0, c.d_x.p, s);
  for (int pi = 0; pi < 2; ++pi) {
    const int prec = pi == 0 ? SDG_PREC_F64 : SDG_PREC_F32;
    if (!(c.precisions & prec)) continue;
    int best = 0;
    double best_t = 1e30;
    for (int var = 0; var < kNumVariants; ++var) {
      if ((var == 8 && !compressed_available(c, prec)) || (c.aniso && !aniso_variant(var))) {
        c.tune_us[pi][var] = 0.0;
        continue;
      }
      if (pi == 0) c.variant64 = var; else c.variant32 = var;
      for (int w = 0; w < 3; ++w) apply_op(c, c.d_x.p, c.d_r.p, prec, false, s);
      SDG_HIP(hipEventRecord(e0, s));
      const int reps = 10;
      for (int w = 0; w < reps; ++w) apply_op(c, c.d_x.p, c.d_r.p, prec, false, s);
      SDG_HIP(hipEventRecord(e1, s));
      SDG_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      SDG_HIP(hipEventElapsedTime(&ms, e0, e1));
      const double us = 1e3 * ms / reps;
      c.tune_us[pi][var] = us;
      if (us < best_t) { best_t = us; best = var; }
    }
    if (pi == 0) c.variant64 = best; else c.variant32 = best;
  }
  // batched applies: column grid against the matrix-core tile widths, per
  // precision (the matrix-core kernel applies the isotropic law only)
  c.bvariant = c.bvariant32 = 0;
  if (c.max_rhs > 1 && !c.aniso) {
    const int R = c.max_rhs;
    vec_fill(c.n_slab * R, 1.0, c.d_x.p, s);
    for (int pi = 0; pi < 2; ++pi) {
      const int prec = pi == 0 ? SDG_PREC_F64 : SDG_PREC_F32;
      if (!(c.precisions & prec)) continue;
      int& bvar = pi == 0 ? c.bvariant : c.bvariant32;
      double* tb = pi == 0 ? c.tune_b_us : c.tune_b32_us;
      int best = 0;
      double best_t = 1e30;
      for (int bv = 0; bv < 3; ++bv) {
        bvar = bv;
        apply_op(c, c.d_x.p, c.d_r.p, prec, false, s, R);
        SDG_HIP(hipEventRecord(e0, s));
        const int reps = 3;
        for (int w = 0; w < reps; ++w) apply_op(c, c.d_x.p, c.d_r.p, prec, false, s, R);
        SDG_HIP(hipEventRecord(e1, s));
        SDG_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        SDG_HIP(hipEventElapsedTime(&ms, e0, e1));
        tb[bv] = 1e3 * ms / reps;
        if (tb[bv] < best_t) { best_t = tb[bv]; best = bv; }
      }
      bvar = best;
    }
  }
  SDG_HIP(hipEventDestroy(e0));
  SDG_HIP(hipEventDestroy(e1));
}

void apply_precond(Ctx& c, int kind, const double* x, double* y, bool transpose, hipStream_t s, int ncols) {
  const HostSetup& hs = c.hs;
  if (kind == SDG_PRECOND_MASS) {
    OpArgs a = base_args(c, SDG_PREC_F64);
    a.Mref = c.d_Minv.p;
    a.curved_M = c.d_curved_Minv.p;
    a.elem_w = c.d_winv.p;
    a.v = x;
    a.y = y;
    a.c = transpose ? c.precA : c.precF;
    a.n_cols = ncols;
    a.cs_v = a.cs_y = c.n_slab;
    launch_elem(hs.dim, hs.p, hs.ng, a, s);
    SDG_HIP(hipGetLastError());
  } else if (kind == SDG_PRECOND_PATCH) {
    require(c.d_P2.p != nullptr, SDG_ESTATE, "patch preconditioner not assembled (pass SDG_ASSEMBLE_PATCH_PRECOND)");
    require(!transpose, SDG_EUNSUPPORTED, "the transposed patch preconditioner is not built");
    launch_patch_apply(hs.n_elem, c.p2_nb, c.p2_slots, c.d_P2.p, c.d_P2nbr.p, x, y, s, ncols, c.n_slab);
  } else if (kind == SDG_PRECOND_BLOCK) {
    require(c.d_Pblk.p != nullptr || c.d_Pq.p != nullptr, SDG_ESTATE,
            "block preconditioner not assembled (pass SDG_ASSEMBLE_BLOCK_PRECOND)");
    if (c.pblk_factored)
      launch_block_apply_fact(hs.n_elem, hs.ng, hs.dim * hs.nphi, c.d_Pq.p, c.d_Pb.p, x, y, transpose, s, ncols,
                              c.n_slab);
    else
      launch_block_apply(hs.n_elem, hs.ng * hs.dim * hs.nphi, c.d_Pblk.p, x, y, transpose, s, ncols, c.n_slab);
  } else {
    vec_copy(c.n_slab * ncols, x, y, s);
  }
}

// Elements and nodal basis values of sampling points, located on the host and
// kept on the device: repeated calls with the same points reuse them.
void locate_points(Ctx& c, int64_t n_pts, const double* pts) {
  const HostSetup& hs = c.hs;
  const size_t nd = (size_t)n_pts * hs.dim;
  if (c.samp_pts.size() == nd && std::equal(pts, pts + nd, c.samp_pts.begin()) && c.d_samp_elem.p) return;
  std::vector<int64_t> el(n_pts);
  std::vector<double> phi((size_t)n_pts * hs.nphi);
  for (int64_t q = 0; q < n_pts; ++q) {
    el[q] = locate_point(hs, pts + q * hs.dim);
    require(el[q] >= 0, SDG_EINVAL, "sample point outside the mesh");
    eval_velocity_basis(hs, el[q], pts + q * hs.dim, &phi[q * hs.nphi], 1e-12);
  }
  c.d_samp_elem.alloc(n_pts);
  c.d_samp_phi.alloc(phi.size());
  SDG_HIP(hipMemcpy(c.d_samp_elem.p, el.data(), el.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  SDG_HIP(hipMemcpy(c.d_samp_phi.p, phi.data(), phi.size() * sizeof(double), hipMemcpyHostToDevice));
  c.samp_pts.assign(pts, pts + nd);
}

// Right-hand side of eq. (velocity.sys) (or velocity.sys.cn) for R columns
// into d_b (point sources from d_src_amp when src), and the initial guess
// (old state at every time node) into d_x.
void step_rhs(Ctx& c, const double* v_state, const double* sigma_state, int R, bool src, hipStream_t s,
              bool extrap, int hist = 0) {
  const HostSetup& hs = c.hs;
  const int d = hs.dim, ng = hs.ng, nvs = d * hs.nphi;
  const double dt = hs.dt;
  if (c.scheme == SDG_SCHEME_CN) {
    OpArgs a = base_args(c, SDG_PREC_F64);
    a.v = v_state;
    a.sig_in = sigma_state;
    a.z = c.d_z.p;
    a.y = c.d_b.p;
    a.use_g = 1;
    a.c.Cg[0] = -dt * dt / 4.0;
    a.c.Cs[0] = dt;
    a.c.Tm[0] = 1.0;
    a.n_cols = R;
    a.cs_v = c.n_state;
    a.cs_sig_in = c.n_sig_state;
    a.cs_z = c.z_col;
    a.cs_y = c.n_slab;
    launch_face(d, hs.p, 1, SDG_PREC_F64, kScatter, a, s);
    launch_elem(d, hs.p, 1, a, s);
  } else {
    std::vector<double> Ti = inverse(hs.T, ng);
    OpArgs a = base_args(c, SDG_PREC_F64);
    a.sig_in = sigma_state;
    a.z = c.d_z.p;
    a.use_g = 0;
    a.c.Cs[0] = 1.0;
    a.n_cols = R;
    a.cs_sig_in = c.n_sig_state;
    a.cs_z = c.z_col;
    launch_face(d, hs.p, 1, SDG_PREC_F64, kScatter, a, s);
    OpArgs e = base_args(c, SDG_PREC_F64);
    e.v = v_state;
    e.v_spatial = 1;
    e.z = c.d_z.p;
    e.y = c.d_b.p;
    e.n_cols = R;
    e.cs_v = c.n_state;
    e.cs_z = c.z_col;
    e.cs_y = c.n_slab;
    for (int aa = 0; aa < ng; ++aa) {
      e.c.Tm[aa * ng] = hs.e0[aa];
      double q = 0.0;
      for (int b = 0; b < ng; ++b) q += Ti[aa * ng + b] * hs.e0[b];
      e.c.Cs[aa] = dt * hs.w[aa] * q;
    }
    launch_elem(d, hs.p, ng, e, s);
  }
  SDG_HIP(hipGetLastError());
  if (src) launch_add_sources(c, c.d_b.p, c.d_src_amp.p, s, R);
  if (extrap && hist >= 2) {
    // one-node slabs: the trajectory of the last slabs extrapolated in time,
    // linearly (2 x_n - x_{n-1}) or quadratically (3 x_n - 3 x_{n-1} + x_{n-2})
    const int64_t N = c.n_slab * R;
    if (hist >= 3) {
      vec_copy(N, c.d_prev3.p, c.d_x.p, s);
      vec_axpby(N, 3.0, c.d_prev.p, 1.0, c.d_x.p, s);
      vec_axpby(N, -3.0, c.d_prev2.p, 1.0, c.d_x.p, s);
    } else {
      vec_copy(N, c.d_prev.p, c.d_x.p, s);
      vec_axpby(N, -1.0, c.d_prev2.p, 2.0, c.d_x.p, s);
    }
  } else if (extrap) {
    launch_time_map(hs.n_elem * R, ng, nvs, hs.Ext.data(), c.d_prev.p, c.d_x.p, s);
  } else {
    launch_broadcast_time(hs.n_elem * R, ng, nvs, v_state, c.d_x.p, s);
  }
}

// Stress back-substitution (eq. NM26 or NM26.cn) from the velocity slab in
// d_x, then the end-of-slab state, for R columns.
void step_backsub(Ctx& c, double* v_state, double* sigma_state, double* v_slab, double* sigma_slab, int R,
                  hipStream_t s, bool extrap, bool hist = false) {
  const HostSetup& hs = c.hs;
  const int d = hs.dim, ng = hs.ng, nvs = d * hs.nphi;
  const double dt = hs.dt;
  const int64_t N = c.n_slab * R;
  OpArgs a = base_args(c, SDG_PREC_F64);
  a.sig_in = sigma_state;
  a.use_g = 1;
  a.s_out = sigma_slab;
  a.s_end = c.d_tmp_sig.p;
  a.n_cols = R;
  a.cs_v = c.n_slab;
  a.cs_sig_in = c.n_sig_state;
  a.cs_s_out = hs.n_face * ng * hs.nsig * hs.npsi;
  a.cs_s_end = c.n_sig_state;
  if (c.scheme == SDG_SCHEME_CN) {
    vec_copy(N, v_state, c.d_t.p, s);
    vec_axpby(N, 1.0, c.d_x.p, 1.0, c.d_t.p, s);  // v^n + v^{n+1}
    a.v = c.d_t.p;
    a.c.Cg[0] = -dt / 2.0;
    a.c.Cs[0] = 1.0;
    a.c.send[0] = 1.0;
    launch_face(d, hs.p, 1, SDG_PREC_F64, kWriteStress, a, s);
    SDG_HIP(hipGetLastError());
    vec_copy(c.n_sig_state * R, c.d_tmp_sig.p, sigma_state, s);
    if (v_slab) vec_copy(N, c.d_x.p, v_slab, s);
    vec_copy(c.n_state * R, c.d_x.p, v_state, s);
  } else {
    std::vector<double> Ti = inverse(hs.T, ng);
    a.v = c.d_x.p;
    for (int aa = 0; aa < ng; ++aa) {
      double q = 0.0;
      for (int b = 0; b < ng; ++b) {
        a.c.Cg[aa * ng + b] = -dt * Ti[aa * ng + b] * hs.w[b];
        q += Ti[aa * ng + b] * hs.e0[b];
      }
      a.c.Cs[aa] = q;
      a.c.send[aa] = hs.e1[aa];
    }
    launch_face(d, hs.p, ng, SDG_PREC_F64, kWriteStress, a, s);
    SDG_HIP(hipGetLastError());
    vec_copy(c.n_sig_state * R, c.d_tmp_sig.p, sigma_state, s);
    if (v_slab) vec_copy(N, c.d_x.p, v_slab, s);
    launch_end_of_slab(hs.n_elem * R, ng, nvs, c.d_e1.p, c.d_x.p, v_state, s);
  }
  if (extrap && hist) {
    // the oldest slab's buffer takes the new one
    std::swap(c.d_prev3.p, c.d_prev2.p);
    std::swap(c.d_prev2.p, c.d_prev.p);
  }
  if (extrap) vec_copy(N, c.d_x.p, c.d_prev.p, s);
}

// Partition of the independent systems of a batched solve with ncols columns,
// or of the meshes of a mesh batch (rebuilt when the column count changes).
// Sources are located on one mesh with one velocity basis; a new mesh or
// degree makes their element indices and basis values meaningless.
void clear_sources(Ctx& c) {
  c.n_src = 0;
  c.p_src = 0;
  c.src_elem.clear();
  c.src_phi.clear();
  c.src_dir.clear();
  c.d_src_elem.free();
  c.d_src_phi.free();
  c.d_src_dir.free();
  c.graphs.clear();
}

MultiSys& systems(Ctx& c, int ncols) {
  const int key = c.n_mesh > 1 ? -1 : ncols;
  if (c.msys_key != key) {
    std::vector<int64_t> off;
    if (c.n_mesh > 1) {
      const int64_t per = (int64_t)c.hs.ng * c.hs.dim * c.hs.nphi;
      for (int64_t e : c.mesh_elem_off) off.push_back(e * per);
    } else {
      for (int r = 0; r <= ncols; ++r) off.push_back((int64_t)r * c.n_slab);
    }
    c.graphs.clear();  // recorded graphs point into the old partition
    c.msys.build(off);
    c.msys_key = key;
  }
  return c.msys;
}

}  // namespace sdg

using namespace sdg;

extern "C" {

const char* sdg_last_error(void) { return g_err.c_str(); }

int sdg_create(sdg_ctx** out, int device) {
  if (out) *out = nullptr;
  return guard([&] {
    require(out != nullptr, SDG_EINVAL, "null output pointer");
    int n = 0;
    SDG_HIP(hipGetDeviceCount(&n));
    require(device >= 0 && device < n, SDG_EDEVICE, "no such HIP device");
    SDG_HIP(hipSetDevice(device));
    // resolve this device's copy of the allocation-free apply's scratch
    // array now, once per device, with the device current
    (void)noalloc_scratch(device);
    Ctx* c = new Ctx();
    c->device = device;
    *out = reinterpret_cast<sdg_ctx*>(c);
  });
}

void sdg_destroy(sdg_ctx* ctx) {
  if (!ctx) return;
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  delete c;
}

int sdg_set_mesh(sdg_ctx* ctx, int dim, int64_t n_vert, const double* xyz, int64_t n_elem, const int64_t* elem,
                 const double* period) {
  return guard([&] {
    Ctx& c = ctx_of(ctx);
    require(dim == 2 || dim == 3, SDG_EINVAL, "dim must be 2 or 3");
    require(n_vert > 0 && n_elem > 0 && xyz && elem, SDG_EINVAL, "empty mesh");
    require(n_elem < (int64_t)1 << 31, SDG_EINVAL, "too many elements");
    c.dim = dim;
    c.xyz.assign(xyz, xyz + n_vert * dim);
    c.elem.assign(elem, elem + n_elem * (dim + 1));
    c.n_mesh = 1;
    c.mesh_vert_off = {0, n_vert};
    c.mesh_elem_off = {0, n_elem};
    if (period) {
      c.period.assign(period, period + dim);
      for (double P : c.period) require(P > 0 && std::isfinite(P), SDG_EINVAL, "period must be positive");
    } else {
      c.period.clear();
    }
    for (double x : c.xyz) require(std::isfinite(x), SDG_EINVAL, "non-finite vertex coordinate");
    clear_sources(c);
    c.curved_q = 0;
    c.curved_ids.clear();
    c.curved_nodes.clear();
    c.have_mesh = true;
    c.assembled = false;
  });
}

int sdg_set_curved_elements(sdg_ctx* ctx, int q, int64_t n_curved, const int64_t* elem_ids, const double* nodes) {
  return guard([&] {
    Ctx& c = ctx_of(ctx);
    require(c.have_mesh, SDG_ESTATE, "set the mesh first");
    require(n_curved >= 0, SDG_EINVAL, "negative count");
    if (n_curved == 0) {
      c.curved_q = 0;
      c.curved_ids.clear();
      c.curved_nodes.clear();
      c.assembled = false;
      return;
    }
    require(c.dim == 2, SDG_EUNSUPPORTED, "curved elements are supported in 2D");
    require(c.period.empty() && c.n_mesh == 1, SDG_EUNSUPPORTED,
            "curved elements need a single non-periodic mesh");
    require(q >= 1 && q <= 4, SDG_EINVAL, "geometry degree must be 1..4");
    require(elem_ids && nodes, SDG_EINVAL, "null curved-element array");
    const int64_t nq = (int64_t)(q + 1) * (q + 2) / 2;
    clear_sources(c);  // their basis values depend on the geometry
    c.curved_q = q;
    c.curved_ids.assign(elem_ids, elem_ids + n_curved);
    c.curved_nodes.assign(nodes, nodes + n_curved * nq * c.dim);
    c.assembled = false;
  });
}

int sdg_set_mesh_batch(sdg_ctx* ctx, int dim, int n_mesh, const int64_t* vert_off, const double* xyz,
                       const int64_t* elem_off, const int64_t* elem) {
  return guard([&] {
    Ctx& c = ctx_of(ctx);
    require(dim == 2 || dim == 3, SDG_EINVAL, "dim must be 2 or 3");
    require(n_mesh >= 1 && n_mesh <= kMaxSystems, SDG_EINVAL, "n_mesh must be in [1, 1024]");
    require(vert_off && xyz && elem_off && elem, SDG_EINVAL, "null mesh array");
    require(vert_off[0] == 0 && elem_off[0] == 0, SDG_EINVAL, "offsets must start at 0");
    for (int q = 0; q < n_mesh; ++q)
      require(vert_off[q + 1] > vert_off[q] && elem_off[q + 1] > elem_off[q], SDG_EINVAL,
              "every mesh of the batch needs vertices and elements");
    const int64_t nv = vert_off[n_mesh], ne = elem_off[n_mesh];
    require(ne < (int64_t)1 << 31, SDG_EINVAL, "too many elements");
    const int nvpe = dim + 1;
    std::vector<int64_t> el((size_t)ne * nvpe);
    for (int q = 0; q < n_mesh; ++q) {
      const int64_t nvq = vert_off[q + 1] - vert_off[q];
      for (int64_t e = elem_off[q]; e < elem_off[q + 1]; ++e)
        for (int k = 0; k < nvpe; ++k) {
          const int64_t v = elem[e * nvpe + k];
          require(v >= 0 && v < nvq, SDG_EMESH, "vertex index outside its mesh");
          el[e * nvpe + k] = v + vert_off[q];
        }
    }
    c.dim = dim;
    c.xyz.assign(xyz, xyz + nv * dim);
    for (double x : c.xyz) require(std::isfinite(x), SDG_EINVAL, "non-finite vertex coordinate");
    c.elem.swap(el);
    c.period.clear();
    c.n_mesh = n_mesh;
    c.mesh_vert_off.assign(vert_off, vert_off + n_mesh + 1);
    c.mesh_elem_off.assign(elem_off, elem_off + n_mesh + 1);
    clear_sources(c);
    c.curved_q = 0;
    c.curved_ids.clear();
    c.curved_nodes.clear();
    c.have_mesh = true;
    c.assembled = false;
  });
}

int sdg_set_discretization(sdg_ctx* ctx, int p, int p_gamma, int scheme, double dt) {
  return guard([&] {
    Ctx& c = ctx_of(ctx);
    require(c.have_mesh, SDG_ESTATE, "set the mesh first");
    require(p >= 1 && p_gamma >= 0 && p_gamma + 1 <= kMaxGamma, SDG_EINVAL, "degree out of range");
    require(scheme == SDG_SCHEME_STDG || scheme == SDG_SCHEME_CN, SDG_EINVAL, "unknown scheme");
    require(scheme != SDG_SCHEME_CN || p_gamma == 0, SDG_EINVAL, "Crank-Nicolson requires p_gamma = 0");
    require(dt > 0 && std::isfinite(dt), SDG_EINVAL, "dt must be positive");
    require(have_kernels(c.dim, p, p_gamma + 1), SDG_EUNSUPPORTED,
            "no kernels compiled for dim=" + std::to_string(c.dim) + " p=" + std::to_string(p) +
                " N_gamma=" + std::to_string(p_gamma + 1));
    require(have_kernels(c.dim, p, 1), SDG_EUNSUPPORTED, "no N_gamma=1 kernels for this degree");
    c.p = p;
    c.pg = p_gamma;
    c.scheme = scheme;
    c.dt = dt;
    if (p != c.p_src) clear_sources(c);
    c.have_disc = true;
    c.assembled = false;
  });
}

int sdg_set_material(sdg_ctx* ctx, const double* lambda, const double* mu, const double* rho) {
  return guard([&] {
    Ctx& c = ctx_of(ctx);
    require(c.have_mesh, SDG_ESTATE, "set the mesh first");
    require(lambda && mu && rho, SDG_EINVAL, "null material array");
    const size_t n = c.elem.size() / (c.dim + 1);
    c.lam.assign(lambda, lambda + n);
    c.mu.assign(mu, mu + n);
    c.rho.assign(rho, rho + n);
    for (size_t i = 0; i < n; ++i)
      require(std::isfinite(lambda[i]) && std::isfinite(mu[i]) && std::isfinite(rho[i]) && lambda[i] >= 0 &&
                  mu[i] > 0 && rho[i] > 0,
              SDG_EINVAL, "material parameters must be finite with lambda >= 0, mu > 0, rho > 0");
    c.aniso = false;
    c.elemE.clear();
    c.have_mat = true;
    c.assembled = false;
  });
}

int sdg_set_material_anisotropic(sdg_ctx* ctx, const double* stiffness, const double* rho) {
  return guard([&] {
    Ctx& c = ctx_of(ctx);
    require(c.have_mesh, SDG_ESTATE, "set the mesh first");
    require(stiffness && rho, SDG_EINVAL, "null material array");
    const size_t n = c.elem.size() / (c.dim + 1);
    const int ns = n_sig_of(c.dim);
    c.elemE.assign(stiffness, stiffness + n * ns * ns);
    c.rho.assign(rho, rho + n);
    // E~ W^-1 (W = 1 on normal, 2 on shear components) holds the tensor
    // entries E_ijkl and is symmetric by the major symmetry; it is made
    // exactly symmetric here
    auto wt = [&](int k) { return k < c.dim ? 1.0 : 2.0; };
    for (size_t i = 0; i < n; ++i) {
      require(std::isfinite(rho[i]) && rho[i] > 0, SDG_EINVAL, "density must be finite and positive");
      double* E = &c.elemE[i * ns * ns];
      double scale = 0.0;
      for (int a = 0; a < ns * ns; ++a) {
        require(std::isfinite(E[a]), SDG_EINVAL, "non-finite stiffness entry");
        scale = std::max(scale, std::fabs(E[a]));
      }
      for (int a = 0; a < ns; ++a)
        for (int b = a + 1; b < ns; ++b) {
          const double x = E[a * ns + b] / wt(b), y = E[b * ns + a] / wt(a);
          require(std::fabs(x - y) <= 1e-12 * scale, SDG_EINVAL,
                  "stiffness violates the major symmetry (E~ W^-1 must be symmetric)");
          const double m = 0.5 * (x + y);
          E[a * ns + b] = m * wt(b);
          E[b * ns + a] = m * wt(a);
        }
    }
    // the isotropic parameters are not used with an anisotropic material; the
    // set-up's own checks take positive placeholders
    c.lam.assign(n, 1.0);
    c.mu.assign(n, 1.0);
    c.aniso = true;
    c.have_mat = true;
    c.assembled = false;
  });
}

int sdg_assemble(sdg_ctx* ctx, unsigned precisions, int max_rhs) {
  return guard([&] {
    Ctx& c = ctx_of(ctx);
    require(c.have_mesh && c.have_disc && c.have_mat, SDG_ESTATE, "mesh, discretization and material must be set");
    require((precisions & (SDG_PREC_F64 | SDG_PREC_F32)) != 0 && (precisions & ~15u) == 0, SDG_EINVAL,
            "precisions must be a non-empty subset of SDG_PREC_F64 | SDG_PREC_F32 (| SDG_ASSEMBLE_BLOCK_PRECOND "
            "| SDG_ASSEMBLE_PATCH_PRECOND)");
    require(max_rhs >= 1 && max_rhs <= kMaxSystems, SDG_EINVAL, "max_rhs must be in [1, 1024]");
    require(max_rhs == 1 || c.n_mesh == 1, SDG_EUNSUPPORTED, "batched right-hand sides on a mesh batch");
    SDG_HIP(hipSetDevice(c.device));
    c.assembled = false;
    c.msys_key = 0;
    c.samp_pts.clear();
    c.graphs.clear();
    HostSetup& hs = c.hs;
    const int64_t n_elem = (int64_t)(c.elem.size() / (c.dim + 1));
    const int64_t n_vert = (int64_t)(c.xyz.size() / c.dim);
    CurvedInput cin;
    cin.q = c.curved_q;
    cin.n = (int64_t)c.curved_ids.size();
    cin.ids = c.curved_ids.data();
    cin.nodes = c.curved_nodes.data();
    build_host_setup(hs, c.dim, n_vert, c.xyz.data(), n_elem, c.elem.data(), c.period.empty() ? nullptr : c.period.data(),
                     c.p, c.pg, c.scheme, c.dt, c.lam.data(), c.mu.data(), c.rho.data(), &cin);
    hs.face_E.clear();
    hs.face_Cw.clear();
    if (c.aniso) set_anisotropic_faces(hs, c.elemE.data());
    const int d = hs.dim, ng = hs.ng, nphi = hs.nphi;
    c.mesh_face_off.assign(c.n_mesh + 1, hs.n_face);
    {
      // faces are ordered by left element and never join two meshes
      int64_t j = 0;
      for (int q = 0; q < c.n_mesh; ++q) {
        while (j < hs.n_face && hs.faces[j].left < c.mesh_elem_off[q]) ++j;
        c.mesh_face_off[q] = j;
      }
    }
    c.d_face_sys.free();
    c.d_elem_sys.free();
    if (c.n_mesh > 1) {
      // mesh of each face and element: the systems of a mesh-batch solve
      std::vector<int> fs(hs.n_face), es(hs.n_elem);
      for (int q = 0; q < c.n_mesh; ++q) {
        for (int64_t e = c.mesh_elem_off[q]; e < c.mesh_elem_off[q + 1]; ++e) es[e] = q;
        const int64_t f1 = q + 1 < c.n_mesh ? c.mesh_face_off[q + 1] : hs.n_face;
        for (int64_t f = c.mesh_face_off[q]; f < f1; ++f) fs[f] = q;
      }
      c.d_face_sys.alloc(fs.size());
      SDG_HIP(hipMemcpy(c.d_face_sys.p, fs.data(), fs.size() * sizeof(int), hipMemcpyHostToDevice));
      c.d_elem_sys.alloc(es.size());
      SDG_HIP(hipMemcpy(c.d_elem_sys.p, es.data(), es.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    c.n_slab = hs.n_elem * ng * d * nphi;
    c.n_state = hs.n_elem * d * nphi;
    c.n_sig_state = hs.n_face * hs.nsig * hs.npsi;
    c.precisions = precisions & 3u;
    c.max_rhs = max_rhs;

    // time coefficients
    const double dt = hs.dt;
    Coefs op{}, adj{};
    if (c.scheme == SDG_SCHEME_CN) {
      op.Tm[0] = 1.0;
      op.Cg[0] = dt * dt / 4.0;
    } else {
      std::vector<double> Ti = inverse(hs.T, ng), WTW(ng * ng);
      for (int a = 0; a < ng; ++a)
        for (int b = 0; b < ng; ++b) WTW[a * ng + b] = dt * dt * hs.w[a] * Ti[a * ng + b] * hs.w[b];
      set_sq(op.Tm, hs.T, ng, false);
      set_sq(op.Cg, WTW, ng, false);
      set_sq(adj.Tm, hs.T, ng, true);
      set_sq(adj.Cg, WTW, ng, true);
    }
    if (c.scheme == SDG_SCHEME_CN) adj = op;
    c.op = op;
    c.adj = adj;
    // mass block-Jacobi preconditioner: (Tm (x) w Mref)^-1 = Tm^-1 (x) w^-1 Mref^-1
    {
      Coefs pf{}, pa{};
      std::vector<double> Tm(ng * ng);
      for (int a = 0; a < ng * ng; ++a) Tm[a] = op.Tm[a];
      std::vector<double> Ti = inverse(Tm, ng);
      set_sq(pf.Tm, Ti, ng, false);
      set_sq(pa.Tm, Ti, ng, true);
      c.precF = pf;
      c.precA = pa;
      std::vector<double> Mi = inverse(hs.Mref, nphi);
      c.d_Minv.alloc(Mi.size());
      SDG_HIP(hipMemcpy(c.d_Minv.p, Mi.data(), Mi.size() * sizeof(double), hipMemcpyHostToDevice));
      std::vector<double> wi(hs.n_elem);
      for (int64_t e = 0; e < hs.n_elem; ++e) wi[e] = 1.0 / hs.elem_w[e];
      c.d_winv.alloc(wi.size());
      SDG_HIP(hipMemcpy(c.d_winv.p, wi.data(), wi.size() * sizeof(double), hipMemcpyHostToDevice));
      // curved elements: their own mass matrices and inverses
      c.d_curved_idx.free();
      c.d_curved_M.free();
      c.d_curved_Minv.free();
      if (!hs.curved_ids.empty()) {
        c.d_curved_idx.alloc(hs.curved_idx.size());
        SDG_HIP(hipMemcpy(c.d_curved_idx.p, hs.curved_idx.data(), hs.curved_idx.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice));
        c.d_curved_M.alloc(hs.curved_M.size());
        SDG_HIP(hipMemcpy(c.d_curved_M.p, hs.curved_M.data(), hs.curved_M.size() * sizeof(double),
                          hipMemcpyHostToDevice));
        std::vector<double> Ci(hs.curved_M.size());
        for (size_t k = 0; k < hs.curved_ids.size(); ++k) {
          std::vector<double> Mk(hs.curved_M.begin() + k * nphi * nphi, hs.curved_M.begin() + (k + 1) * nphi * nphi);
          std::vector<double> Mi2 = inverse(Mk, nphi);
          std::copy(Mi2.begin(), Mi2.end(), Ci.begin() + k * nphi * nphi);
        }
        c.d_curved_Minv.alloc(Ci.size());
        SDG_HIP(hipMemcpy(c.d_curved_Minv.p, Ci.data(), Ci.size() * sizeof(double), hipMemcpyHostToDevice));
      }
    }
    c.d_Pblk.free();
    c.d_Pq.free();
    c.d_Pb.free();
    c.pblk_factored = false;
    if (precisions & SDG_ASSEMBLE_BLOCK_PRECOND) {
      BlockPrecond bp = block_inverses(hs, op);
      c.pblk_factored = bp.factored;
      if (bp.factored) {
        c.d_Pq.alloc(bp.Q.size());
        SDG_HIP(hipMemcpy(c.d_Pq.p, bp.Q.data(), bp.Q.size() * sizeof(float), hipMemcpyHostToDevice));
        c.d_Pb.alloc(bp.B.size());
        SDG_HIP(hipMemcpy(c.d_Pb.p, bp.B.data(), bp.B.size() * sizeof(float), hipMemcpyHostToDevice));
      } else {
        c.d_Pblk.alloc(bp.P.size());
        SDG_HIP(hipMemcpy(c.d_Pblk.p, bp.P.data(), bp.P.size() * sizeof(float), hipMemcpyHostToDevice));
      }
    }

    c.d_P2.free();
    c.d_P2nbr.free();
    c.p2_nb = c.p2_slots = 0;
    if (precisions & SDG_ASSEMBLE_PATCH_PRECOND) {
      PatchPrecond pp = patch_inverses(hs, op);
      c.d_P2.alloc(pp.P.size());
      SDG_HIP(hipMemcpy(c.d_P2.p, pp.P.data(), pp.P.size() * sizeof(float), hipMemcpyHostToDevice));
      c.d_P2nbr.alloc(pp.nbr.size());
      SDG_HIP(hipMemcpy(c.d_P2nbr.p, pp.nbr.data(), pp.nbr.size() * sizeof(int32_t), hipMemcpyHostToDevice));
      c.p2_nb = pp.nb;
      c.p2_slots = pp.slots;
    }

    // compressed 3D operator (face-kernel variant 8), kept beside the blocks
    for (DevBuf<double>* b : {&c.d_cmpC64, &c.d_cmpA, &c.d_cmpB, &c.d_cmpF, &c.d_cmpG}) b->free();
    c.d_cmpC32.free();
    c.cmp_bytes_f64 = c.cmp_bytes_f32 = 0;
    if (hs.dim == 3 && hs.p <= 2) {
      CompressedOp co;
      build_compressed(hs, c.elem.data(), co);
      auto up = [](DevBuf<double>& b, const std::vector<double>& v) {
        b.alloc(v.size());
        SDG_HIP(hipMemcpy(b.p, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
      };
      if (precisions & SDG_PREC_F64) up(c.d_cmpC64, co.C);
      if (precisions & SDG_PREC_F32) {
        std::vector<float> f(co.C.begin(), co.C.end());
        c.d_cmpC32.alloc(f.size());
        SDG_HIP(hipMemcpy(c.d_cmpC32.p, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
      }
      up(c.d_cmpA, co.fa);
      up(c.d_cmpB, co.eB);
      up(c.d_cmpF, co.F);
      up(c.d_cmpG, co.G);
      // bytes per apply: C of the sides that exist, the face-term coefficients
      // and the element factors
      const int64_t nside = 2 * hs.n_face - hs.n_bface;
      c.cmp_bytes_f64 = nside * (int64_t)co.npsi * co.npsi * 8 + nside * 3 * 8 + hs.n_elem * 9 * 8;
      c.cmp_bytes_f32 = nside * (int64_t)co.npsi * co.npsi * 4 + nside * 3 * 8 + hs.n_elem * 9 * 8;
    }

    // operator blocks
    c.d_faces.alloc(hs.n_face);
    SDG_HIP(hipMemcpy(c.d_faces.p, hs.faces.data(), hs.n_face * sizeof(FaceRec), hipMemcpyHostToDevice));
    if (precisions & SDG_PREC_F64) {
      c.d_Dt64.alloc(hs.Dt.size());
      SDG_HIP(hipMemcpy(c.d_Dt64.p, hs.Dt.data(), hs.Dt.size() * sizeof(double), hipMemcpyHostToDevice));
    } else {
      c.d_Dt64.free();
    }
    if (precisions & SDG_PREC_F32) {
      std::vector<float> f(hs.Dt.begin(), hs.Dt.end());
      c.d_Dt32.alloc(f.size());
      SDG_HIP(hipMemcpy(c.d_Dt32.p, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
    } else {
      c.d_Dt32.free();
    }
    c.d_face_lm.alloc(hs.face_lm.size());
    SDG_HIP(hipMemcpy(c.d_face_lm.p, hs.face_lm.data(), hs.face_lm.size() * sizeof(double), hipMemcpyHostToDevice));
    c.d_face_E.free();
    c.d_face_Cw.free();
    if (c.aniso) {
      c.d_face_E.alloc(hs.face_E.size());
      SDG_HIP(hipMemcpy(c.d_face_E.p, hs.face_E.data(), hs.face_E.size() * sizeof(double), hipMemcpyHostToDevice));
      c.d_face_Cw.alloc(hs.face_Cw.size());
      SDG_HIP(hipMemcpy(c.d_face_Cw.p, hs.face_Cw.data(), hs.face_Cw.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    c.d_elem_w.alloc(hs.elem_w.size());
    SDG_HIP(hipMemcpy(c.d_elem_w.p, hs.elem_w.data(), hs.elem_w.size() * sizeof(double), hipMemcpyHostToDevice));
    c.d_Mref.alloc(hs.Mref.size());
    SDG_HIP(hipMemcpy(c.d_Mref.p, hs.Mref.data(), hs.Mref.size() * sizeof(double), hipMemcpyHostToDevice));
    {
      std::vector<double> tw(ng, 1.0);
      if (c.scheme != SDG_SCHEME_CN) tw = hs.w;
      c.d_tw.alloc(ng);
      SDG_HIP(hipMemcpy(c.d_tw.p, tw.data(), ng * sizeof(double), hipMemcpyHostToDevice));
      c.d_e1.alloc(ng);
      SDG_HIP(hipMemcpy(c.d_e1.p, hs.e1.data(), ng * sizeof(double), hipMemcpyHostToDevice));
      std::vector<double> e0(ng, 1.0);
      if (c.scheme != SDG_SCHEME_CN) e0 = hs.e0;
      c.d_e0.alloc(ng);
      SDG_HIP(hipMemcpy(c.d_e0.p, e0.data(), ng * sizeof(double), hipMemcpyHostToDevice));
    }
    // adjoint: element -> face table with the volume fraction of the element
    // in the dual cell of each of its faces
    {
      const int nfe = d + 1;
      std::vector<double> wt((size_t)hs.n_elem * nfe, 0.0);
      for (int64_t e = 0; e < hs.n_elem; ++e)
        for (int f = 0; f < nfe; ++f) {
          const int64_t j = hs.elem_face[e * nfe + f];
          require(j >= 0 && j < hs.n_face, SDG_EMESH, "element face without a face record");
          const FaceRec& fr = hs.faces[j];
          if (fr.left == e && fr.lf == f) wt[e * nfe + f] = hs.face_wt[2 * j];
          else if (fr.right == e && fr.rf == f) wt[e * nfe + f] = hs.face_wt[2 * j + 1];
          else throw Error(SDG_EMESH, "element-face table is inconsistent");
        }
      c.d_ef_wt.alloc(wt.size());
      SDG_HIP(hipMemcpy(c.d_ef_wt.p, wt.data(), wt.size() * sizeof(double), hipMemcpyHostToDevice));
      c.d_elem_face.alloc(hs.elem_face.size());
      SDG_HIP(hipMemcpy(c.d_elem_face.p, hs.elem_face.data(), hs.elem_face.size() * sizeof(int32_t),
                        hipMemcpyHostToDevice));
      c.d_detJ.alloc(hs.n_elem);
      SDG_HIP(hipMemcpy(c.d_detJ.p, hs.elem_detJ.data(), hs.n_elem * sizeof(double), hipMemcpyHostToDevice));
      c.d_lam_s.alloc((size_t)hs.n_face * ng * hs.nsig * hs.npsi);
      c.d_face_grad.alloc((size_t)hs.n_face * 2);
    }

    // workspaces (every solver vector holds max_rhs columns)
    const size_t R = (size_t)max_rhs;
    c.z_col = hs.n_elem * (d + 1) * ng * d * nphi;
    c.d_z.alloc((size_t)c.z_col * R);
    const size_t n = c.n_slab * R;
    const bool multi = max_rhs > 1 || c.n_mesh > 1;
    // Crank-Nicolson single systems run CG, unless the patch preconditioner
    // (not symmetric) asks for GMRES
    const bool cg_only = c.scheme == SDG_SCHEME_CN && !multi && !(precisions & SDG_ASSEMBLE_PATCH_PRECOND);
    c.d_V.alloc(cg_only ? n : (size_t)(kMaxRestart + 1) * n);
    c.d_x.alloc(n);
    c.d_b.alloc(n);
    c.d_r.alloc(n);
    c.d_w.alloc(n);
    c.d_t.alloc(n);
    c.d_d.alloc(n);
    c.d_e.alloc(n);
    c.d_partials.alloc((size_t)kRedBlocks * kRedSlots);
    c.d_sc.alloc(1);
    SDG_HIP(hipMemset(c.d_sc.p, 0, sizeof(DevScalars)));
    if (!c.h_pinned) SDG_HIP(hipHostMalloc((void**)&c.h_pinned, 16 * sizeof(double), hipHostMallocDefault));
    if (!c.h_poll) {
      SDG_HIP(hipHostMalloc((void**)&c.h_poll, (kMaxRestart + 1) * sizeof(double),
                            hipHostMallocCoherent | hipHostMallocMapped));
      for (int i = 0; i <= kMaxRestart; ++i) c.h_poll[i] = 0.0;
      SDG_HIP(hipHostGetDevicePointer((void**)&c.d_poll, c.h_poll, 0));
    }
    c.d_tmp_state.alloc(c.n_state * R);
    c.d_prev.alloc(n);
    c.prev_valid = false;
    c.prev_count = 0;
    c.d_tmp_sig.alloc(c.n_sig_state * R);
    c.d_src_amp.alloc((size_t)std::max<int64_t>(c.n_src, 1) * ng);
    SDG_HIP(hipDeviceSynchronize());
    c.assembled = true;
    const char* forced = std::getenv("SDG_OP_VARIANT");
    if (forced) {
      c.variant64 = c.variant32 = std::max(0, std::min(kNumVariants - 1, std::atoi(forced)));
    } else {
      autotune(c);
    }
  });
}

int sdg_set_operator_variant(sdg_ctx* ctx, int variant) {
  return guard([&] {
    Ctx& c = ctx_of(ctx);
    require(c.assembled, SDG_ESTATE, "assemble first");
    require(variant >= -1 && variant < kNumVariants, SDG_EINVAL, "variant must be -1 (autotune) or 0..8");
    require(variant != 8 || compressed_available(c, SDG_PREC_F64) || compressed_available(c, SDG_PREC_F32),
            SDG_EUNSUPPORTED, "variant 8 needs the compressed operator (3D, p <= 2)");
    require(!c.aniso || variant < 0 || aniso_variant(variant), SDG_EUNSUPPORTED,
            "with an anisotropic material only face-kernel variants 3, 4 and 8 apply");
    SDG_HIP(hipSetDevice(c.device));
    c.graphs.clear();
    if (variant < 0) autotune(c);
    else c.variant64 = c.variant32 = variant;
  });
}

int sdg_set_batched_variant(sdg_ctx* ctx, int bvariant) {
  return guard([&] {
    Ctx& c = ctx_of(ctx);
    require(c.assembled, SDG_ESTATE, "assemble first");
    require(bvariant >= 0 && bvariant <= 2, SDG_EINVAL, "batched variant must be 0, 1 or 2");
    require(!c.aniso || bvariant == 0, SDG_EUNSUPPORTED,
            "with an anisotropic material batched applies use the column grid (batched variant 0)");
    c.graphs.clear();
    c.bvariant = c.bvariant32 = bvariant;
  });
}

int sdg_query(const sdg_ctx* ctx, sdg_sizes* out) {
  return guard([&] {
    require(ctx && out, SDG_EINVAL, "null argument");
    const Ctx& c = *reinterpret_cast<const Ctx*>(ctx);
    require(c.assembled, SDG_ESTATE, "assemble first");
    const HostSetup& hs = c.hs;
    std::memset(out, 0, sizeof(*out));
    out->dim = hs.dim;
    out->p = hs.p;
    out->p_gamma = hs.pg;
    out->scheme = hs.scheme;
    out->n_phi = hs.nphi;
    out->n_psi = hs.npsi;
    out->n_gamma = hs.ng;
    out->n_sigma = hs.nsig;
    out->n_elem = hs.n_elem;
    out->n_face = hs.n_face;
    out->n_face_boundary = hs.n_bface;
    out->n_vel_slab = c.n_slab;
    out->n_vel_state = c.n_state;
    out->n_stress_state = c.n_sig_state;
    out->n_stress_slab = c.n_sig_state * hs.ng;
    out->dt = hs.dt;
    for (int a = 0; a < hs.ng; ++a) out->tau[a] = hs.scheme == SDG_SCHEME_CN ? 0.5 : hs.tau[a];
    // bytes actually read per apply: boundary faces carry one block
    const int64_t blk = (int64_t)hs.nphi * hs.dim * hs.npsi;
    const int64_t nblk = 2 * hs.n_face - hs.n_bface;
    out->op_bytes_f64 = nblk * blk * 8;
    out->op_bytes_f32 = nblk * blk * 4;
    out->cmp_bytes_f64 = c.cmp_bytes_f64;
    out->cmp_bytes_f32 = c.cmp_bytes_f32;
    out->max_rhs = c.max_rhs;
    out->op_variant = c.variant64;
    out->op_variant_f32 = c.variant32;
    out->op_bvariant = c.bvariant;
    for (int v = 0; v < 3; ++v) out->tune_us_batched[v] = c.tune_b_us[v];
    out->op_bvariant_f32 = c.bvariant32;
    out->reserved0 = 0;
    for (int v = 0; v < 3; ++v) out->tune_us_batched_f32[v] = c.tune_b32_us[v];
    for (int w = 0; w < 2; ++w) out->proj_min_degree[w] = c.assembled ? projection_min_degree(c.hs, w) : 0;
    for (int v = 0; v < kNumVariants; ++v) { out->tune_us_f64[v] = c.tune_us[0][v]; out->tune_us_f32[v] = c.tune_us[1][v]; }
  });
}

int sdg_face_table(const sdg_ctx* ctx, int64_t* left, int32_t* left_face, int64_t* right, int32_t* right_face) {
  return guard([&] {
    require(ctx != nullptr, SDG_EINVAL, "null context");
    const Ctx& c = *reinterpret_cast<const Ctx*>(ctx);
    require(c.assembled, SDG_ESTATE, "assemble first");
    for (int64_t j = 0; j < c.hs.n_face; ++j) {
      const FaceRec& r = c.hs.faces[j];
      if (left) left[j] = r.left;
      if (left_face) left_face[j] = r.lf;
      if (right) right[j] = r.right;
      if (right_face) right_face[j] = r.rf;
    }
  });
}

static int apply_common(sdg_ctx* ctx, const double* v, double* y, int n_rhs, int precision, void* stream,
                        bool transpose) {
  return guard([&] {
    Ctx& c = ctx_of(ctx);
    require(c.assembled, SDG_ESTATE, "assemble first");
    require(v && y, SDG_EINVAL, "null vector");
    require(v != y, SDG_EINVAL, "v and y must not alias");
    require(n_rhs >= 1 && n_rhs <= c.max_rhs, SDG_EINVAL, "n_rhs must be in [1, max_rhs of sdg_assemble]");
    check_prec(c, precision);
    SDG_HIP(hipSetDevice(c.device));
    apply_op(c, v, y, precision, transpose, (hipStream_t)stream, n_rhs);
  });
}

int sdg_apply_velocity_operator(sdg_ctx* ctx, const double* v, double* y, int n_rhs, int precision, void* stream) {
  return apply_common(ctx, v, y, n_rhs, precision, stream, false);
}

int sdg_apply_adjoint(sdg_ctx* ctx, const double* w, double* y, int n_rhs, int precision, void* stream) {
  return apply_common(ctx, w, y, n_rhs, precision, stream, true);
}

int sdg_apply_preconditioner(sdg_ctx* ctx, int kind, const double* x, double* y, int n_rhs, void* stream) {
  return guard([&] {
    Ctx& c = ctx_of(ctx);
    require(c.assembled, SDG_ESTATE, "assemble first");
    require(x && y, SDG_EINVAL, "null vector");
    require(x != y, SDG_EINVAL, "x and y must not alias");
    require(n_rhs >= 1 && n_rhs <= c.max_rhs, SDG_EINVAL, "n_rhs must be in [1, max_rhs of sdg_assemble]");
    require(kind >= SDG_PRECOND_NONE && kind <= SDG_PRECOND_PATCH, SDG_EINVAL, "unknown preconditioner");
    SDG_HIP(hipSetDevice(c.device));
    apply_precond(c, kind, x, y, false, (hipStream_t)stream, n_rhs);
    SDG_HIP(hipGetLastError());
  });
}

int sdg_apply_velocity_operator_noalloc(sdg_ctx* ctx, const double* v, double* y, int n_rhs, int precision,
                                        void* stream) {
  return guard([&] {
    Ctx& c = ctx_of(ctx);
    require(c.assembled, SDG_ESTATE, "assemble first");
    require(v && y, SDG_EINVAL, "null vector");
    require(v != y, SDG_EINVAL, "v and y must not alias");
    require(n_rhs >= 1 && n_rhs <= c.max_rhs, SDG_EINVAL, "n_rhs must be in [1, max_rhs of sdg_assemble]");
    check_prec(c, precision);
    // the face slots of every column; FP32 applies write FP32 slots, but the
    // limit is stated for FP64 slots so that it does not depend on precision
    const size_t need = (size_t)c.z_col * (size_t)n_rhs * sizeof(double);
    require(need <= noalloc_scratch_bytes(), SDG_EINVAL,
            "face-slot workspace of " + std::to_string(need) + " bytes exceeds the " +
                std::to_string(noalloc_scratch_bytes()) + "-byte scratch array of the allocation-free apply");
    SDG_HIP(hipSetDevice(c.device));
    apply_op(c, v, y, precision, false, (hipStream_t)stream, n_rhs, noalloc_scratch(c.device));
  });
}

static int set_sources_impl(sdg_ctx* ctx, int64_t n_src, const double* pos, const double* dir, const int32_t* mesh) {
  return guard([&] {
    Ctx& c = ctx_of(ctx);
    require(c.assembled, SDG_ESTATE, "assemble first");
    require(n_src >= 0, SDG_EINVAL, "negative source count");
    require(n_src == 0 || (pos && dir), SDG_EINVAL, "null source arrays");
    const HostSetup& hs = c.hs;
    std::vector<int64_t> el(n_src);
    std::vector<double> phi((size_t)n_src * hs.nphi), dr((size_t)n_src * hs.dim);
    for (int64_t s = 0; s < n_src; ++s) {
      int64_t e0 = 0, e1 = -1;
      if (mesh) {
        require(mesh[s] >= 0 && mesh[s] < c.n_mesh, SDG_EINVAL, "source mesh index out of range");
        e0 = c.mesh_elem_off[mesh[s]];
        e1 = c.mesh_elem_off[mesh[s] + 1];
      }
      int64_t e = locate_point(hs, pos + s * hs.dim, e0, e1);
      require(e >= 0, SDG_EINVAL, "source " + std::to_string(s) + " lies outside the mesh");
      eval_velocity_basis(hs, e, pos + s * hs.dim, &phi[s * hs.nphi], 1e-12);
      el[s] = e;
      for (int k = 0; k < hs.dim; ++k) dr[s * hs.dim + k] = dir[s * hs.dim + k];
    }
    SDG_HIP(hipSetDevice(c.device));
    c.graphs.clear();
    c.n_src = n_src;
    c.p_src = c.p;
    c.src_elem = el;
    c.src_phi = phi;
    c.src_dir = dr;
    c.d_src_elem.alloc(std::max<int64_t>(n_src, 1));
    c.d_src_phi.alloc(std::max<size_t>(phi.size(), 1));
    c.d_src_dir.alloc(std::max<size_t>(dr.size(), 1));
    c.d_src_amp.alloc((size_t)std::max<int64_t>(n_src, 1) * hs.ng);
    if (n_src) {
      SDG_HIP(hipMemcpy(c.d_src_elem.p, el.data(), el.size() * sizeof(int64_t), hipMemcpyHostToDevice));
      SDG_HIP(hipMemcpy(c.d_src_phi.p, phi.data(), phi.size() * sizeof(double), hipMemcpyHostToDevice));
      SDG_HIP(hipMemcpy(c.d_src_dir.p, dr.data(), dr.size() * sizeof(double), hipMemcpyHostToDevice));
    }
  });
}

int sdg_set_sources(sdg_ctx* ctx, int64_t n_src, const double* pos, const double* dir) {
  return set_sources_impl(ctx, n_src, pos, dir, nullptr);
}

int sdg_set_mesh_sources(sdg_ctx* ctx, int64_t n_src, const double* pos, const double* dir, const int32_t* mesh) {
  if (!mesh && n_src > 0) return guard([] { throw Error(SDG_EINVAL, "null mesh index array"); });
  return set_sources_impl(ctx, n_src, pos, dir, mesh);
}

int sdg_solve_step(sdg_ctx* ctx, double* v_state, double* sigma_state, const double* amp, int n_rhs,
                   const sdg_solve_opts* opts, sdg_solve_info* info, double* v_slab, double* sigma_slab,
                   void* stream) {
  SolveResult res;
  int rc = guard([&] {
    Ctx& c = ctx_of(ctx);
    require(c.assembled, SDG_ESTATE, "assemble first");
    require(v_state && sigma_state && opts, SDG_EINVAL, "null argument");
    require(n_rhs >= 1 && n_rhs <= c.max_rhs, SDG_EINVAL, "n_rhs must be in [1, max_rhs of sdg_assemble]");
    require(opts->rtol > 0 && opts->max_iter > 0, SDG_EINVAL, "rtol and max_iter must be positive");
    require((opts->flags & ~(SDG_SOLVE_GRAPH | SDG_SOLVE_EXTRAPOLATE | SDG_SOLVE_CGS2 | SDG_SOLVE_DEVICE_STOP)) == 0,
            SDG_EINVAL,
            "unknown solve flags");
    const int prec = opts->precision == 0 ? SDG_PREC_F64 : opts->precision;
    check_prec(c, SDG_PREC_F64);
    if (prec == SDG_PREC_F32) check_prec(c, SDG_PREC_F32);
    const int R = n_rhs;
    const bool graph = (opts->flags & SDG_SOLVE_GRAPH) != 0;
    const bool multi = R > 1 || c.n_mesh > 1 || graph;
    int solver = opts->solver;
    if (solver == SDG_SOLVER_AUTO) solver = c.scheme == SDG_SCHEME_CN && !multi ? SDG_SOLVER_CG : SDG_SOLVER_GMRES;
    require(solver == SDG_SOLVER_CG || solver == SDG_SOLVER_GMRES, SDG_EINVAL, "unknown solver");
    require(!multi || solver == SDG_SOLVER_GMRES, SDG_EUNSUPPORTED,
            "batched, mesh-batch and graph solves use GMRES (SDG_SOLVER_GMRES or AUTO)");
    require(solver != SDG_SOLVER_CG || opts->precond != SDG_PRECOND_PATCH, SDG_EUNSUPPORTED,
            "the patch preconditioner is not symmetric: use GMRES with it");
    require(solver != SDG_SOLVER_GMRES || c.d_V.n >= (size_t)(kMaxRestart + 1) * c.n_slab * R, SDG_EINVAL,
            "GMRES workspace is only allocated for the space-time scheme, batched solves or the patch preconditioner");
    const int restart = opts->restart > 0 ? opts->restart : 30;
    require(restart <= kMaxRestart, SDG_EINVAL, "restart must be <= 32");
    require(opts->precond >= SDG_PRECOND_NONE && opts->precond <= SDG_PRECOND_PATCH, SDG_EINVAL,
            "unknown preconditioner");
    SDG_HIP(hipSetDevice(c.device));
    hipStream_t s = (hipStream_t)stream;
    const int64_t N = c.n_slab * R;
    KrylovCfg kc;
    kc.check_every = opts->check_every > 0 ? opts->check_every : 5;
    kc.restart = restart;
    kc.precond = opts->precond;
    kc.rtol = opts->rtol;
    kc.max_iter = opts->max_iter;
    kc.delayed = (opts->flags & SDG_SOLVE_CGS2) == 0;
    kc.device_stop = (opts->flags & SDG_SOLVE_DEVICE_STOP) != 0;
    // extrapolated initial guess: the previous slab continued in time; without
    // a previous slab of this width, seed it with the old state at every node
    // (the continuation of a constant is the constant)
    const bool extrap = (opts->flags & SDG_SOLVE_EXTRAPOLATE) != 0;
    if (extrap && (!c.prev_valid || c.prev_R != R)) {
      launch_broadcast_time(c.hs.n_elem * R, c.hs.ng, c.hs.dim * c.hs.nphi, v_state, c.d_prev.p, s);
      c.prev_count = 1;
    }
    c.prev_valid = extrap;
    c.prev_R = R;
    // one-node slabs outside graph mode keep the trajectory's last slabs and
    // extrapolate them (a recorded graph would keep the history length it
    // was recorded with)
    const bool hist = extrap && c.hs.ng == 1 && !graph;
    if (!hist) c.prev_count = extrap ? 1 : 0;
    if (hist && (c.d_prev2.n != c.d_prev.n || c.d_prev3.n != c.d_prev.n)) {
      c.d_prev2.alloc(c.d_prev.n);
      c.d_prev3.alloc(c.d_prev.n);
      c.prev_count = 1;
    }
    const int hist_order = hist ? std::min(c.prev_count, 3) : 0;

    if (graph) {
      MultiSys& m = systems(c, R);
      StepGraphs& G = c.graphs;
      if (!G.stream) SDG_HIP(hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking));
      hipStream_t gs = G.stream;
      // FP64: GMRES on A x = b.  FP32: the FP32 operator inside FP64
      // iterative refinement, every decision on the device: inner GMRES on
      // A32 e = d from e = 0, then x += e, d = b - A64 x and the per-system
      // outer test, which also sets the next inner targets.
      const bool ir = prec == SDG_PREC_F32;
      const double inner_tol = opts->inner_rtol > 0 ? opts->inner_rtol : 1e-4;
      const int max_ref = opts->max_refine > 0 ? opts->max_refine : 10;
      const int* act = m.active_flags();
      MultiOp op = [&c, R, gs, prec, act](const double* in, double* out, bool masked) {
        apply_op(c, in, out, prec, false, gs, R, nullptr, masked ? act : nullptr);
      };
      std::function<void(const double*, double*)> pre = [&c, R, gs, kc](const double* in, double* out) {
        apply_precond(c, kc.precond, in, out, false, gs, R);
      };
      const std::function<void(const double*, double*)>* pp = kc.precond != SDG_PRECOND_NONE ? &pre : nullptr;
      double* const kb = ir ? c.d_d.p : c.d_b.p;  // the Krylov system's right-hand side and unknown
      double* const kx = ir ? c.d_e.p : c.d_x.p;
      auto outer_residual = [&]() {  // d = b - A64 x, the outer test and the inner targets
        apply_op(c, c.d_x.p, c.d_t.p, SDG_PREC_F64, false, gs, R);
        vec_copy(N, c.d_b.p, c.d_d.p, gs);
        vec_axpby(N, -1.0, c.d_t.p, 1.0, c.d_d.p, gs);
        multi_refine_check(m, c.d_d.p, kc.rtol, inner_tol, gs);
        vec_fill(N, 0.0, c.d_e.p, gs);
      };
      const bool src = amp && c.n_src > 0;
      const bool same = G.head && G.v == v_state && G.sig == sigma_state && G.vslab == v_slab &&
                        G.sslab == sigma_slab && G.R == R && G.precond == kc.precond && G.restart == restart &&
                        G.rtol == kc.rtol && G.src == src && G.flags == opts->flags && G.prec == prec &&
                        (!ir || G.inner_rtol == inner_tol) && G.check_every == kc.check_every;
      if (!same) {
        G.clear();
        auto record = [&](auto&& body) {
          SDG_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeRelaxed));
          hipGraph_t g = nullptr;
          try {
            body();
          } catch (...) {
            (void)hipStreamEndCapture(gs, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
          }
          SDG_HIP(hipStreamEndCapture(gs, &g));
          hipGraphExec_t e = nullptr;
          const hipError_t err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
          (void)hipGraphDestroy(g);
          SDG_HIP(err);
          return e;
        };
        int mv = 0;
        bool done = false;
        G.head = record([&] {
          step_rhs(c, v_state, sigma_state, R, src, gs, extrap);
          if (ir) {
            multi_outer_setup(m, c.d_b.p, gs);
            outer_residual();
          } else {
            multi_setup(m, c.d_b.p, c.d_x.p, kc.rtol, gs);
          }
          if (!kc.delayed)
            multi_cycle(m, kb, kx, kc, gs, op, pp, c.d_V.p, c.d_r.p, c.d_w.p, c.d_t.p, false, restart, &mv, &done);
        });
        if (kc.delayed) {
          // the cycle in parts of check_every steps, polled between parts as
          // the eager solver polls, and the early end after each part
          const int ce = std::max(1, std::min(kc.check_every, restart));
          for (int j0 = 0; j0 < restart; j0 += ce) {
            const int j1 = std::min(j0 + ce, restart);
            G.part.push_back(record([&] {
              multi_cycle_part(m, kb, kx, kc, gs, op, pp, c.d_V.p, c.d_w.p, c.d_t.p, restart, j0, j1, &mv);
            }));
            G.part_end.push_back(j1);
            if (j1 < restart)
              G.stop.push_back(record([&] { multi_cycle_stop(m, kx, kc, gs, pp, c.d_V.p, c.d_w.p, c.d_t.p, j1); }));
          }
        } else {
          G.cycle = record([&] {
            multi_cycle(m, kb, kx, kc, gs, op, pp, c.d_V.p, c.d_r.p, c.d_w.p, c.d_t.p, false, restart, &mv, &done);
          });
        }
        G.verify = record([&] { multi_residual(m, kb, kx, gs, op, c.d_r.p); });
        if (ir) {
          G.refine = record([&] {
            vec_axpby(N, 1.0, c.d_e.p, 1.0, c.d_x.p, gs);
            outer_residual();
          });
        }
        G.tail = record([&] { step_backsub(c, v_state, sigma_state, v_slab, sigma_slab, R, gs, extrap); });
        G.v = v_state;
        G.sig = sigma_state;
        G.vslab = v_slab;
        G.sslab = sigma_slab;
        G.R = R;
        G.precond = kc.precond;
        G.restart = restart;
        G.rtol = kc.rtol;
        G.src = src;
        G.flags = opts->flags;
        G.prec = prec;
        G.inner_rtol = inner_tol;
        G.check_every = kc.check_every;
      }
      SDG_HIP(hipStreamSynchronize(s));
      if (src)
        SDG_HIP(hipMemcpyAsync(c.d_src_amp.p, amp, c.n_src * c.hs.ng * sizeof(double), hipMemcpyHostToDevice, gs));
      SDG_HIP(hipGraphLaunch(G.head, gs));
      res.iters = kc.delayed ? 0 : restart;
      res.matvecs = (kc.delayed ? 0 : restart + 1) + (ir ? 1 : 0);
      // one restart cycle: whole, or in parts with a poll after each
      auto run_cycle = [&]() {
        if (!kc.delayed) {
          SDG_HIP(hipGraphLaunch(G.cycle, gs));
          res.iters += restart;
          res.matvecs += restart + 1;
          return;
        }
        int j0 = 0;
        for (size_t p = 0; p < G.part.size(); ++p) {
          SDG_HIP(hipGraphLaunch(G.part[p], gs));
          res.iters += G.part_end[p] - j0;
          res.matvecs += G.part_end[p] - j0 + (p == 0 ? 1 : 0);
          j0 = G.part_end[p];
          if (p + 1 < G.part.size() && multi_nactive(m, gs) == 0) {
            SDG_HIP(hipGraphLaunch(G.stop[p], gs));
            return;
          }
        }
      };
      if (kc.delayed) run_cycle();
      for (;;) {
        if (multi_nactive(m, gs) == 0) {
          SDG_HIP(hipGraphLaunch(G.verify, gs));
          ++res.matvecs;
          if (multi_nactive(m, gs) == 0) {
            if (!ir) {
              res.converged = true;
              break;
            }
            // inner solve done: apply the correction and test the outer system
            SDG_HIP(hipGraphLaunch(G.refine, gs));
            ++res.matvecs;
            ++res.refinements;
            if (multi_nouter(m, gs) == 0) {
              res.converged = true;
              break;
            }
            if (res.refinements >= max_ref) break;
          }
        }
        if (res.iters >= kc.max_iter) break;
        run_cycle();
      }
      SDG_HIP(hipGraphLaunch(G.tail, gs));
      if (ir) multi_outer_result(m, gs, res);
      else multi_result(m, gs, res);
      SDG_HIP(hipStreamSynchronize(gs));
      if (!res.converged) throw Error(SDG_ENOCONV, "Krylov solver did not reach rtol within max_iter");
      return;
    }

    // 1. right-hand side (one launch for all columns)
    const bool src = amp && c.n_src > 0;
    if (src) SDG_HIP(hipMemcpyAsync(c.d_src_amp.p, amp, c.n_src * c.hs.ng * sizeof(double), hipMemcpyHostToDevice, s));
    step_rhs(c, v_state, sigma_state, R, src, s, extrap, hist_order);

    // 2. Krylov solve from the old state copied to every time node
    auto inner = [&](const double* b, double* x, double tol, int maxit, int pr, bool x_zero) {
      KrylovCfg k2 = kc;
      k2.rtol = tol;
      k2.max_iter = maxit;
      k2.prec = pr;
      k2.x_zero = x_zero && !multi;
      // FP32 inner solves of several systems take the targets the outer test set
      k2.keep_targets = multi && pr == SDG_PREC_F32;
      // the refinement loop computes the FP64 residual after every inner solve
      k2.recurrence_only = pr == SDG_PREC_F32;
      if (!multi) return solver == SDG_SOLVER_CG ? solve_cg(c, b, x, k2, s) : solve_gmres(c, b, x, k2, s);
      MultiSys& m = systems(c, R);
      const int* act = m.active_flags();
      MultiOp op = [&](const double* in, double* out, bool masked) {
        apply_op(c, in, out, pr, false, s, R, nullptr, masked ? act : nullptr);
      };
      std::function<void(const double*, double*)> pre = [&](const double* in, double* out) {
        apply_precond(c, k2.precond, in, out, false, s, R);
      };
      return solve_gmres_multi(m, b, x, k2, s, op, k2.precond != SDG_PRECOND_NONE ? &pre : nullptr, c.d_V.p,
                               c.d_r.p, c.d_w.p, c.d_t.p);
    };
    if (prec == SDG_PREC_F64) {
      res = inner(c.d_b.p, c.d_x.p, opts->rtol, opts->max_iter, SDG_PREC_F64, false);
    } else {
      // FP32 operator inside FP64 iterative refinement
      const double inner_tol = opts->inner_rtol > 0 ? opts->inner_rtol : 1e-4;
      const int max_ref = opts->max_refine > 0 ? opts->max_refine : 10;
      // several systems: each system's outer test on the device; a system at
      // rtol takes no further inner step (its inner target is +inf)
      if (multi) multi_outer_setup(systems(c, R), c.d_b.p, s);
      auto rel_residual = [&](double* bnorm_out) {
        // d = b - A64 x and the worst relative residual over the systems
        apply_op(c, c.d_x.p, c.d_t.p, SDG_PREC_F64, false, s, R);
        ++res.matvecs;
        vec_copy(N, c.d_b.p, c.d_d.p, s);
        vec_axpby(N, -1.0, c.d_t.p, 1.0, c.d_d.p, s);
        if (!multi) {
          const double bn = std::sqrt(vec_dot_host(c, N, c.d_b.p, c.d_b.p, s));
          const double rn = std::sqrt(vec_dot_host(c, N, c.d_d.p, c.d_d.p, s));
          *bnorm_out = bn;
          return bn > 0 ? rn / bn : rn;
        }
        MultiSys& m = systems(c, R);
        multi_refine_check(m, c.d_d.p, opts->rtol, inner_tol, s);
        SolveResult o;
        multi_outer_result(m, s, o);
        *bnorm_out = o.bnorm;
        return o.rel_res;
      };
      for (int k = 0; k <= max_ref; ++k) {
        double bnorm = 0.0;
        const double rr = rel_residual(&bnorm);
        require(std::isfinite(rr), SDG_ENONFINITE, "non-finite residual");
        res.rel_res = rr;
        res.bnorm = bnorm;
        if (rr <= opts->rtol || k == max_ref || res.iters >= opts->max_iter) {
          res.converged = rr <= opts->rtol;
          break;
        }
        // correction: A32 e = d from a zero initial guess, then x += e.  One
        // system: an inner solve needs to reduce d only by what is left to
        // rtol (with a factor 2 to spare), never more tightly than inner_tol
        // asks; the device sets several systems' targets
        const double tol_k = multi ? inner_tol : std::max(inner_tol, 0.5 * opts->rtol / rr);
        vec_fill(N, 0.0, c.d_e.p, s);
        SolveResult in = inner(c.d_d.p, c.d_e.p, tol_k, opts->max_iter - res.iters, SDG_PREC_F32, true);
        res.iters += in.iters;
        res.matvecs += in.matvecs;
        ++res.refinements;
        vec_axpby(N, 1.0, c.d_e.p, 1.0, c.d_x.p, s);
      }
    }

    // 3. stress back-substitution and 4. end-of-slab state
    step_backsub(c, v_state, sigma_state, v_slab, sigma_slab, R, s, extrap, hist);
    if (hist) c.prev_count = std::min(c.prev_count + 1, 3);
    SDG_HIP(hipStreamSynchronize(s));
    if (!res.converged) throw Error(SDG_ENOCONV, "Krylov solver did not reach rtol within max_iter");
  });
  if (info) {
    info->iterations = res.iters;
    info->matvecs = res.matvecs;
    info->refinements = res.refinements;
    info->converged = res.converged ? 1 : 0;
    info->rel_residual = res.rel_res;
    info->b_norm = res.bnorm;
  }
  return rc;
}

int sdg_adjoint_step(sdg_ctx* ctx, const double* v_old, const double* v_slab, double* vbar, double* sigma_bar,
                     double* grad, const sdg_solve_opts* opts, sdg_solve_info* info, void* stream) {
  SolveResult res;
  int rc = guard([&] {
    Ctx& c = ctx_of(ctx);
    require(c.assembled, SDG_ESTATE, "assemble first");
    require(v_old && v_slab && vbar && sigma_bar && grad && opts, SDG_EINVAL, "null argument");
    require(opts->rtol > 0 && opts->max_iter > 0, SDG_EINVAL, "rtol and max_iter must be positive");
    require(opts->precision == 0 || opts->precision == SDG_PREC_F64, SDG_EUNSUPPORTED,
            "the adjoint step runs in FP64");
    require(!c.aniso, SDG_EUNSUPPORTED, "the adjoint step takes an isotropic material");
    require(c.hs.curved_ids.empty(), SDG_EUNSUPPORTED, "the adjoint step takes straight elements");
    check_prec(c, SDG_PREC_F64);
    int solver = opts->solver;
    if (solver == SDG_SOLVER_AUTO) solver = c.scheme == SDG_SCHEME_CN ? SDG_SOLVER_CG : SDG_SOLVER_GMRES;
    require(solver == SDG_SOLVER_CG || solver == SDG_SOLVER_GMRES, SDG_EINVAL, "unknown solver");
    require(solver != SDG_SOLVER_GMRES || c.d_V.n >= (size_t)(kMaxRestart + 1) * c.n_slab, SDG_EINVAL,
            "GMRES workspace is only allocated for the space-time scheme");
    const int restart = opts->restart > 0 ? opts->restart : 30;
    require(restart <= kMaxRestart, SDG_EINVAL, "restart must be <= 32");
    require(opts->precond >= SDG_PRECOND_NONE && opts->precond <= SDG_PRECOND_BLOCK, SDG_EINVAL,
            "unknown preconditioner");
    SDG_HIP(hipSetDevice(c.device));
    hipStream_t s = (hipStream_t)stream;
    const HostSetup& hs = c.hs;
    const int d = hs.dim, ng = hs.ng, nvs = d * hs.nphi;
    const int64_t ne = hs.n_elem;
    const double dt = hs.dt;
    const bool cn = c.scheme == SDG_SCHEME_CN;
    std::vector<double> TiT(ng * ng, 1.0);
    if (!cn) {
      std::vector<double> Ti = inverse(hs.T, ng);
      for (int a = 0; a < ng; ++a)
        for (int b = 0; b < ng; ++b) TiT[a * ng + b] = Ti[b * ng + a];
    }
    auto tite1 = [&](int a) {
      double q = 0.0;
      for (int b = 0; b < ng; ++b) q += TiT[a * ng + b] * hs.e1[b];
      return q;
    };

    // 1. right-hand side of the transposed velocity system:
    //    space-time  b_a = e1_a vbar - dt w_a (T^-T e1)_a D E^T sbar
    //    Crank-Nicolson  b = vbar - dt/2 D E^T sbar
    {
      OpArgs f = base_args(c, SDG_PREC_F64);
      f.sig_in = sigma_bar;
      f.sig_in_Et = 1;
      f.z = c.d_z.p;
      f.use_g = 0;
      f.c.Cs[0] = 1.0;
      launch_face(d, hs.p, 1, SDG_PREC_F64, kScatter, f, s);
      OpArgs e = base_args(c, SDG_PREC_F64);
      e.v = vbar;
      e.v_spatial = 1;
      e.mass_identity = 1;
      e.z = c.d_z.p;
      e.y = c.d_b.p;
      if (cn) {
        e.c.Tm[0] = 1.0;
        e.c.Cs[0] = -dt / 2.0;
      } else {
        for (int a = 0; a < ng; ++a) {
          e.c.Tm[a * ng] = hs.e1[a];
          e.c.Cs[a] = -dt * hs.w[a] * tite1(a);
        }
      }
      launch_elem(d, hs.p, ng, e, s);
      SDG_HIP(hipGetLastError());
    }

    // 2. Krylov solve of A^T L_v = b (zero initial guess)
    vec_fill(c.n_slab, 0.0, c.d_x.p, s);
    KrylovCfg kc;
    kc.check_every = opts->check_every > 0 ? opts->check_every : 5;
    kc.restart = restart;
    kc.precond = opts->precond;
    kc.rtol = opts->rtol;
    kc.max_iter = opts->max_iter;
    kc.prec = SDG_PREC_F64;
    kc.transpose = true;
    kc.delayed = (opts->flags & SDG_SOLVE_CGS2) == 0;
    kc.device_stop = (opts->flags & SDG_SOLVE_DEVICE_STOP) != 0;
    kc.x_zero = true;
    res = solver == SDG_SOLVER_CG ? solve_cg(c, c.d_b.p, c.d_x.p, kc, s) : solve_gmres(c, c.d_b.p, c.d_x.p, kc, s);

    // 3. stress multipliers L_s and the new stress adjoint:
    //    space-time  L_s = T^-T e1 (x) sbar + dt (T^-T W) (x) D^T L_v,  sbar' = e0^T L_s
    //    Crank-Nicolson  L_s = sbar + dt/2 D^T L_v,  sbar' = 2 L_s - sbar
    {
      OpArgs a = base_args(c, SDG_PREC_F64);
      a.v = c.d_x.p;
      a.sig_in = sigma_bar;
      a.use_g = 1;
      a.vsum = 1;
      a.s_out = c.d_lam_s.p;
      if (cn) {
        a.c.Cs[0] = 1.0;
        a.c.Cg[0] = dt / 2.0;
        a.c.send[0] = 1.0;
      } else {
        for (int aa = 0; aa < ng; ++aa) {
          a.c.Cs[aa] = tite1(aa);
          for (int b = 0; b < ng; ++b) a.c.Cg[aa * ng + b] = dt * TiT[aa * ng + b] * hs.w[b];
          a.c.send[aa] = hs.e0[aa];
        }
        a.s_end = c.d_tmp_sig.p;
      }
      launch_face(d, hs.p, ng, SDG_PREC_F64, kWriteStress, a, s);
      SDG_HIP(hipGetLastError());
    }

    // 4. material gradients
    {
      vec_fill(2 * hs.n_face, 0.0, c.d_face_grad.p, s);
      GradArgs g{};
      g.n_face = hs.n_face;
      g.n_elem = ne;
      g.faces = c.d_faces.p;
      g.Dt = c.d_Dt64.p;
      g.lam_s = c.d_lam_s.p;
      g.face_out = c.d_face_grad.p;
      RhoCoefs rcf{};
      if (cn) {
        vec_copy(c.n_slab, v_slab, c.d_t.p, s);
        vec_axpby(c.n_slab, 1.0, v_old, 1.0, c.d_t.p, s);  // v^{n+1} + v^n
        g.v = c.d_t.p;
        g.coef = -dt / 2.0;
        g.wq[0] = 1.0;
        rcf.Bq[0] = -1.0;
        rcf.Bo[0] = 1.0;
      } else {
        g.v = v_slab;
        g.coef = -dt;
        for (int b = 0; b < ng; ++b) g.wq[b] = hs.w[b];
        for (int a = 0; a < ng; ++a) {
          rcf.Bo[a] = hs.e0[a];
          for (int b = 0; b < ng; ++b) rcf.Bq[a * ng + b] = -hs.T[a * ng + b];
        }
      }
      launch_grad_face(d, hs.p, ng, g, s);
      SDG_HIP(hipGetLastError());
      launch_face_to_elem(ne, d + 1, c.d_elem_face.p, c.d_ef_wt.p, c.d_face_grad.p, grad, grad + ne, s);
      launch_grad_rho(ne, ng, d, hs.nphi, rcf, c.d_Mref.p, c.d_detJ.p, c.d_x.p, v_slab, v_old, grad + 2 * ne, s);
      SDG_HIP(hipGetLastError());
    }

    // 5. velocity adjoint at the start of the slab
    if (cn) {
      // vbar' = rho Mbar L_v - dt/2 D E^T L_s
      OpArgs f = base_args(c, SDG_PREC_F64);
      f.sig_in = c.d_lam_s.p;
      f.sig_in_Et = 1;
      f.z = c.d_z.p;
      f.use_g = 0;
      f.c.Cs[0] = -dt / 2.0;
      launch_face(d, hs.p, 1, SDG_PREC_F64, kScatter, f, s);
      OpArgs e = base_args(c, SDG_PREC_F64);
      e.v = c.d_x.p;
      e.z = c.d_z.p;
      e.y = vbar;
      e.c.Tm[0] = 1.0;
      launch_elem(d, hs.p, 1, e, s);
      vec_axpby(c.n_sig_state, 2.0, c.d_lam_s.p, -1.0, sigma_bar, s);
    } else {
      // vbar' = rho Mbar (e0^T L_v)
      launch_end_of_slab(ne, ng, nvs, c.d_e0.p, c.d_x.p, c.d_tmp_state.p, s);
      OpArgs e = base_args(c, SDG_PREC_F64);
      e.v = c.d_tmp_state.p;
      e.y = vbar;
      e.c.Tm[0] = 1.0;
      launch_elem(d, hs.p, 1, e, s);
      vec_copy(c.n_sig_state, c.d_tmp_sig.p, sigma_bar, s);
    }
    SDG_HIP(hipGetLastError());
    SDG_HIP(hipStreamSynchronize(s));
    if (!res.converged) throw Error(SDG_ENOCONV, "Krylov solver did not reach rtol within max_iter");
  });
  if (info) {
    info->iterations = res.iters;
    info->matvecs = res.matvecs;
    info->refinements = 0;
    info->converged = res.converged ? 1 : 0;
    info->rel_residual = res.rel_res;
    info->b_norm = res.bnorm;
  }
  return rc;
}

int sdg_sample_velocity_adjoint(sdg_ctx* ctx, int n_rhs, int64_t n_pts, const double* pts, const double* obs_bar,
                                double* vbar, void* stream) {
  return guard([&] {
    Ctx& c = ctx_of(ctx);
    require(c.assembled, SDG_ESTATE, "assemble first");
    require(n_rhs == 1, SDG_EUNSUPPORTED, "the sampling transpose takes one right-hand side");
    require(n_pts >= 0 && (n_pts == 0 || (vbar && pts && obs_bar)), SDG_EINVAL, "null argument");
    if (n_pts == 0) return;
    const HostSetup& hs = c.hs;
    require(hs.dim * hs.nphi <= 256, SDG_EUNSUPPORTED, "element too large for the sampling transpose kernel");
    SDG_HIP(hipSetDevice(c.device));
    hipStream_t s = (hipStream_t)stream;
    locate_points(c, n_pts, pts);
    launch_sample_adjoint(n_pts, hs.nphi, hs.dim, c.d_samp_elem.p, c.d_samp_phi.p, obs_bar, vbar, s);
    SDG_HIP(hipGetLastError());
    SDG_HIP(hipStreamSynchronize(s));
  });
}

int sdg_energy(sdg_ctx* ctx, const double* v_state, const double* sigma_state, int n_rhs, double* out, void* stream) {
  return guard([&] {
    Ctx& c = ctx_of(ctx);
    require(c.assembled, SDG_ESTATE, "assemble first");
    require(v_state && sigma_state && out, SDG_EINVAL, "null argument");
    require(n_rhs >= 1 && n_rhs <= c.max_rhs, SDG_EINVAL, "n_rhs must be in [1, max_rhs of sdg_assemble]");
    SDG_HIP(hipSetDevice(c.device));
    hipStream_t s = (hipStream_t)stream;
    if (c.n_mesh > 1) {
      // one value per mesh of the batch: its element and face ranges
      require(n_rhs == 1, SDG_EUNSUPPORTED, "batched right-hand sides on a mesh batch");
      for (int q = 0; q < c.n_mesh; ++q) {
        launch_energy(c, v_state, sigma_state, &c.d_sc.p->dots[1], s, c.mesh_elem_off[q],
                      c.mesh_elem_off[q + 1] - c.mesh_elem_off[q], c.mesh_face_off[q],
                      c.mesh_face_off[q + 1] - c.mesh_face_off[q]);
        SDG_HIP(hipMemcpyAsync(c.h_pinned, &c.d_sc.p->dots[1], sizeof(double), hipMemcpyDeviceToHost, s));
        SDG_HIP(hipStreamSynchronize(s));
        out[q] = c.h_pinned[0];
      }
      return;
    }
    for (int r = 0; r < n_rhs; ++r) {
      launch_energy(c, v_state + (int64_t)r * c.n_state, sigma_state + (int64_t)r * c.n_sig_state,
                    &c.d_sc.p->dots[1], s);
      SDG_HIP(hipMemcpyAsync(c.h_pinned, &c.d_sc.p->dots[1], sizeof(double), hipMemcpyDeviceToHost, s));
      SDG_HIP(hipStreamSynchronize(s));
      out[r] = c.h_pinned[0];
    }
  });
}

int sdg_sample_velocity(sdg_ctx* ctx, const double* v_state, int n_rhs, int64_t n_pts, const double* pts,
                        double* out, void* stream) {
  return guard([&] {
    Ctx& c = ctx_of(ctx);
    require(c.assembled, SDG_ESTATE, "assemble first");
    require(n_rhs >= 1 && n_rhs <= c.max_rhs, SDG_EINVAL, "n_rhs must be in [1, max_rhs of sdg_assemble]");
    require(n_pts >= 0 && (n_pts == 0 || (v_state && pts && out)), SDG_EINVAL, "null argument");
    if (n_pts == 0) return;
    SDG_HIP(hipSetDevice(c.device));
    hipStream_t s = (hipStream_t)stream;
    locate_points(c, n_pts, pts);
    const HostSetup& hs = c.hs;
    for (int r = 0; r < n_rhs; ++r)
      launch_sample(n_pts, hs.nphi, hs.dim, c.d_samp_elem.p, c.d_samp_phi.p, v_state + (int64_t)r * c.n_state,
                    out + (int64_t)r * n_pts * hs.dim, s);
    SDG_HIP(hipGetLastError());
    SDG_HIP(hipStreamSynchronize(s));
  });
}

int sdg_eval_stress(sdg_ctx* ctx, const double* sigma_state, int n_rhs, int64_t n_pts, const double* pts,
                    const int64_t* face, double* out, void* stream) {
  return guard([&] {
    Ctx& c = ctx_of(ctx);
    require(c.assembled, SDG_ESTATE, "assemble first");
    require(n_rhs == 1, SDG_EUNSUPPORTED, "batched right-hand sides are not built in this version");
    require(n_pts >= 0 && (n_pts == 0 || (sigma_state && pts && face && out)), SDG_EINVAL, "null argument");
    if (n_pts == 0) return;
    const HostSetup& hs = c.hs;
    std::vector<double> psi(n_pts * hs.npsi);
    for (int64_t q = 0; q < n_pts; ++q) {
      require(face[q] >= 0 && face[q] < hs.n_face, SDG_EINVAL, "face index out of range");
      eval_dual_canonical(hs, c.elem.data(), face[q], 1, pts + q * hs.dim, &psi[q * hs.npsi]);
    }
    SDG_HIP(hipSetDevice(c.device));
    hipStream_t s = (hipStream_t)stream;
    DevBuf<int64_t> df;
    DevBuf<double> dp;
    df.alloc(n_pts);
    dp.alloc(psi.size());
    SDG_HIP(hipMemcpy(df.p, face, n_pts * sizeof(int64_t), hipMemcpyHostToDevice));
    SDG_HIP(hipMemcpy(dp.p, psi.data(), psi.size() * sizeof(double), hipMemcpyHostToDevice));
    launch_eval_stress(n_pts, hs.npsi, hs.nsig, df.p, dp.p, sigma_state, out, s);
    SDG_HIP(hipStreamSynchronize(s));
  });
}

static void check_projection(const Ctx& c, int which, int degree) {
  require(c.assembled, SDG_ESTATE, "assemble first");
  require(which == 0 || which == 1, SDG_EINVAL, "which must be 0 (elements) or 1 (dual elements)");
  const int lo = projection_min_degree(c.hs, which);
  require(degree >= lo && degree <= lo + 16, SDG_EINVAL,
          "projection degree must be in [" + std::to_string(lo) + ", " + std::to_string(lo + 16) + "]");
}

int sdg_projection_points(const sdg_ctx* ctx, int which, int degree, int64_t* n_per_cell, double* pts,
                          double* wts) {
  return guard([&] {
    require(ctx != nullptr, SDG_EINVAL, "null context");
    const Ctx& c = *reinterpret_cast<const Ctx*>(ctx);
    check_projection(c, which, degree);
    const HostSetup& hs = c.hs;
    const int nq = projection_rule_size(hs, which, degree);
    if (n_per_cell) *n_per_cell = nq;
    if (pts) projection_points(hs, c.elem.data(), which, degree, pts, wts);
    else require(wts == nullptr, SDG_EINVAL, "weights are written together with the points");
  });
}

int sdg_project_state(sdg_ctx* ctx, int which, int degree, const double* values, double* out, void* stream) {
  return guard([&] {
    Ctx& c = ctx_of(ctx);
    check_projection(c, which, degree);
    require(values && out, SDG_EINVAL, "null argument");
    const HostSetup& hs = c.hs;
    const int64_t n = which == 0 ? c.n_state : c.n_sig_state;
    const int64_t nval =
        (which == 0 ? hs.n_elem * hs.dim : hs.n_face * hs.nsig) * projection_rule_size(hs, which, degree);
    for (int64_t i = 0; i < nval; ++i) require(std::isfinite(values[i]), SDG_ENONFINITE, "non-finite value");
    std::vector<double> host(n);
    project_values(hs, c.elem.data(), which, degree, values, host.data());
    SDG_HIP(hipSetDevice(c.device));
    hipStream_t s = (hipStream_t)stream;
    SDG_HIP(hipMemcpyAsync(out, host.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
    SDG_HIP(hipStreamSynchronize(s));
  });
}

}  // extern "C"
