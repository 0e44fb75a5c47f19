// Library context: host setup products, device copies of the operator and
// every workspace the apply / solve entry points use (allocated once, at
// assemble time).
#pragma once

#include <functional>

#include "sdg_internal.hpp"

namespace sdg {

constexpr int kMaxRestart = 32;
constexpr int kRedBlocks = 512;   // grid size of the reduction kernels
constexpr int kRedSlots = 2 * kMaxRestart + 2;  // partial-sum slots per reduction block

// Device-resident scalars of the Krylov solvers.
struct DevScalars {
  double rr, pq, rr_new, alpha, beta;
  double norm;          // last computed norm
  double inv_norm;
  double resid;         // GMRES residual estimate |g_{j+1}|
  double H[(kMaxRestart + 1) * kMaxRestart];  // column-major, ld = kMaxRestart+1
  double cs[kMaxRestart], sn[kMaxRestart];
  double g[kMaxRestart + 1];
  double h1[kMaxRestart + 1], h2[kMaxRestart + 1];
  double y[kMaxRestart];
  double dots[kRedSlots];
  double reorth;        // 1 when the current Arnoldi step needs a second projection
  double n_reorth;      // count of second projections (diagnostics)
  // delayed reorthogonalisation: the Hessenberg matrix before the Givens
  // rotations (column-major, ld = kMaxRestart+1) and the coefficients of the
  // update sweep (h2 holds the reorthogonalisation coefficients b)
  double Hu[(kMaxRestart + 1) * kMaxRestart];
  double f[kMaxRestart + 1];
  double e;
  // CG's stop on the device: the fused update's finalize counts the
  // iterations it ran, copies (r.r, count) to cg_stat for one read-back and
  // clears cg_on once sqrt(r.r) <= cg_tol; the iterations queued after that
  // return at entry.
  double cg_tol;
  double cg_stat[2];
  int cg_on, cg_iters;
};

// Scalars of one system of a multi-system Krylov solve.
struct SysScalars {
  double H[(kMaxRestart + 1) * kMaxRestart];  // column-major, ld = kMaxRestart+1
  double cs[kMaxRestart], sn[kMaxRestart];
  double g[kMaxRestart + 1];
  double h1[kMaxRestart + 1], h2[kMaxRestart + 1];
  double y[kMaxRestart];
  double dot, norm, inv_norm, resid, tol_abs, bnorm, rnorm;
  int32_t active, k;
  // delayed reorthogonalisation (as DevScalars)
  double Hu[(kMaxRestart + 1) * kMaxRestart];
  double f[kMaxRestart + 1];
  double e;
};
constexpr int kMaxSystems = 1024;

template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  void alloc(size_t count) {
    free();
    if (count == 0) return;
    SDG_HIP(hipMalloc(&p, count * sizeof(T)));
    n = count;
  }
  void free() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  ~DevBuf() { free(); }
};

// Independent systems as contiguous segments [off[s], off[s+1]) of one
// vector, with the reduction-block partition used by the segmented kernels.
// Operator of the multi-system solver: masked = true inside Arnoldi steps,
// where the work of converged systems may be skipped.
using MultiOp = std::function<void(const double*, double*, bool masked)>;

struct MultiSys {
  int S = 0;
  int64_t n_total = 0;
  int n_blocks = 0;
  std::vector<int64_t> off;
  DevBuf<int> d_blk_seg, d_seg_blk0;
  DevBuf<int64_t> d_blk_beg, d_blk_end;
  DevBuf<SysScalars> d_ss;
  DevBuf<double> d_partials;
  DevBuf<int> d_nactive;
  // iterative refinement driven on the device: outer ||b_s|| (S values),
  // then the last outer relative residual per system (S values)
  DevBuf<double> d_outer;
  DevBuf<int> d_nouter;  // systems whose outer residual is above rtol
  const int* active_flags() const;  // &d_ss[0].active (stride: mask_stride())
  static int mask_stride();
  int* h_pinned = nullptr;
  void build(const std::vector<int64_t>& offsets);
  void read_scalars(std::vector<SysScalars>& out, hipStream_t s) const;
  MultiSys() = default;
  MultiSys(const MultiSys&) = delete;
  MultiSys& operator=(const MultiSys&) = delete;
  ~MultiSys();
};

// Step recorded in HIP graphs, with the arguments it was recorded for.
struct StepGraphs {
  hipGraphExec_t head = nullptr, cycle = nullptr, verify = nullptr, tail = nullptr;
  hipGraphExec_t refine = nullptr;  // FP32 inner solves: x += e, new d, outer test
  // delayed GMRES: the restart cycle in parts between polls, and the early
  // ends of a cycle after each part but the last
  std::vector<hipGraphExec_t> part, stop;
  std::vector<int> part_end;
  int prec = 0;
  double inner_rtol = 0.0;
  hipStream_t stream = nullptr;
  const void *v = nullptr, *sig = nullptr, *vslab = nullptr, *sslab = nullptr;
  int R = 0, precond = 0, restart = 0, max_iter = 0, check_every = 0, flags = 0;
  double rtol = 0.0;
  bool src = false;
  void clear() {
    for (hipGraphExec_t* g : {&head, &cycle, &verify, &tail, &refine})
      if (*g) { (void)hipGraphExecDestroy(*g); *g = nullptr; }
    for (hipGraphExec_t g : part) (void)hipGraphExecDestroy(g);
    for (hipGraphExec_t g : stop) (void)hipGraphExecDestroy(g);
    part.clear();
    stop.clear();
    part_end.clear();
  }
  ~StepGraphs() {
    clear();
    if (stream) (void)hipStreamDestroy(stream);
  }
};

struct Ctx {
  int device = 0;
  // inputs
  int dim = 0;
  std::vector<double> xyz;
  std::vector<int64_t> elem;
  std::vector<double> period;
  bool have_mesh = false, have_disc = false, have_mat = false, assembled = false;
  int p = 0, pg = 0, scheme = 0;
  double dt = 0.0;
  std::vector<double> lam, mu, rho;
  // curved elements given by sdg_set_curved_elements (geometry degree, ids,
  // nodes); cleared with the mesh
  int curved_q = 0;
  std::vector<int64_t> curved_ids;
  std::vector<double> curved_nodes;
  // anisotropic material: per-element Voigt stiffness (n_elem * n_sigma^2)
  bool aniso = false;
  std::vector<double> elemE;
  unsigned precisions = 0;
  int max_rhs = 1;

  HostSetup hs;
  int64_t n_slab = 0, n_state = 0, n_sig_state = 0;

  // operator on device
  DevBuf<FaceRec> d_faces;
  DevBuf<double> d_Dt64;
  DevBuf<float> d_Dt32;
  DevBuf<double> d_face_lm, d_elem_w, d_Mref;
  DevBuf<double> d_face_E, d_face_Cw;  // anisotropic dual material (empty when isotropic)
  DevBuf<int> d_face_sys, d_elem_sys;   // mesh of each face / element (mesh batches only)
  // curved elements: index per element (-1 straight), their mass matrices
  // and the inverses of those (mass preconditioner); empty without curved
  // elements
  DevBuf<int32_t> d_curved_idx;
  DevBuf<double> d_curved_M, d_curved_Minv;
  DevBuf<double> d_z;  // element face slots
  Coefs op{}, adj{};   // operator and its transpose
  int variant64 = 0, variant32 = 0;   // face-kernel variant per precision (autotuned)
  double tune_us[2][kNumVariants] = {{0}};  // measured apply times [prec][variant]
  int bvariant = 0;              // batched FP64 apply: 0 column grid, 1/2 matrix-core kernel
  int bvariant32 = 0;            // the same for the FP32 apply
  double tune_b_us[3] = {0};     // measured batched FP64 applies (max_rhs columns) per bvariant
  double tune_b32_us[3] = {0};   // and FP32
  // preconditioners: mass block-Jacobi (reference mass inverse, 1/(rho|J|),
  // T^-1) and the element diagonal-block inverses of eq. (pre1) in FP32,
  // column-major per element
  DevBuf<double> d_Minv, d_winv;
  Coefs precF{}, precA{};
  DevBuf<float> d_Pblk;                 // explicit inverses (one time node), packed upper triangles
  DevBuf<float> d_Pq, d_Pb;             // factored inverses (several time nodes)
  bool pblk_factored = false;
  // patch preconditioner (Appendix A, eqs. APPRE1-APPRE2): first block rows
  // of the stencil inverses [elem][slot][q][r] and the stencils [elem][slot]
  DevBuf<float> d_P2;
  DevBuf<int32_t> d_P2nbr;
  int p2_nb = 0, p2_slots = 0;
  // compressed 3D operator (variant 8): per face side C, face-term
  // coefficients, per element |J| J^-1, reference tables
  DevBuf<double> d_cmpC64, d_cmpA, d_cmpB, d_cmpF, d_cmpG;
  DevBuf<float> d_cmpC32;
  int64_t cmp_bytes_f64 = 0, cmp_bytes_f32 = 0;

  // solver workspace
  DevBuf<double> d_V;                   // (restart+1) * n_slab   (GMRES) or 4 * n_slab (CG)
  DevBuf<double> d_x, d_b, d_r, d_w, d_t, d_d, d_e;
  DevBuf<double> d_partials;            // kRedSlots * kRedBlocks, slot-major
  DevBuf<double> d_cg_partials;         // fused CG update: r.r and r.z per element group
  DevBuf<float> d_cg32;                 // FP32-vector CG: r, p, q, z, x (n_slab each)
  DevBuf<DevScalars> d_sc;
  double* h_pinned = nullptr;           // pinned host copy of a few scalars
  // convergence poll of the delayed GMRES: {latest stamp, estimate of step
  // 0, 1, ... of the cycle} written by the device into coherent pinned
  // memory; stamps increase over the context's lifetime
  double* h_poll = nullptr;
  double* d_poll = nullptr;             // device address of h_poll
  double poll_seq = 0.0;
  DevBuf<double> d_tmp_state, d_tmp_sig; // state-sized scratch (energy, back-substitution)

  // sources (located for degree p_src on the current mesh)
  int64_t n_src = 0;
  int p_src = 0;
  std::vector<int64_t> src_elem;
  std::vector<double> src_phi, src_dir;
  DevBuf<double> d_src_phi, d_src_dir, d_src_amp;
  DevBuf<double> d_tw;  // time quadrature weights of the slab (CN: {1})
  DevBuf<double> d_e1;  // end-of-slab weights gamma_a(1)
  DevBuf<double> d_e0;  // start-of-slab weights gamma_a(0)

  // adjoint: stress multipliers of the slab, face gradients, element-face
  // table with the volume fractions of the dual-cell material
  DevBuf<double> d_lam_s, d_face_grad, d_detJ, d_ef_wt;
  DevBuf<int32_t> d_elem_face;
  DevBuf<int64_t> d_src_elem;

  // several independent systems: batched columns or a mesh batch
  int n_mesh = 1;
  std::vector<int64_t> mesh_vert_off, mesh_elem_off;  // n_mesh + 1 each
  std::vector<int64_t> mesh_face_off;                  // n_mesh + 1, set by sdg_assemble
  MultiSys msys;
  int msys_key = 0;        // columns the partition was built for (-1: mesh batch)
  int64_t z_col = 0;       // face-slot workspace per column

  StepGraphs graphs;
  // previous slab solution, for the extrapolated initial guess
  DevBuf<double> d_prev;
  bool prev_valid = false;
  int prev_R = 0;
  // one-node slabs (Crank-Nicolson, p_gamma = 0): the two slabs before d_prev
  // and how many of d_prev, d_prev2, d_prev3 hold consecutive slabs of the
  // current trajectory
  DevBuf<double> d_prev2, d_prev3;
  int prev_count = 0;

  // located sampling points of the last call
  std::vector<double> samp_pts;
  DevBuf<int64_t> d_samp_elem;
  DevBuf<double> d_samp_phi;

  ~Ctx() {
    if (h_pinned) (void)hipHostFree(h_pinned);
    if (h_poll) (void)hipHostFree(h_poll);
  }
};

// operator application on slab vectors (FP64 in / out)
// ncols > 1: ncols independent columns stored one after another (stride n_slab)
// z: face-slot workspace of z_col values per column (default: the context's)
void apply_op(Ctx& c, const double* v, double* y, int prec, bool transpose, hipStream_t s, int ncols = 1,
              void* z = nullptr, const int* mask_active = nullptr, double* dot_part = nullptr,
              const int* run_flag = nullptr);
bool fp32_vectors_ok(const Ctx& c);
void apply_op_f32v(Ctx& c, const float* v, float* y, hipStream_t s, double* dot_part, const int* run_flag = nullptr);

// Face-slot workspace of the allocation-free apply: a file-scope device
// array of noalloc_scratch_bytes() per GPU; noalloc_scratch(device) returns
// this device's copy (resolved once per device, with the device current).
size_t noalloc_scratch_bytes();
void* noalloc_scratch(int device);

// vector kernels
void vec_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);
void vec_copy(int64_t n, const double* x, double* y, hipStream_t s);
void vec_fill(int64_t n, double value, double* y, hipStream_t s);
double vec_dot_host(Ctx& c, int64_t n, const double* x, const double* y, hipStream_t s);

// solvers: solve A x = b in place (x holds the initial guess)
struct SolveResult {
  int iters = 0, matvecs = 0, refinements = 0;
  bool converged = false;
  double rel_res = 0.0, bnorm = 0.0;
};
struct KrylovCfg {
  double rtol = 1e-10;
  int max_iter = 1000, restart = 30, check_every = 5;
  int prec = SDG_PREC_F64;   // operator precision
  int precond = SDG_PRECOND_NONE;
  bool transpose = false;    // solve with A^T (adjoint)
  bool delayed = true;       // GMRES: delayed reorthogonalisation (one reduction per step)
  bool device_stop = false;  // CG with the fused update: stop on the device (SDG_SOLVE_DEVICE_STOP)
  bool x_zero = false;       // x is zero on entry: the first residual is b itself (no operator apply)
  bool keep_targets = false; // multi-system: per-system targets already set (multi_refine_check)
  // the caller tests the residual itself (inner solves of iterative
  // refinement): CG reports its recurrence's residual instead of applying
  // the operator once more at the end
  bool recurrence_only = false;
};
SolveResult solve_cg(Ctx& c, const double* b, double* x, const KrylovCfg& k, hipStream_t s);
SolveResult solve_gmres(Ctx& c, const double* b, double* x, const KrylovCfg& k, hipStream_t s);
// Pieces of the multi-system GMRES, also used to record the step in HIP
// graphs (poll = false: no host synchronisation inside):
//   multi_setup     per-system ||b||, tolerances, x = 0 where b = 0;
//   multi_residual  r = b - A x, per-system ||r||, activity flags;
//   multi_cycle     residual + one restart cycle of at most max_steps Arnoldi
//                   steps with device-side masks, then the correction.
void multi_setup(MultiSys& m, const double* b, double* x, double rtol, hipStream_t s);
void multi_residual(MultiSys& m, const double* b, const double* x, hipStream_t s,
                    const MultiOp& op, double* r);
int multi_cycle(MultiSys& m, const double* b, double* x, const KrylovCfg& k, hipStream_t s,
                const MultiOp& op,
                const std::function<void(const double*, double*)>* pre, double* V, double* r, double* w, double* t,
                bool poll, int max_steps, int* matvecs, bool* all_converged);
//   multi_cycle_part / multi_cycle_stop  the delayed cycle split at its
//                   polling points (graph mode records each part once)
void multi_cycle_part(MultiSys& m, const double* b, double* x, const KrylovCfg& k, hipStream_t s,
                      const MultiOp& op,
                      const std::function<void(const double*, double*)>* pre, double* V, double* w, double* t,
                      int steps, int j0, int j1, int* matvecs);
void multi_cycle_stop(MultiSys& m, double* x, const KrylovCfg& k, hipStream_t s,
                      const std::function<void(const double*, double*)>* pre, double* V, double* w, double* t,
                      int j);
int multi_nactive(MultiSys& m, hipStream_t s);
void multi_result(MultiSys& m, hipStream_t s, SolveResult& res);
// Iterative refinement with every decision on the device (graph-capturable):
//   multi_outer_setup   per-system ||b|| of the outer system;
//   multi_refine_check  from d = b - A x: per-system outer relative residual,
//                       the count of systems above rtol, and the inner
//                       targets (inner_rtol ||d_s||; none for converged
//                       systems, which then take no inner step);
//   multi_nouter        that count (host read, synchronises);
//   multi_outer_result  worst outer relative residual and largest ||b_s||.
void multi_outer_setup(MultiSys& m, const double* b, hipStream_t s);
void multi_refine_check(MultiSys& m, const double* d, double rtol, double inner_rtol, hipStream_t s);
int multi_nouter(MultiSys& m, hipStream_t s);
void multi_outer_result(MultiSys& m, hipStream_t s, SolveResult& res);
// Largest ||r_s|| / ||b_s|| over the systems of m (bnorm_max: largest ||b_s||).
double multi_rel_residual(MultiSys& m, const double* b, const double* r, hipStream_t s, double* bnorm_max);
MultiSys& systems(Ctx& c, int ncols);
void locate_points(Ctx& c, int64_t n_pts, const double* pts);
// Restarted GMRES on the independent systems of m (right preconditioning
// with *pre when given); V holds (restart+1) basis vectors of m.n_total.
SolveResult solve_gmres_multi(MultiSys& m, const double* b, double* x, const KrylovCfg& k, hipStream_t s,
                              const MultiOp& op,
                              const std::function<void(const double*, double*)>* pre, double* V, double* r,
                              double* w, double* t);
// y = P^-1 x for the chosen preconditioner (transpose: P^-T)
void apply_precond(Ctx& c, int kind, const double* x, double* y, bool transpose, hipStream_t s, int ncols = 1);
void launch_block_apply(int64_t n_elem, int nv, const float* P, const double* x, double* y, bool transpose,
                        hipStream_t s, int ncols = 1, int64_t cstride = 0);
void launch_block_apply_fact(int64_t n_elem, int ng, int ns, const float* Q, const float* B, const double* x,
                             double* y, bool transpose, hipStream_t s, int ncols = 1, int64_t cstride = 0);
void launch_patch_apply(int64_t n_elem, int nb, int slots, const float* P, const int32_t* nbr, const double* x,
                        double* y, hipStream_t s, int ncols, int64_t cstride);

// step pieces
void launch_broadcast_time(int64_t n_elem, int ng, int nvs, const double* state, double* slab,
                           hipStream_t s);
void launch_time_map(int64_t n_elem, int ng, int nvs, const double* Mt, const double* in, double* out,
                     hipStream_t s);
void launch_end_of_slab(int64_t n_elem, int ng, int nvs, const double* w, const double* slab,
                        double* state, hipStream_t s);
void launch_add_sources(Ctx& c, double* b, const double* amp_dev, hipStream_t s, int ncols = 1);
// energy of elements [e0, e0+ne) and faces [f0, f0+nf) (negative counts: to the end)
void launch_energy(Ctx& c, const double* v, const double* sig, double* out_dev, hipStream_t s, int64_t e0 = 0,
                   int64_t ne = -1, int64_t f0 = 0, int64_t nf = -1);
void launch_grad_rho(int64_t n_elem, int ng, int dim, int nphi, const RhoCoefs& tc, const double* Mref,
                     const double* detJ, const double* L, const double* X, const double* vold, double* g,
                     hipStream_t s);
void launch_face_to_elem(int64_t n_elem, int nfe, const int32_t* ef, const double* wt, const double* fg,
                         double* g_lam, double* g_mu, hipStream_t s);
void launch_sample_adjoint(int64_t n, int nphi, int dim, const int64_t* elem, const double* phi,
                           const double* obar, double* vbar, hipStream_t s);
void launch_sample(int64_t n, int nphi, int dim, const int64_t* elem, const double* phi,
                   const double* v, double* out, hipStream_t s);
void launch_eval_stress(int64_t n, int npsi, int nsig, const int64_t* face, const double* psi,
                        const double* sig, double* out, hipStream_t s);

}  // namespace sdg
