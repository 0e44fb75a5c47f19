/*
 * sdg.h -- C ABI of the MI355X library for the staggered space-time
 * discontinuous Galerkin scheme for linear elasticity of Tavelli & Dumbser
 * (arXiv:1802.04516).
 *
 * The hot path is the matrix-free application of the velocity Schur
 * complement, eq. (velocity.sys) of Section 4 and its Crank-Nicolson form
 * (velocity.sys.cn):
 *
 *     A = T (x) rho Mbar  +  dt^2 (W T^-1 W) (x) K,
 *     K v = sum_j D_j E_j sum_{i in {l(j), r(j)}} D_{i,j}^T v_i,
 *
 * where T, W are the time matrices of the Gauss-Legendre-Lagrange time basis
 * (Section 3), D_{i,j} the blocks of eq. (MD_3) expressed in an orthonormal
 * dual (stress) basis so that the dual mass matrices M_j of eq. (MD_2) are
 * the identity, and E_j the isotropic Hooke law of eq. (1.1b).  For
 * Crank-Nicolson A = rho Mbar + dt^2/4 K.
 *
 * Conventions
 *   - Every function returns SDG_OK (0) or a negative SDG_E* code; the
 *     message of the last failure on the calling thread is returned by
 *     sdg_last_error().  No C++ exception crosses the boundary.
 *   - Host arrays (const pointers documented as "host") are read during the
 *     call and copied; the caller keeps ownership.
 *   - Device arrays (documented as "device") are caller-owned allocations on
 *     the context's device, contiguous, float64 unless stated otherwise.
 *     The library never frees them and keeps no reference after the call.
 *   - `stream` is a hipStream_t (NULL = default stream).  Work is enqueued
 *     in stream order; only sdg_solve_step and the reductions returning host
 *     scalars synchronise the stream.
 *   - All workspace is allocated by sdg_assemble; the apply and solve entry
 *     points allocate nothing.
 *   - A context is used by one host thread at a time.
 *
 * Layouts at the boundary
 *   velocity slab    [elem][a][c][k]     a < N_gamma time node, c < dim
 *                                        component, k < N_phi nodal basis
 *                                        function (equispaced nodes of the
 *                                        reference simplex, order: 2D
 *                                        for j, for i: (i,j)/p; 3D for k,
 *                                        for j, for i: (i,j,k)/p).
 *   velocity state   [elem][c][k]        the end-of-slab value v(t^{n,-}).
 *   stress state     [face][s][m]        Voigt component s (2D: xx, yy, xy;
 *                                        3D: xx, yy, zz, yz, xz, xy,
 *                                        Section 2) and canonical dual basis
 *                                        function m.
 *   batched vectors  [r][...]: n_rhs right-hand sides stored one after
 *                                        another (column r of a velocity slab
 *                                        starts at r * n_vel_slab, of a state
 *                                        at r * n_vel_state, ...).
 *   Faces are numbered by ascending (l(j), local face of l(j)) where the
 *   left element l(j) is the lower element index and local face f of a
 *   simplex is the one opposite its local vertex f.
 *   Canonical dual basis of face j: the Gram-Schmidt orthonormalisation over
 *   the dual element R_j of
 *     2D: xi^a eta^b, (a, b) lexicographic with a major, a, b <= p, in the
 *         frame x = n1 + xi e1 + eta e2, e1 = (d1 - d2)/2, e2 = (d1 + d2)/2,
 *         d1 = n2 - n1 (face vertices, n1 of lower global vertex index),
 *         d2 = b_r - b_l (barycentres; on a boundary face b_r = n1 + n2 - b_l);
 *     3D: x^a y^b z^c of total degree <= p, by degree, then a descending,
 *         then b descending.
 */
#ifndef SDG_H
#define SDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SDG_OK = 0,
  SDG_EINVAL = -1,        /* bad argument (null pointer, size, enum value)          */
  SDG_ENOMEM = -2,        /* host or device allocation failed                       */
  SDG_EDEVICE = -3,       /* a HIP call failed                                      */
  SDG_EMESH = -4,         /* degenerate element, non-manifold or unmatched face     */
  SDG_ENOCONV = -5,       /* Krylov solver hit max_iter; state holds last iterate   */
  SDG_ENONFINITE = -6,    /* NaN/Inf met in a residual                              */
  SDG_EUNSUPPORTED = -7,  /* degree / dimension combination not compiled in         */
  SDG_ESTATE = -8         /* call order violated (e.g. apply before assemble)       */
};

enum { SDG_SCHEME_STDG = 0, SDG_SCHEME_CN = 1 };
enum { SDG_PREC_F64 = 1, SDG_PREC_F32 = 2 };
/* extra sdg_assemble flags: also build the block preconditioner (eq. pre1),
 * the patch preconditioner (eqs. APPRE1-APPRE2) */
enum { SDG_ASSEMBLE_BLOCK_PRECOND = 4, SDG_ASSEMBLE_PATCH_PRECOND = 8 };
enum { SDG_SOLVER_AUTO = 0, SDG_SOLVER_CG = 1, SDG_SOLVER_GMRES = 2 };
/* Preconditioners (Appendix A):
 * MASS  = element block-Jacobi on the mass term, (T (x) rho Mbar_i)^-1, no storage;
 * BLOCK = Pre1, element block-Jacobi on the full diagonal block of the
 *         velocity operator (eq. pre1), inverses stored at assemble time;
 * PATCH = Pre2, for each element the first block row of the inverse of the
 *         velocity operator restricted to the element and its face
 *         neighbours (eqs. APPRE1, APPRE2), stored at assemble time in FP32,
 *         (N_gamma d N_phi)^2 (d + 2) floats per element; not symmetric, so
 *         it is used with GMRES (CG rejects it) and not in the adjoint. */
enum { SDG_PRECOND_NONE = 0, SDG_PRECOND_MASS = 1, SDG_PRECOND_BLOCK = 2, SDG_PRECOND_PATCH = 3 };
/* Solve flags (sdg_solve_opts.flags):
 * GRAPH        replay the step from HIP graphs (see sdg_solve_step);
 * EXTRAPOLATE  initial guess continued from the previous slab (sdg_solve_step);
 * CGS2         single-system GMRES orthogonalises each new basis vector within
 *              its own step (classical Gram-Schmidt, a second projection when
 *              the test of Daniel, Gragg, Kaufman and Stewart asks for it: three
 *              sweeps over the basis).  The default delays the second projection
 *              of a vector to the next step (Swirydowicz et al. 2020, Bielich et
 *              al. 2022): one reduction and two sweeps per step; the residual
 *              estimate polled every check_every steps then lags by one step.
 * DEVICE_STOP  CG with the explicit element block preconditioner (Crank-
 *              Nicolson, Section 4) stops on the device: the iteration whose
 *              residual meets rtol clears a flag, and the up to check_every - 1
 *              iterations already queued behind it return at entry instead of
 *              iterating on.  The solution is then the first iterate that meets
 *              rtol (without the flag, the iterate of the next poll); the
 *              reported iterations are those that ran.  Ignored elsewhere. */
enum { SDG_SOLVE_GRAPH = 1, SDG_SOLVE_EXTRAPOLATE = 2, SDG_SOLVE_CGS2 = 4, SDG_SOLVE_DEVICE_STOP = 8 };

typedef struct sdg_ctx sdg_ctx;

typedef struct {
  int32_t dim, p, p_gamma, scheme;
  int32_t n_phi, n_psi, n_gamma, n_sigma;
  int64_t n_elem, n_face, n_face_boundary;
  int64_t n_vel_slab;     /* n_elem * n_gamma * dim * n_phi            */
  int64_t n_vel_state;    /* n_elem * dim * n_phi                      */
  int64_t n_stress_state; /* n_face * n_sigma * n_psi                  */
  int64_t n_stress_slab;  /* n_face * n_gamma * n_sigma * n_psi        */
  double dt;
  double tau[8];          /* time nodes of the slab in [0, 1]          */
  int64_t op_bytes_f64;   /* bytes of the stored FP64 operator blocks  */
  int64_t op_bytes_f32;
  int32_t max_rhs;        /* largest n_rhs accepted by the apply calls */
  int32_t op_variant;     /* face-kernel variant in use for FP64 (see sdg_set_operator_variant) */
  int32_t op_variant_f32;
  int32_t op_bvariant;    /* batched FP64 apply (see sdg_set_batched_variant) */
  double tune_us_f64[9];  /* autotuner timings of the variants (microseconds per apply; 0 = not available) */
  double tune_us_f32[9];
  double tune_us_batched[3]; /* batched applies of max_rhs columns per batched variant */
  int64_t cmp_bytes_f64;  /* bytes read per apply by the compressed 3D operator (variant 8), 0 if not built */
  int64_t cmp_bytes_f32;
  int32_t op_bvariant_f32;   /* batched FP32 apply */
  int32_t reserved0;
  double tune_us_batched_f32[3];
  int32_t proj_min_degree[2]; /* lowest rule degree sdg_projection_points / sdg_project_state accept for
                                 elements [0] and dual elements [1] */
} sdg_sizes;

typedef struct {
  int32_t solver;      /* SDG_SOLVER_*; AUTO = CG for Crank-Nicolson, GMRES otherwise    */
  int32_t precision;   /* SDG_PREC_F64, or SDG_PREC_F32 = FP32 operator inside FP64
                          iterative refinement (outer residuals and updates and every
                          inner product stay FP64; the inner CG of one system with the
                          block preconditioner and face-kernel variant 3 keeps its
                          vectors in FP32)                                            */
  double rtol;         /* stop when ||b - A v||_2 <= rtol ||b||_2                       */
  int32_t max_iter;    /* total Krylov iterations (inner iterations for FP32)          */
  int32_t restart;     /* GMRES restart length (<= 32)                                  */
  int32_t check_every; /* host convergence poll period in iterations                    */
  int32_t max_refine;  /* outer refinement sweeps for SDG_PREC_F32                      */
  double inner_rtol;   /* relative tolerance of each inner FP32 solve; a system's inner
                          solve reduces its right-hand side d only to 0.5 rtol ||b||
                          when that target is looser                              */
  int32_t precond;     /* SDG_PRECOND_*: right preconditioner (GMRES) / PCG (CG)        */
  int32_t flags;       /* SDG_SOLVE_GRAPH | _EXTRAPOLATE | _CGS2 | _DEVICE_STOP         */
} sdg_solve_opts;

typedef struct {
  int32_t iterations;  /* Krylov iterations performed                     */
  int32_t matvecs;     /* operator applications (all precisions)          */
  int32_t refinements; /* outer refinement sweeps (FP32 mode)             */
  int32_t converged;
  double rel_residual; /* final ||b - A v|| / ||b|| in FP64               */
  double b_norm;
} sdg_solve_info;

/* Message of the last failed call on this thread ("" if none). */
const char* sdg_last_error(void);

/* Create a context bound to HIP device `device`.  *out is set to NULL on
 * failure.  Returns SDG_EDEVICE if the device cannot be used. */
int sdg_create(sdg_ctx** out, int device);

/* Free the context and everything it allocated.  NULL-safe. */
void sdg_destroy(sdg_ctx* ctx);

/* Mesh (Section 3): n_vert vertices xyz[n_vert*dim] (host), n_elem simplices
 * elem[n_elem*(dim+1)] (host, vertex indices).  period (host, dim doubles)
 * or NULL: on a periodic mesh vertices on opposite sides are identified and
 * each element is unwrapped by the minimum-image rule relative to its first
 * vertex.  Boundary conditions (Section 6): the paper's tests use periodic
 * boundaries (given by `period`) and the free surface sigma . n = 0; a face
 * with a single element is a free-surface face, so no per-face boundary tag
 * is taken (an interior face cannot be free surface, and a one-sided face
 * has no other condition to carry).  The dual element of a free-surface face
 * is T_{l,j} alone and the face integral of eq. (MD_3) is dropped there
 * (natural traction-free condition).
 * Returns SDG_EMESH for a degenerate element, a face shared by more than
 * two elements or an unmatched periodic face.  Replaces any earlier mesh
 * and drops the point sources of sdg_set_sources. */
int sdg_set_mesh(sdg_ctx* ctx, int dim, int64_t n_vert, const double* xyz,
                 int64_t n_elem, const int64_t* elem, const double* period);

/* A batch of independent meshes of one dimension (Section 3 for each),
 * solved together: mesh q has vertices xyz[vert_off[q]*dim ..
 * vert_off[q+1]*dim) and elements elem[elem_off[q]*(dim+1) ..
 * elem_off[q+1]*(dim+1)) whose vertex indices are local to the mesh (host
 * arrays; offsets int64, n_mesh+1 entries starting at 0).  The library
 * concatenates them into one mesh (meshes share no faces, no periodicity):
 * elements, faces, materials and every state vector are laid out mesh after
 * mesh in element order, and sdg_solve_step runs one Krylov process per mesh
 * (own tolerance, segmented reductions) inside shared launches.  Boundary
 * faces are free surface as in sdg_set_mesh.  Replaces any earlier mesh and
 * drops the point sources. */
int sdg_set_mesh_batch(sdg_ctx* ctx, int dim, int n_mesh, const int64_t* vert_off, const double* xyz,
                       const int64_t* elem_off, const int64_t* elem);

/* Curved elements (Section 3: sub- and iso-parametric maps of the
 * reference triangle), 2D, on a single non-periodic mesh set by
 * sdg_set_mesh.  Element elem_ids[c] (c < n_curved, each listed once) is
 * the image of the reference triangle under the Lagrange map of degree q
 * (1..4) through its (q+1)(q+2)/2 geometry nodes, given in
 * nodes[c][node][2] (host) in the velocity node order of degree q:
 * node (i, j)/q of the reference triangle, for j in 0..q, for i in
 * 0..q-j, vertex 0 at (0,0), 1 at (1,0), 2 at (0,1).  The corner nodes must
 * be the element's vertices, and a face shared with another element must
 * be straight (its nodes at the affine positions): only boundary faces,
 * which are free surface, may curve (SDG_EMESH at sdg_assemble otherwise).
 * A curved element's velocity basis is the reference basis composed with
 * the inverse map; its barycentre and sub-simplices T_{i,j}, hence the dual
 * elements, are the images of the reference ones; its mass, coupling
 * blocks (eq. MD_3) and dual Gram matrices are integrated in reference
 * coordinates with |det J|.  Point sources, sampling and the projection of
 * initial data locate points in it by Newton iteration on the map.
 * n_curved = 0 removes all curved elements.  Cleared by sdg_set_mesh; drops
 * the point sources; takes effect at the next sdg_assemble.  The adjoint
 * step refuses a mesh with curved elements (SDG_EUNSUPPORTED); SDG_EINVAL
 * for a bad degree, index or node, SDG_EUNSUPPORTED in 3D, on a periodic
 * mesh or a mesh batch. */
int sdg_set_curved_elements(sdg_ctx* ctx, int q, int64_t n_curved, const int64_t* elem_ids,
                            const double* nodes);

/* Space degree p (Section 3: N_phi = C(p+dim, dim) velocity functions,
 * N_psi = (p+1)^2 in 2D and N_phi in 3D stress functions), time degree
 * p_gamma (N_gamma = p_gamma + 1), scheme SDG_SCHEME_STDG (eqs. NM25-NM26)
 * or SDG_SCHEME_CN (eqs. NM25.cn-NM26.cn, requires p_gamma = 0), time step
 * dt > 0.  SDG_EUNSUPPORTED if the (dim, p, N_gamma) kernels are not
 * compiled in.  A new p drops the point sources of sdg_set_sources (their
 * basis values belong to the old degree). */
int sdg_set_discretization(sdg_ctx* ctx, int p, int p_gamma, int scheme, double dt);

/* Per-element Lame parameters and density (host, n_elem each; lambda >= 0,
 * mu > 0, rho > 0).  The density is discretised on the main grid and the
 * stiffness on the dual grid (Section 4, eq. NM1); rho_i is taken constant
 * per element and E_j, the isotropic Hooke law of eq. (1.1b), constant per
 * dual element R_j with the volume-weighted lambda_j = (|T_{l,j}| lambda_l +
 * |T_{r,j}| lambda_r) / |R_j| and likewise mu_j (the L2 projection of the
 * piecewise-constant element values onto constants on R_j).  SDG_EINVAL for
 * a non-finite or out-of-range value. */
int sdg_set_material(sdg_ctx* ctx, const double* lambda, const double* mu, const double* rho);

/* General (anisotropic) linear elastic material, Section 2: per element the
 * n_sigma x n_sigma matrix E~ of the Voigt form s~ = E~ e~ (host, n_elem
 * matrices row-major, n_sigma = 3 in 2D, 6 in 3D), with the Voigt order
 * (xx, yy, xy) in 2D and (xx, yy, zz, yz, xz, xy) in 3D and the strain with
 * tensor shear components e_xy = (d_y u + d_x v) / 2, so that an isotropic
 * material has 2 mu on the shear diagonal (eq. 5), and density rho (n_elem,
 * > 0).  The stiffness tensor has the major symmetry E_ijkl = E_klij, which
 * makes E~ W^-1 symmetric (W = 1 on normal, 2 on shear components); the
 * library symmetrises it and rejects (SDG_EINVAL) a violation beyond 1e-12
 * of the largest entry, or a non-finite entry.  As in sdg_set_material,
 * E_j on the dual element R_j is the volume-weighted mean of its two
 * elements' E~ and must be positive definite (checked at sdg_assemble,
 * SDG_EINVAL).  The Hooke law of eq. (1.1) then enters every operator apply,
 * right-hand side, back-substitution and energy.  The face kernels that
 * apply it are variants 3, 4 and 8 (sdg_set_operator_variant refuses the
 * others, autotuning picks among these) and batched applies use the column
 * grid; sdg_adjoint_step refuses an anisotropic material
 * (SDG_EUNSUPPORTED).  sdg_set_material returns to an isotropic material. */
int sdg_set_material_anisotropic(sdg_ctx* ctx, const double* stiffness, const double* rho);

/* Build topology, geometry, bases and the operator blocks on the host and
 * upload them: the element mass Mbar_i and time matrices of eqs. (MD_2) to
 * (MD_2_3), the coupling blocks D_{i,j} of eq. (MD_3) in the canonical dual
 * basis (where M_j = I, and Q_{i,j} of eq. (MD_6) equals -D_{i,j}^T by the
 * identity of Section 5), and the dual material.  SDG_ESTATE unless mesh,
 * discretization and material are set; SDG_EMESH for a mesh the set-up
 * rejects.  precisions = SDG_PREC_F64 | SDG_PREC_F32 selects which
 * copies of the blocks are stored; OR in SDG_ASSEMBLE_BLOCK_PRECOND to also
 * invert the element diagonal blocks of the velocity operator (eq. pre1,
 * stored in FP32: (d N_phi)^2 floats per element for one time node; for
 * several, the generalised eigenvectors of the element stiffness and mass
 * and the N_gamma x N_gamma inverses per eigenvalue, (d N_phi)^2 +
 * d N_phi N_gamma^2 floats).  max_rhs (1..1024) sizes the workspaces for
 * batched applies and solves (every Krylov vector holds max_rhs columns). */
int sdg_assemble(sdg_ctx* ctx, unsigned precisions, int max_rhs);

/* Sizes of the assembled discretization (Section 3: N_phi, N_psi, N_gamma
 * and the unknown counts of eqs. NM25-NM26), the stored operator bytes and
 * the autotuner's choices and timings, copied to *out (host).  SDG_ESTATE
 * before sdg_assemble. */
int sdg_query(const sdg_ctx* ctx, sdg_sizes* out);

/* Face-kernel variant (tile shape) of the operator apply:
 *   0 = LDS kernel with flat loops;
 *   1 = register-tiled kernel with the most faces per workgroup that fit in
 *       64 KiB of LDS; 2 = the same with half as many;
 *   4 = column-parallel kernel (one thread per face and stress column, half
 *       of the at most 256/(d N_psi) faces per workgroup that fit in 64 KiB
 *       of LDS); 3 = the same kernel persistent (one workgroup per resident
 *       slot), loading the next chunk's blocks while computing the current
 *       one;
 *   5 = column-parallel kernel that reads the blocks from HBM straight into
 *       registers (about 256/(d N_psi) faces per workgroup); 6 = the same
 *       with the scatter summed across the face's lanes from the block
 *       columns already in registers (d N_psi rounded up to a power of two
 *       lanes per face; where that exceeds 64, variant 5);
 *   7 = one face per wavefront on the FP64 matrix cores (the face gradient
 *       and scatter as 16x16x4 MFMA sequences, the rows padded to 16; in
 *       FP32, or where N_gamma d > 16 or N_phi > 16, variant 5);
 *   8 = compressed 3D operator (tetrahedra, p <= 2; built by sdg_assemble
 *       beside the blocks): no block is read; each face side's block of eq.
 *       (MD_3) is applied through its factors, the change of basis C from
 *       the canonical dual basis to a reference basis of P_p on the side's
 *       reference sub-simplex (N_psi^2 values per side), the face-term
 *       coefficients of the side and |J| J^-1 of its element, and reference
 *       tables of the four local faces (SDG_EUNSUPPORTED elsewhere);
 *  -1 reruns the autotuner (sdg_assemble runs it: every variant is timed on
 *       the assembled operator and the fastest kept, per precision).
 * All variants compute the same operator. */
int sdg_set_operator_variant(sdg_ctx* ctx, int variant);

/* Kernel of the batched operator apply (n_rhs > 1), for both precisions:
 * 0 = the face kernel variant above launched once per column (column grid),
 * 1 and 2 = the matrix-core kernel (v_mfma_f64_16x16x4, or
 * v_mfma_f32_16x16x4 with FP32 face slots in an FP32 apply: the face
 * gradient and the scatter of each face become GEMMs over the columns)
 * with 8 or 16 columns per workgroup.  sdg_assemble picks the fastest per
 * precision for max_rhs columns when max_rhs > 1 (op_bvariant,
 * op_bvariant_f32); shapes the matrix-core kernel does not cover (N_gamma d
 * not dividing 16, or N_phi > 16) use the column grid whatever is set. */
int sdg_set_batched_variant(sdg_ctx* ctx, int bvariant);

/* Face table in the library's face order (Section 3: each face Gamma_j has a
 * left element l(j) and, off the boundary, a right element r(j); host arrays
 * of n_face entries):
 * left element, its local face, right element (-1 on the boundary), its
 * local face (-1 on the boundary).  Any pointer may be NULL. */
int sdg_face_table(const sdg_ctx* ctx, int64_t* left, int32_t* left_face,
                   int64_t* right, int32_t* right_face);

/* y = A v for n_rhs right-hand sides (device, slab layout, column after
 * column, n_rhs <= max_rhs), one launch of each kernel for all columns.
 * precision SDG_PREC_F64 or SDG_PREC_F32 (FP32 blocks and arithmetic, FP64
 * input/output).  v and y must not alias. */
int sdg_apply_velocity_operator(sdg_ctx* ctx, const double* v, double* y, int n_rhs,
                                int precision, void* stream);

/* Allocation-free form of sdg_apply_velocity_operator, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, layouts, result
 * (bit for bit) and errors, with one more limit: the face-slot workspace,
 * (dim+1) N_gamma dim N_phi FP64 values per element and column, lives in a
 * file-scope device array of 256 MiB per GPU (resolved by sdg_create, held
 * until the process ends) instead of the context's workspace; a larger
 * n_elem * n_rhs gives SDG_EINVAL.  The call makes no allocation.  Every
 * call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (concurrent streams or threads, any context) race and give undefined
 * results.  Every slot is written before it is read within a call, so
 * nothing from an earlier call carries over. */
int sdg_apply_velocity_operator_noalloc(sdg_ctx* ctx, const double* v, double* y, int n_rhs, int precision,
                                        void* stream);

/* y = P^-1 x for the preconditioner `kind` (SDG_PRECOND_*; NONE copies),
 * the approximate inverse the Krylov solves apply on the right (Appendix A):
 * x, y device slab vectors of n_rhs columns (must not alias).  SDG_ESTATE
 * if BLOCK or PATCH was not assembled. */
int sdg_apply_preconditioner(sdg_ctx* ctx, int kind, const double* x, double* y, int n_rhs, void* stream);

/* y = A^T w: the transpose of the velocity operator of eq. (velocity.sys),
 * A^T = T^T (x) rho Mbar + dt^2 (W T^-T W) (x) K (K is symmetric, Section 5),
 * used by the discrete adjoint.  Same arguments, layouts and errors as
 * sdg_apply_velocity_operator. */
int sdg_apply_adjoint(sdg_ctx* ctx, const double* w, double* y, int n_rhs,
                      int precision, void* stream);

/* Point sources S_v = d delta(x - x_s) S(t) / rho (Section 6.3): positions
 * pos[n_src*dim], directions dir[n_src*dim] (host).  Each source is located
 * once (lowest element index on ties) and its nodal basis values stored.
 * With n_rhs > 1, right-hand side r of a batched solve carries source
 * r % n_src only; with n_rhs = 1 all sources act together. */
int sdg_set_sources(sdg_ctx* ctx, int64_t n_src, const double* pos, const double* dir);

/* As sdg_set_sources on a mesh batch: source s is located in mesh mesh[s]
 * (host int32) only; all sources act in one solve. */
int sdg_set_mesh_sources(sdg_ctx* ctx, int64_t n_src, const double* pos, const double* dir,
                         const int32_t* mesh);

/* One implicit time step of n_rhs independent states:
 *   1. right-hand side of eq. (velocity.sys) (or velocity.sys.cn) from the
 *      old state v_state (device [r][elem][c][k]) and sigma_state (device
 *      [r][face][s][m]) plus the point sources with amplitudes
 *      amp[n_src*N_gamma] (host; S(t) at the slab's time nodes, the
 *      midpoint for Crank-Nicolson; NULL = no source);
 *   2. Krylov solve for the velocity slab (CG or restarted GMRES; with
 *      n_rhs > 1 or on a mesh batch, GMRES with one Arnoldi process, one
 *      tolerance and one convergence flag per column or mesh, sharing every
 *      kernel launch; rtol then bounds every column's relative residual);
 *   3. stress back-substitution, eq. (NM26) or (NM26.cn);
 *   4. overwrite v_state and sigma_state with the end-of-slab values.
 * v_slab / sigma_slab (device, optional) receive the slab DOFs.
 * The initial guess is the old state copied to every time node; with
 * opts->flags & SDG_SOLVE_EXTRAPOLATE it is the previous step's velocity
 * slab (kept by the context) continued to the new slab's time nodes, which
 * is meant for consecutive steps of one trajectory: the first such step,
 * or one after a step without the flag or with another n_rhs, starts from
 * the old state as usual.  With one time node per slab (Crank-Nicolson,
 * p_gamma = 0), where that continuation is the old state itself, the eager
 * step extrapolates the trajectory instead: 2 x_n - x_{n-1} from the second
 * such step and 3 x_n - 3 x_{n-1} + x_{n-2} from the third (x_k: the slab of
 * step k; the context keeps the last three, graph mode keeps the
 * continuation).  Every guess converges to the same tolerance.
 * On SDG_ENOCONV the states hold the step computed from the last iterate
 * and *info is filled.
 * With opts->flags & SDG_SOLVE_GRAPH (GMRES, FP64 or FP32 + refinement)
 * the step's launches are recorded once into HIP graphs (right-hand side +
 * first restart cycle, one restart cycle, residual check, back-substitution;
 * with SDG_PREC_F32 also the refinement update x += e with the new outer
 * residual) and replayed; the host only reads the device count of
 * unconverged systems between replays.  With the default delayed
 * orthogonalisation each restart cycle is recorded in parts of
 * check_every steps, polled between parts as the eager solver polls, so
 * both take the same iterations; with SDG_SOLVE_CGS2 every cycle runs its
 * full restart length (converged systems are masked on the device).  With
 * SDG_PREC_F32 each system's outer test runs on the device: a system that
 * has reached rtol takes no further inner step, and the step ends when
 * every system has, or after max_refine corrections.  The graphs are kept while the state, slab and amplitude
 * pointers, n_rhs and the solver options stay the same; they are rebuilt
 * otherwise and dropped by sdg_assemble, sdg_set_sources and
 * sdg_set_operator_variant.  The call synchronises `stream` before the
 * replays, which run on a stream of the context. */
int sdg_solve_step(sdg_ctx* ctx, double* v_state, double* sigma_state, const double* amp,
                   int n_rhs, const sdg_solve_opts* opts, sdg_solve_info* info,
                   double* v_slab, double* sigma_slab, void* stream);

/* Total energy 1/2 sum_i rho_i int |v|^2 + 1/2 sum_j int sigma : E_j^-1 sigma
 * (Section 5.2) of a state, FP64, written to out[n_rhs] (host), one value
 * per column; on a mesh batch (n_rhs = 1) out[n_mesh], one value per mesh. */
int sdg_energy(sdg_ctx* ctx, const double* v_state, const double* sigma_state, int n_rhs,
               double* out, void* stream);

/* Velocity of a state at n_pts host points pts[n_pts*dim], written to
 * out[n_rhs*n_pts*dim] (device, [r][pt][c]): the expansion of eq. (NM1),
 * v_h(x) = sum_k phi_k^(i)(x) v_{k,i} in the element i containing x (the
 * receivers of Section 6).  Points outside the mesh give SDG_EINVAL; a point
 * on a shared boundary takes the lowest element index.  The located elements of the last point set are kept, so
 * repeated calls with the same points locate them once. */
int sdg_sample_velocity(sdg_ctx* ctx, const double* v_state, int n_rhs, int64_t n_pts,
                        const double* pts, double* out, void* stream);

/* Stress of a state at points: the expansion of eq. (NM1) on the dual grid,
 * sigma_h(x) = sum_m psi_m^(j)(x) sigma_{m,j} in the canonical dual basis of
 * face j.  pts[n_pts*dim] (host) with the face index face[n_pts] (host) of
 * the dual element each point lies in; out [pt][s][r] (device).  SDG_EINVAL
 * for a face index out of range. */
int sdg_eval_stress(sdg_ctx* ctx, const double* sigma_state, int n_rhs, int64_t n_pts,
                    const double* pts, const int64_t* face, double* out, void* stream);

/* L2 projection of initial data onto the discrete spaces: the state at
 * t^{0,-} (the paper fixes no initial projection; this is the L2 projection
 * onto the velocity space of Section 3 per element, and onto the dual space
 * per dual element R_j in the canonical dual basis, where the dual mass is
 * the identity).  which = 0: elements, which = 1: dual elements.  degree:
 * the projection rule integrates polynomials of total degree <= degree
 * exactly; it must lie in [dmin, dmin + 16] with dmin = 2p for elements and
 * psi_deg + p for dual elements (psi_deg = 2p in 2D, p in 3D), so that the
 * mass of the discrete space is exact; larger degrees integrate
 * non-polynomial data more accurately.
 * sdg_projection_points writes the number of rule points per cell to
 * *n_per_cell and, when pts is not NULL, the points pts[cell][q][dim] and
 * weights wts[cell][q] (host; wts may be NULL).  On a periodic mesh the
 * points of a cell lie in its unwrapped frame (possibly outside the periodic
 * box).  A free-surface dual element is T_{l,j} alone: the second half of its
 * points repeats the first with zero weights.
 * sdg_project_state takes the caller's data at those points, values
 * [cell][q][comp] (host; comp = dim velocity components, or n_sigma Voigt
 * stresses), and writes the projected state to out (device; velocity state
 * [elem][c][k] or stress state [face][s][m]).  Synchronises `stream`.
 * SDG_ENONFINITE for a non-finite value, SDG_EINVAL for a degree out of
 * range. */
int sdg_projection_points(const sdg_ctx* ctx, int which, int degree, int64_t* n_per_cell, double* pts,
                          double* wts);
int sdg_project_state(sdg_ctx* ctx, int which, int degree, const double* values, double* out, void* stream);

/* Discrete adjoint of one implicit step (Lagrangian method applied to the
 * slab system of eqs. NM25/NM26, or NM25.cn/NM26.cn).  Write the step as
 *   A(theta) X = Bm(theta) u_old + F,   u_new = Ex X,
 * with X the slab DOFs, u = (v, sigma) the states at t^{n,-} and t^{n+1,-},
 * theta the per-element lambda, mu, rho.  Given the adjoint of the new state
 * ubar_new = (vbar, sigma_bar) (device; velocity [elem][c][k], stress
 * [face][s][m] in the canonical dual basis, i.e. dJ/du_new including the
 * misfit terms at t^{n+1,-}), this call
 *   1. forms the right-hand side Ex^T ubar_new of the transposed system
 *      reduced to the velocity unknowns;
 *   2. solves A_v^T L_v = b with the Krylov method of opts (FP64 only;
 *      the velocity operator is the transpose of eq. (velocity.sys));
 *   3. back-substitutes the stress multipliers L_s;
 *   4. adds to grad (device, [3][n_elem]: lambda, mu, rho) the term
 *      L^T (dBm/dtheta u_old - dA/dtheta X).  The face parameters are the
 *      volume-weighted element parameters of the two sub-triangles of the
 *      dual cell, so face gradients are passed to the elements with the
 *      weights |T_{i,j}|/|R_j|;
 *   5. overwrites vbar, sigma_bar with Bm^T L = the adjoint of u_old.
 * v_old (device [elem][c][k]) is the forward state at t^{n,-} and v_slab
 * (device [elem][a][c][k]) the forward velocity slab of the step, as
 * returned in sdg_solve_step's v_slab.  The source term does not depend on
 * theta.  On SDG_ENOCONV the outputs hold the values from the last iterate
 * and *info is filled. */
int sdg_adjoint_step(sdg_ctx* ctx, const double* v_old, const double* v_slab, double* vbar,
                     double* sigma_bar, double* grad, const sdg_solve_opts* opts,
                     sdg_solve_info* info, void* stream);

/* Transpose of sdg_sample_velocity (the point evaluation of eq. NM1), for
 * the adjoint of a receiver misfit: vbar[e(x_q)][c][k] += phi_k(x_q)
 * obs_bar[q][c] for the host points pts[n_pts*dim] (obs_bar device
 * [pt][c], vbar device [elem][c][k]).  SDG_EINVAL for a point outside the
 * mesh.  Points are processed in order, so the
 * result is deterministic when several lie in one element. */
int sdg_sample_velocity_adjoint(sdg_ctx* ctx, int n_rhs, int64_t n_pts, const double* pts,
                                const double* obs_bar, double* vbar, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SDG_H */
