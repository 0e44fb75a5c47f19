"""MI355X library for the staggered space-time DG scheme for linear elasticity
(Tavelli & Dumbser, arXiv:1802.04516): Python binding of the C ABI.

This module only marshals arguments into ``libsdg.so`` (see include/sdg.h);
every step of the hot path runs in the library's HIP kernels.  PyTorch is
used for device memory and streams.  There is no fallback: if the library is
not built, or a GPU is not present, the calls raise.

The functions ``sdg_*`` mirror the C entry points one to one; ``Context``
wraps them for convenience.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsdg.so")

SDG_OK = 0
SDG_EINVAL, SDG_ENOMEM, SDG_EDEVICE, SDG_EMESH = -1, -2, -3, -4
SDG_ENOCONV, SDG_ENONFINITE, SDG_EUNSUPPORTED, SDG_ESTATE = -5, -6, -7, -8
SDG_SCHEME_STDG, SDG_SCHEME_CN = 0, 1
SDG_PREC_F64, SDG_PREC_F32 = 1, 2
SDG_ASSEMBLE_BLOCK_PRECOND = 4
SDG_ASSEMBLE_PATCH_PRECOND = 8
SDG_SOLVER_AUTO, SDG_SOLVER_CG, SDG_SOLVER_GMRES = 0, 1, 2
SDG_PRECOND_NONE, SDG_PRECOND_MASS, SDG_PRECOND_BLOCK, SDG_PRECOND_PATCH = 0, 1, 2, 3
N_VARIANTS = 9
SDG_SOLVE_GRAPH = 1
SDG_SOLVE_EXTRAPOLATE = 2
SDG_SOLVE_CGS2 = 4
SDG_SOLVE_DEVICE_STOP = 8

_ERRNAMES = {SDG_EINVAL: "EINVAL", SDG_ENOMEM: "ENOMEM", SDG_EDEVICE: "EDEVICE", SDG_EMESH: "EMESH",
             SDG_ENOCONV: "ENOCONV", SDG_ENONFINITE: "ENONFINITE", SDG_EUNSUPPORTED: "EUNSUPPORTED",
             SDG_ESTATE: "ESTATE"}

EXPORTED = ("sdg_last_error", "sdg_create", "sdg_destroy", "sdg_set_mesh", "sdg_set_discretization",
            "sdg_set_material", "sdg_set_material_anisotropic", "sdg_set_curved_elements", "sdg_assemble", "sdg_query", "sdg_set_operator_variant", "sdg_set_batched_variant", "sdg_face_table",
            "sdg_apply_velocity_operator", "sdg_apply_adjoint", "sdg_set_sources", "sdg_solve_step",
            "sdg_energy", "sdg_sample_velocity", "sdg_eval_stress", "sdg_adjoint_step",
            "sdg_sample_velocity_adjoint", "sdg_set_mesh_batch", "sdg_set_mesh_sources",
            "sdg_projection_points", "sdg_project_state", "sdg_apply_velocity_operator_noalloc",
            "sdg_apply_preconditioner")


class SdgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class Sizes(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("p", ctypes.c_int32), ("p_gamma", ctypes.c_int32),
                ("scheme", ctypes.c_int32), ("n_phi", ctypes.c_int32), ("n_psi", ctypes.c_int32),
                ("n_gamma", ctypes.c_int32), ("n_sigma", ctypes.c_int32), ("n_elem", ctypes.c_int64),
                ("n_face", ctypes.c_int64), ("n_face_boundary", ctypes.c_int64),
                ("n_vel_slab", ctypes.c_int64), ("n_vel_state", ctypes.c_int64),
                ("n_stress_state", ctypes.c_int64), ("n_stress_slab", ctypes.c_int64),
                ("dt", ctypes.c_double), ("tau", ctypes.c_double * 8), ("op_bytes_f64", ctypes.c_int64),
                ("op_bytes_f32", ctypes.c_int64), ("max_rhs", ctypes.c_int32), ("op_variant", ctypes.c_int32),
                ("op_variant_f32", ctypes.c_int32), ("op_bvariant", ctypes.c_int32),
                ("tune_us_f64", ctypes.c_double * 9), ("tune_us_f32", ctypes.c_double * 9),
                ("tune_us_batched", ctypes.c_double * 3), ("cmp_bytes_f64", ctypes.c_int64),
                ("cmp_bytes_f32", ctypes.c_int64), ("op_bvariant_f32", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("tune_us_batched_f32", ctypes.c_double * 3), ("proj_min_degree", ctypes.c_int32 * 2)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int32), ("precision", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("restart", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("max_refine", ctypes.c_int32), ("inner_rtol", ctypes.c_double), ("precond", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("matvecs", ctypes.c_int32), ("refinements", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("rel_residual", ctypes.c_double), ("b_norm", ctypes.c_double)]


_lib = None
_P = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)
_I64P = ctypes.POINTER(ctypes.c_int64)
_I32P = ctypes.POINTER(ctypes.c_int32)


def lib():
    """Load libsdg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1802_04516_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    i = ctypes.c_int
    sig = {
        "sdg_last_error": ([], ctypes.c_char_p),
        "sdg_create": ([ctypes.POINTER(_P), i], i),
        "sdg_destroy": ([_P], None),
        "sdg_set_mesh": ([_P, i, ctypes.c_int64, _DP, ctypes.c_int64, _I64P, _DP], i),
        "sdg_set_discretization": ([_P, i, i, i, ctypes.c_double], i),
        "sdg_set_material": ([_P, _DP, _DP, _DP], i),
        "sdg_set_material_anisotropic": ([_P, _DP, _DP], i),
        "sdg_set_curved_elements": ([_P, i, ctypes.c_int64, _I64P, _DP], i),
        "sdg_assemble": ([_P, ctypes.c_uint, i], i),
        "sdg_query": ([_P, ctypes.POINTER(Sizes)], i),
        "sdg_set_operator_variant": ([_P, i], i),
        "sdg_set_batched_variant": ([_P, i], i),
        "sdg_face_table": ([_P, _I64P, _I32P, _I64P, _I32P], i),
        "sdg_apply_velocity_operator": ([_P, _P, _P, i, i, _P], i),
        "sdg_apply_adjoint": ([_P, _P, _P, i, i, _P], i),
        "sdg_apply_velocity_operator_noalloc": ([_P, _P, _P, i, i, _P], i),
        "sdg_apply_preconditioner": ([_P, i, _P, _P, i, _P], i),
        "sdg_set_sources": ([_P, ctypes.c_int64, _DP, _DP], i),
        "sdg_solve_step": ([_P, _P, _P, _DP, i, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), _P, _P, _P], i),
        "sdg_energy": ([_P, _P, _P, i, _DP, _P], i),
        "sdg_sample_velocity": ([_P, _P, i, ctypes.c_int64, _DP, _P, _P], i),
        "sdg_eval_stress": ([_P, _P, i, ctypes.c_int64, _DP, _I64P, _P, _P], i),
        "sdg_adjoint_step": ([_P, _P, _P, _P, _P, _P, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), _P], i),
        "sdg_sample_velocity_adjoint": ([_P, i, ctypes.c_int64, _DP, _P, _P, _P], i),
        "sdg_set_mesh_batch": ([_P, i, i, _I64P, _DP, _I64P, _I64P], i),
        "sdg_set_mesh_sources": ([_P, ctypes.c_int64, _DP, _DP, ctypes.POINTER(ctypes.c_int32)], i),
        "sdg_projection_points": ([_P, i, i, _I64P, _DP, _DP], i),
        "sdg_project_state": ([_P, i, i, _DP, _P, _P], i),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(rc: int):
    if rc != SDG_OK:
        raise SdgError(rc, lib().sdg_last_error().decode())


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


def _hp(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype)) if a is not None else None


def _dev(t, numel=None, name="tensor"):
    """Device pointer of a contiguous float64 CUDA/HIP tensor."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor on the GPU")
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 GPU tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------- C mirrors

def sdg_create(device: int = 0):
    h = _P()
    _check(lib().sdg_create(ctypes.byref(h), device))
    return h


def sdg_destroy(h):
    lib().sdg_destroy(h)


def sdg_set_mesh(h, xyz, elem, period=None):
    xyz = _host(xyz, np.float64)
    elem = _host(elem, np.int64)
    dim = xyz.shape[1]
    per = _host(period, np.float64) if period is not None else None
    _check(lib().sdg_set_mesh(h, dim, xyz.shape[0], _hp(xyz, ctypes.c_double), elem.shape[0],
                              _hp(elem, ctypes.c_int64), _hp(per, ctypes.c_double)))


def sdg_set_mesh_batch(h, meshes):
    """meshes: sequence of (xyz (nv, dim), elem (ne, dim+1)) with local vertex indices."""
    xyz = [_host(m[0], np.float64) for m in meshes]
    elem = [_host(m[1], np.int64) for m in meshes]
    dim = xyz[0].shape[1]
    voff = np.concatenate([[0], np.cumsum([x.shape[0] for x in xyz])]).astype(np.int64)
    eoff = np.concatenate([[0], np.cumsum([e.shape[0] for e in elem])]).astype(np.int64)
    X = np.ascontiguousarray(np.concatenate(xyz, axis=0))
    E = np.ascontiguousarray(np.concatenate(elem, axis=0))
    _check(lib().sdg_set_mesh_batch(h, dim, len(meshes), _hp(voff, ctypes.c_int64), _hp(X, ctypes.c_double),
                                    _hp(eoff, ctypes.c_int64), _hp(E, ctypes.c_int64)))
    return voff, eoff


def sdg_set_mesh_sources(h, pos, direction, mesh):
    pos = _host(pos, np.float64)
    d = _host(direction, np.float64)
    mesh = _host(mesh, np.int32)
    _check(lib().sdg_set_mesh_sources(h, pos.shape[0], _hp(pos, ctypes.c_double), _hp(d, ctypes.c_double),
                                      _hp(mesh, ctypes.c_int32)))


def sdg_set_discretization(h, p, p_gamma, scheme, dt):
    _check(lib().sdg_set_discretization(h, p, p_gamma, scheme, float(dt)))


def sdg_set_material(h, lam, mu, rho):
    lam, mu, rho = (_host(x, np.float64) for x in (lam, mu, rho))
    _check(lib().sdg_set_material(h, _hp(lam, ctypes.c_double), _hp(mu, ctypes.c_double),
                                  _hp(rho, ctypes.c_double)))


def sdg_set_material_anisotropic(h, stiffness, rho):
    """stiffness: (n_elem, n_sigma, n_sigma) Voigt matrices E~ (tensor shear
    strains, so 2 mu on the isotropic shear diagonal); rho: (n_elem,)."""
    E, rho = _host(stiffness, np.float64), _host(rho, np.float64)
    if E.ndim != 3 or E.shape[1] != E.shape[2] or E.shape[0] != rho.shape[0]:
        raise ValueError("stiffness must be (n_elem, n_sigma, n_sigma) and rho (n_elem,)")
    _check(lib().sdg_set_material_anisotropic(h, _hp(E, ctypes.c_double), _hp(rho, ctypes.c_double)))


def sdg_set_curved_elements(h, ids, nodes):
    """ids: (n_c,) element indices; nodes: (n_c, (q+1)(q+2)/2, 2) geometry
    nodes of degree q in the velocity node order (None, None: no curved
    elements)."""
    if ids is None or len(ids) == 0:
        _check(lib().sdg_set_curved_elements(h, 1, 0, None, None))
        return
    ids = _host(ids, np.int64)
    nodes = _host(nodes, np.float64)
    nq = nodes.shape[1]
    q = next((k for k in range(1, 5) if (k + 1) * (k + 2) // 2 == nq), None)
    if q is None or nodes.shape[0] != ids.shape[0] or nodes.shape[2] != 2:
        raise ValueError("nodes must be (n_curved, (q+1)(q+2)/2, 2) with q in 1..4")
    _check(lib().sdg_set_curved_elements(h, q, ids.shape[0], _hp(ids, ctypes.c_int64), _hp(nodes, ctypes.c_double)))


def sdg_assemble(h, precisions=SDG_PREC_F64 | SDG_PREC_F32, max_rhs=1):
    _check(lib().sdg_assemble(h, precisions, max_rhs))


def sdg_query(h) -> dict:
    s = Sizes()
    _check(lib().sdg_query(h, ctypes.byref(s)))
    out = {f: getattr(s, f) for f, _ in Sizes._fields_
           if f not in ("tau", "tune_us_f64", "tune_us_f32", "tune_us_batched", "tune_us_batched_f32", "reserved0",
                        "proj_min_degree")}
    out["tau"] = [s.tau[a] for a in range(s.n_gamma)]
    out["tune_us_f64"] = list(s.tune_us_f64)
    out["tune_us_f32"] = list(s.tune_us_f32)
    out["tune_us_batched"] = list(s.tune_us_batched)
    out["tune_us_batched_f32"] = list(s.tune_us_batched_f32)
    out["proj_min_degree"] = list(s.proj_min_degree)
    return out


def sdg_set_operator_variant(h, variant):
    _check(lib().sdg_set_operator_variant(h, variant))


def sdg_face_table(h, n_face):
    l = np.empty(n_face, np.int64)
    lf = np.empty(n_face, np.int32)
    r = np.empty(n_face, np.int64)
    rf = np.empty(n_face, np.int32)
    _check(lib().sdg_face_table(h, _hp(l, ctypes.c_int64), _hp(lf, ctypes.c_int32), _hp(r, ctypes.c_int64),
                                _hp(rf, ctypes.c_int32)))
    return l, lf, r, rf


def sdg_apply_velocity_operator(h, v, y, n_rhs=1, precision=SDG_PREC_F64, stream=None):
    _check(lib().sdg_apply_velocity_operator(h, _dev(v, name="v"), _dev(y, name="y"), n_rhs, precision,
                                             _stream(stream)))


def sdg_apply_velocity_operator_noalloc(h, v, y, n_rhs=1, precision=SDG_PREC_F64, stream=None):
    _check(lib().sdg_apply_velocity_operator_noalloc(h, _dev(v, name="v"), _dev(y, name="y"), n_rhs, precision,
                                                     _stream(stream)))


def sdg_apply_preconditioner(h, kind, x, y, n_rhs=1, stream=None):
    _check(lib().sdg_apply_preconditioner(h, kind, _dev(x, name="x"), _dev(y, name="y"), n_rhs, _stream(stream)))


def sdg_apply_adjoint(h, w, y, n_rhs=1, precision=SDG_PREC_F64, stream=None):
    _check(lib().sdg_apply_adjoint(h, _dev(w, name="w"), _dev(y, name="y"), n_rhs, precision, _stream(stream)))


def sdg_set_sources(h, pos, direction):
    pos = _host(pos, np.float64)
    d = _host(direction, np.float64)
    _check(lib().sdg_set_sources(h, pos.shape[0], _hp(pos, ctypes.c_double), _hp(d, ctypes.c_double)))


def sdg_solve_step(h, v_state, sigma_state, amp=None, n_rhs=1, opts: SolveOpts | None = None,
                   v_slab=None, sigma_slab=None, stream=None, raise_on_noconv=True):
    opts = opts or SolveOpts(SDG_SOLVER_AUTO, SDG_PREC_F64, 1e-10, 1000, 30, 5, 10, 1e-4, SDG_PRECOND_MASS)
    info = SolveInfo()
    a = _host(amp, np.float64) if amp is not None else None
    rc = lib().sdg_solve_step(h, _dev(v_state, name="v_state"), _dev(sigma_state, name="sigma_state"),
                              _hp(a, ctypes.c_double), n_rhs, ctypes.byref(opts), ctypes.byref(info),
                              _dev(v_slab, name="v_slab") if v_slab is not None else None,
                              _dev(sigma_slab, name="sigma_slab") if sigma_slab is not None else None,
                              _stream(stream))
    res = {f: getattr(info, f) for f, _ in SolveInfo._fields_}
    if rc == SDG_ENOCONV and not raise_on_noconv:
        return res
    _check(rc)
    return res


def sdg_adjoint_step(h, v_old, v_slab, vbar, sigma_bar, grad, opts: SolveOpts | None = None, stream=None):
    """One backward step of the discrete adjoint; vbar, sigma_bar are
    overwritten with the adjoint of the start-of-step state and grad
    ([3, n_elem]: lambda, mu, rho) is accumulated."""
    opts = opts or SolveOpts(SDG_SOLVER_AUTO, SDG_PREC_F64, 1e-12, 2000, 30, 5, 10, 1e-4, SDG_PRECOND_MASS)
    info = SolveInfo()
    _check(lib().sdg_adjoint_step(h, _dev(v_old, name="v_old"), _dev(v_slab, name="v_slab"), _dev(vbar, name="vbar"),
                                  _dev(sigma_bar, name="sigma_bar"), _dev(grad, name="grad"), ctypes.byref(opts),
                                  ctypes.byref(info), _stream(stream)))
    return {f: getattr(info, f) for f, _ in SolveInfo._fields_}


def sdg_sample_velocity_adjoint(h, pts, obs_bar, vbar, n_rhs=1, stream=None):
    pts = _host(pts, np.float64)
    _check(lib().sdg_sample_velocity_adjoint(h, n_rhs, pts.shape[0], _hp(pts, ctypes.c_double),
                                             _dev(obs_bar, name="obs_bar"), _dev(vbar, name="vbar"),
                                             _stream(stream)))


def sdg_energy(h, v_state, sigma_state, n_rhs=1, stream=None, n_out=None):
    out = np.zeros(max(n_rhs, n_out or 1))
    _check(lib().sdg_energy(h, _dev(v_state, name="v_state"), _dev(sigma_state, name="sigma_state"), n_rhs,
                            _hp(out, ctypes.c_double), _stream(stream)))
    return out


def sdg_sample_velocity(h, v_state, pts, out, n_rhs=1, stream=None):
    pts = _host(pts, np.float64)
    _check(lib().sdg_sample_velocity(h, _dev(v_state, name="v_state"), n_rhs, pts.shape[0],
                                     _hp(pts, ctypes.c_double), _dev(out, name="out"), _stream(stream)))


def sdg_eval_stress(h, sigma_state, pts, face, out, n_rhs=1, stream=None):
    pts = _host(pts, np.float64)
    face = _host(face, np.int64)
    _check(lib().sdg_eval_stress(h, _dev(sigma_state, name="sigma_state"), n_rhs, pts.shape[0],
                                 _hp(pts, ctypes.c_double), _hp(face, ctypes.c_int64), _dev(out, name="out"),
                                 _stream(stream)))


def projection_min_degree(dim, p, which):
    """Lowest projection rule degree accepted for elements (0) or dual
    elements (1) on a mesh of straight elements (sdg_query reports it for
    the assembled mesh, curved elements included)."""
    return 2 * p if which == 0 else (2 * p if dim == 2 else p) + p


def sdg_projection_points(h, which, degree, n_cells, dim):
    """Points (n_cells, nq, dim) and weights (n_cells, nq) of the projection
    rule of elements (which = 0) or dual elements (which = 1)."""
    nq = ctypes.c_int64(0)
    _check(lib().sdg_projection_points(h, which, degree, ctypes.byref(nq), None, None))
    pts = np.empty((n_cells, nq.value, dim))
    wts = np.empty((n_cells, nq.value))
    _check(lib().sdg_projection_points(h, which, degree, ctypes.byref(nq), _hp(pts, ctypes.c_double),
                                       _hp(wts, ctypes.c_double)))
    return pts, wts


def sdg_project_state(h, which, degree, values, out, stream=None):
    values = _host(values, np.float64)
    _check(lib().sdg_project_state(h, which, degree, _hp(values, ctypes.c_double), _dev(out, name="out"),
                                   _stream(stream)))


# ---------------------------------------------------------------- convenience wrapper

class Context:
    """One mesh / discretisation / material on one GPU."""

    def __init__(self, device: int = 0):
        self.h = sdg_create(device)
        self.device = device
        self.sizes = None
        self.mesh_elem_off = None

    def close(self):
        if self.h:
            sdg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def setup(self, mesh_xyz, elem, period, p, p_gamma, scheme, dt, lam, mu, rho,
              precisions=SDG_PREC_F64 | SDG_PREC_F32, max_rhs=1):
        sdg_set_mesh(self.h, mesh_xyz, elem, period)
        self.mesh_elem_off = None
        sdg_set_discretization(self.h, p, p_gamma, scheme, dt)
        sdg_set_material(self.h, lam, mu, rho)
        sdg_assemble(self.h, precisions, max_rhs)
        self.sizes = sdg_query(self.h)
        return self.sizes

    def setup_curved(self, mesh_xyz, elem, curved, p, p_gamma, scheme, dt, lam, mu, rho,
                     precisions=SDG_PREC_F64 | SDG_PREC_F32, max_rhs=1):
        """As setup() on a non-periodic 2D mesh with curved elements
        curved = (element ids, geometry nodes (n_c, N_q, 2))."""
        sdg_set_mesh(self.h, mesh_xyz, elem, None)
        self.mesh_elem_off = None
        sdg_set_curved_elements(self.h, *curved)
        sdg_set_discretization(self.h, p, p_gamma, scheme, dt)
        sdg_set_material(self.h, lam, mu, rho)
        sdg_assemble(self.h, precisions, max_rhs)
        self.sizes = sdg_query(self.h)
        return self.sizes

    def setup_anisotropic(self, mesh_xyz, elem, period, p, p_gamma, scheme, dt, stiffness, rho,
                          precisions=SDG_PREC_F64 | SDG_PREC_F32, max_rhs=1):
        """As setup(), with per-element Voigt stiffness matrices E~ (Section 2)."""
        sdg_set_mesh(self.h, mesh_xyz, elem, period)
        self.mesh_elem_off = None
        sdg_set_discretization(self.h, p, p_gamma, scheme, dt)
        sdg_set_material_anisotropic(self.h, stiffness, rho)
        sdg_assemble(self.h, precisions, max_rhs)
        self.sizes = sdg_query(self.h)
        return self.sizes

    def setup_batch(self, meshes, p, p_gamma, scheme, dt, lam, mu, rho, precisions=SDG_PREC_F64 | SDG_PREC_F32):
        """Several independent meshes (list of (xyz, elem)) solved together;
        lam, mu, rho are concatenated mesh after mesh."""
        voff, eoff = sdg_set_mesh_batch(self.h, meshes)
        sdg_set_discretization(self.h, p, p_gamma, scheme, dt)
        sdg_set_material(self.h, lam, mu, rho)
        sdg_assemble(self.h, precisions, 1)
        self.sizes = sdg_query(self.h)
        self.mesh_elem_off = eoff
        return self.sizes

    def set_mesh_sources(self, pos, direction, mesh):
        sdg_set_mesh_sources(self.h, pos, direction, mesh)

    def face_table(self):
        return sdg_face_table(self.h, self.sizes["n_face"])

    def _n(self, key):
        return self.sizes[key]

    def apply(self, v, y, precision=SDG_PREC_F64, stream=None, n_rhs=1):
        n = self._n("n_vel_slab") * n_rhs
        _dev(v, n, "v"), _dev(y, n, "y")
        sdg_apply_velocity_operator(self.h, v, y, n_rhs, precision, stream)

    def apply_adjoint(self, w, y, precision=SDG_PREC_F64, stream=None, n_rhs=1):
        n = self._n("n_vel_slab") * n_rhs
        _dev(w, n, "w"), _dev(y, n, "y")
        sdg_apply_adjoint(self.h, w, y, n_rhs, precision, stream)

    def set_operator_variant(self, variant):
        """0..8 pins a face-kernel variant, -1 reruns the autotuner."""
        sdg_set_operator_variant(self.h, variant)
        self.sizes = sdg_query(self.h)
        return self.sizes

    def set_batched_variant(self, bvariant):
        """0: column grid, 1/2: matrix-core kernel with 8/16 columns per workgroup."""
        _check(lib().sdg_set_batched_variant(self.h, bvariant))
        self.sizes = sdg_query(self.h)
        return self.sizes

    def set_sources(self, pos, direction):
        sdg_set_sources(self.h, pos, direction)

    def apply_preconditioner(self, kind, x, y, n_rhs=1, stream=None):
        n = self._n("n_vel_slab") * n_rhs
        _dev(x, n, "x"), _dev(y, n, "y")
        sdg_apply_preconditioner(self.h, kind, x, y, n_rhs, stream)

    def step(self, v_state, sigma_state, amp=None, n_rhs=1, **kw):
        _dev(v_state, self._n("n_vel_state") * n_rhs, "v_state")
        _dev(sigma_state, self._n("n_stress_state") * n_rhs, "sigma_state")
        if kw.get("v_slab") is not None:
            _dev(kw["v_slab"], self._n("n_vel_slab") * n_rhs, "v_slab")
        if kw.get("sigma_slab") is not None:
            _dev(kw["sigma_slab"], self._n("n_stress_slab") * n_rhs, "sigma_slab")
        return sdg_solve_step(self.h, v_state, sigma_state, amp, n_rhs=n_rhs, **kw)

    def energy(self, v_state, sigma_state, n_rhs=1):
        _dev(v_state, self._n("n_vel_state") * n_rhs, "v_state")
        _dev(sigma_state, self._n("n_stress_state") * n_rhs, "sigma_state")
        n_mesh = len(self.mesh_elem_off) - 1 if getattr(self, "mesh_elem_off", None) is not None else 1
        e = sdg_energy(self.h, v_state, sigma_state, n_rhs, n_out=n_mesh)
        if n_mesh > 1:
            return e
        return float(e[0]) if n_rhs == 1 else e

    def adjoint_step(self, v_old, v_slab, vbar, sigma_bar, grad, opts=None, stream=None):
        _dev(v_old, self._n("n_vel_state"), "v_old")
        _dev(v_slab, self._n("n_vel_slab"), "v_slab")
        _dev(vbar, self._n("n_vel_state"), "vbar")
        _dev(sigma_bar, self._n("n_stress_state"), "sigma_bar")
        _dev(grad, 3 * self._n("n_elem"), "grad")
        return sdg_adjoint_step(self.h, v_old, v_slab, vbar, sigma_bar, grad, opts, stream)

    def projection_points(self, which, extra_degree=0):
        """Rule points and weights of the L2 projection of initial data on
        elements (which = 0) or dual elements (which = 1), with a rule exact
        to the lowest accepted degree plus extra_degree."""
        n = self._n("n_elem") if which == 0 else self._n("n_face")
        deg = self.sizes["proj_min_degree"][which] + extra_degree
        return sdg_projection_points(self.h, which, deg, n, self._n("dim"))

    def project_state(self, velocity_fn, stress_fn, extra_degree=0, stream=None):
        """Projected initial state (v, sigma) as device tensors from point
        functions velocity_fn(x) -> (n, dim) and stress_fn(x) -> (n, n_sigma)
        (Voigt order), evaluated at the library's rule points."""
        import torch
        out = []
        for which, fn, key in ((0, velocity_fn, "n_vel_state"), (1, stress_fn, "n_stress_state")):
            pts, _ = self.projection_points(which, extra_degree)
            vals = np.asarray(fn(pts.reshape(-1, pts.shape[-1])), np.float64)
            del pts
            t = torch.empty(self._n(key), dtype=torch.float64, device=f"cuda:{self.device}")
            deg = self.sizes["proj_min_degree"][which] + extra_degree
            sdg_project_state(self.h, which, deg, vals, t, stream)
            out.append(t)
        return out[0], out[1]

    def sample_adjoint(self, pts, obs_bar, vbar, stream=None):
        pts = np.asarray(pts, np.float64)
        _dev(obs_bar, pts.shape[0] * self._n("dim"), "obs_bar")
        _dev(vbar, self._n("n_vel_state"), "vbar")
        sdg_sample_velocity_adjoint(self.h, pts, obs_bar, vbar, stream=stream)
