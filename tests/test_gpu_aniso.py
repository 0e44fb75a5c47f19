"""General (anisotropic) material on the GPU (Section 2, eq. 1.1): the
library's operator, step, preconditioners and energy with per-element Voigt
stiffness matrices E~, against the oracle with the same E~.

Bars as for the isotropic path: operator 1e-12 relative L2 in FP64 and
2e-6 with FP32 blocks, steps 1e-11, energy 1e-13.  The isotropic E~ of
eq. 5 given to the anisotropic entry point must reproduce the isotropic
entry point's operator to rounding (1e-14): that pins the library's
shear-component convention against the paper's matrix.
"""
import numpy as np
import pytest

import synth
from gpu_cases import rel
from oracle.assemble import Blocks
from oracle.mesh import Topology
from oracle.slab import Slab

pytestmark = pytest.mark.gpu

ACASES = {
    # name: (mesh builder, p, p_gamma, scheme, dt, homogeneous material)
    "a2_stdg_p2": (lambda: synth.split_square(6, jitter=0.15, seed=21), 2, 2, "stdg", 0.01, False),
    "a2_cn_p4": (lambda: synth.split_square(4, periodic=True, jitter=0.1, seed=23), 4, 0, "cn", 0.01, False),
    "a3_cn_p2": (lambda: synth.kuhn_cube(2, periodic=False), 2, 0, "cn", 0.01, False),
    "a3_stdg_p1": (lambda: synth.kuhn_cube(3, periodic=True), 1, 1, "stdg", 0.02, False),
}


def _flags(sdg):
    return (sdg.SDG_PREC_F64 | sdg.SDG_PREC_F32 | sdg.SDG_ASSEMBLE_BLOCK_PRECOND
            | sdg.SDG_ASSEMBLE_PATCH_PRECOND)


def abuild(name):
    import paper_1802_04516_amd as sdg
    mk, p, pg, scheme, dt, homog = ACASES[name]
    mesh = mk()
    Et, rho = synth.anisotropic_material(mesh.n_elem, mesh.dim, sigma=0.2, homogeneous=homog, seed=31)
    ctx = sdg.Context(0)
    sizes = ctx.setup_anisotropic(mesh.xyz, mesh.elem, mesh.period, p, pg,
                                  sdg.SDG_SCHEME_CN if scheme == "cn" else sdg.SDG_SCHEME_STDG, dt, Et, rho,
                                  _flags(sdg))
    B = Blocks(Topology(mesh.xyz, mesh.elem, mesh.period), p, None, None, rho, stiffness=Et)
    return dict(name=name, mesh=mesh, ctx=ctx, sizes=sizes, B=B, slab=Slab(B, pg, dt, scheme), p=p, pg=pg,
                scheme=scheme, dt=dt, Et=Et, rho=rho)


@pytest.fixture(scope="module", params=sorted(ACASES))
def acase(request):
    c = abuild(request.param)
    c["S"] = c["slab"].schur()
    yield c
    c["ctx"].close()


def _gpu(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _apply(ctx, v, prec, n_rhs=1):
    import torch
    vt = _gpu(v)
    yt = torch.empty_like(vt)
    ctx.apply(vt, yt, prec, n_rhs=n_rhs)
    torch.cuda.synchronize()
    return yt.cpu().numpy()


def _canon(B, s_raw):
    return np.stack([B.to_canonical(j, s_raw[j]) for j in range(B.topo.n_face)])


def test_anisotropic_apply_every_variant(acase):
    """Each face kernel that applies the general Hooke law, FP64 and FP32,
    against the oracle's Schur complement; the others are refused."""
    import paper_1802_04516_amd as sdg
    ctx, S = acase["ctx"], acase["S"]
    rng = np.random.default_rng(77)
    v = rng.standard_normal(S.shape[0])
    ref = S @ v
    tried = []
    for var in range(sdg.N_VARIANTS):
        if var not in (3, 4, 8):
            with pytest.raises(sdg.SdgError) as ei:
                ctx.set_operator_variant(var)
            assert ei.value.code == sdg.SDG_EUNSUPPORTED
            continue
        if var == 8 and not (acase["mesh"].dim == 3 and acase["p"] <= 2):
            with pytest.raises(sdg.SdgError):
                ctx.set_operator_variant(var)
            continue
        ctx.set_operator_variant(var)
        e64 = rel(_apply(ctx, v, sdg.SDG_PREC_F64), ref)
        e32 = rel(_apply(ctx, v, sdg.SDG_PREC_F32), ref)
        print(f"{acase['name']} variant {var}: f64 {e64:.2e} f32 {e32:.2e}")
        assert e64 <= 1e-12 and e32 <= 2e-6, (var, e64, e32)
        tried.append(var)
    assert 3 in tried and 4 in tried
    sizes = ctx.set_operator_variant(-1)
    assert sizes["op_variant"] in (3, 4, 8) and sizes["op_variant_f32"] in (3, 4, 8)
    assert all(sizes["tune_us_f64"][v] == 0.0 for v in range(sdg.N_VARIANTS) if v not in (3, 4, 8))


def test_anisotropic_step_matches_oracle(acase):
    """Two steps (CG with Pre1 for CN, GMRES with Pre2 for the space-time
    scheme) from a random state, against the oracle's coupled LU step."""
    import torch
    import paper_1802_04516_amd as sdg
    B, slab, ctx = acase["B"], acase["slab"], acase["ctx"]
    d = acase["mesh"].dim
    rng = np.random.default_rng(5)
    v = rng.standard_normal((B.topo.n_elem, d, B.nphi))
    s = 0.1 * rng.standard_normal((B.topo.n_face, B.nsig, B.npsi))
    vg, sg = _gpu(v), _gpu(_canon(B, s))
    cn = acase["scheme"] == "cn"
    solver = sdg.SDG_SOLVER_CG if cn else sdg.SDG_SOLVER_GMRES
    pc = sdg.SDG_PRECOND_BLOCK if cn else sdg.SDG_PRECOND_PATCH
    for n in range(2):
        o = sdg.SolveOpts(solver, sdg.SDG_PREC_F64, 1e-13, 4000, 30, 5, 10, 1e-5, pc)
        info = ctx.step(vg, sg, None, opts=o)
        _, _, v, s = slab.step(v, s)
        ev, es = rel(vg.cpu().numpy(), v), rel(sg.cpu().numpy(), _canon(B, s))
        print(f"{acase['name']} step {n}: {info['iterations']} its, v {ev:.2e} sigma {es:.2e}")
        assert ev <= 1e-11 and es <= 1e-11
    torch.cuda.synchronize()


def test_anisotropic_fp32_refined_step(acase):
    import paper_1802_04516_amd as sdg
    B, slab, ctx = acase["B"], acase["slab"], acase["ctx"]
    d = acase["mesh"].dim
    rng = np.random.default_rng(9)
    v = rng.standard_normal((B.topo.n_elem, d, B.nphi))
    s = 0.1 * rng.standard_normal((B.topo.n_face, B.nsig, B.npsi))
    vg, sg = _gpu(v), _gpu(_canon(B, s))
    o = sdg.SolveOpts(sdg.SDG_SOLVER_AUTO, sdg.SDG_PREC_F32, 1e-12, 4000, 30, 5, 20, 1e-5, sdg.SDG_PRECOND_MASS)
    ctx.step(vg, sg, None, opts=o)
    _, _, v, s = slab.step(v, s)
    assert rel(vg.cpu().numpy(), v) <= 1e-11 and rel(sg.cpu().numpy(), _canon(B, s)) <= 1e-11


def test_anisotropic_energy(acase):
    """The energy with the general compliance W E~^-1 against the oracle's
    quadrature of sigma : E^-1 sigma; CN conserves it."""
    import paper_1802_04516_amd as sdg
    B, slab, ctx = acase["B"], acase["slab"], acase["ctx"]
    d = acase["mesh"].dim
    rng = np.random.default_rng(3)
    v = rng.standard_normal((B.topo.n_elem, d, B.nphi))
    s = 0.1 * rng.standard_normal((B.topo.n_face, B.nsig, B.npsi))
    vg, sg = _gpu(v), _gpu(_canon(B, s))
    E0 = ctx.energy(vg, sg)
    ref = slab.energy(v, s)
    assert abs(E0 - ref) <= 1e-13 * ref, (E0, ref)
    if acase["scheme"] == "cn":
        o = sdg.SolveOpts(sdg.SDG_SOLVER_CG, sdg.SDG_PREC_F64, 1e-15, 8000, 30, 5, 10, 1e-5, sdg.SDG_PRECOND_BLOCK)
        for _ in range(3):
            ctx.step(vg, sg, None, opts=o)
        assert abs(ctx.energy(vg, sg) - E0) <= 1e-12 * E0


def test_anisotropic_preconditioners_match_oracle():
    """Pre1 and Pre2 built from the general Hooke law (Appendix A)."""
    import torch
    import paper_1802_04516_amd as sdg
    c = abuild("a2_stdg_p2")
    slab = c["slab"]
    slab.schur()
    n = slab.nv
    rng = np.random.default_rng(4)
    x = rng.standard_normal(n)
    for kind, P in ((sdg.SDG_PRECOND_BLOCK, slab.block_jacobi()), (sdg.SDG_PRECOND_PATCH, slab.patch_preconditioner())):
        xg = _gpu(x)
        yg = torch.empty_like(xg)
        c["ctx"].apply_preconditioner(kind, xg, yg)
        torch.cuda.synchronize()
        err = rel(yg.cpu().numpy(), P @ x)
        print(f"precond {kind}: {err:.2e}")
        assert err <= 1e-5
    c["ctx"].close()


@pytest.mark.parametrize("dim", [2, 3])
def test_isotropic_voigt_matrix_equals_lame_entry(dim):
    """E~ of eq. 5 through the anisotropic entry gives the Lame entry's
    operator to rounding, in every anisotropic face kernel."""
    import paper_1802_04516_amd as sdg
    mesh = synth.split_square(5, jitter=0.2, seed=41) if dim == 2 else synth.kuhn_cube(2, periodic=False)
    lam, mu, rho = synth.lognormal_material(mesh.n_elem, sigma=0.3, seed=42)
    ns = dim * (dim + 1) // 2
    Et = np.zeros((mesh.n_elem, ns, ns))
    Et[:, :dim, :dim] = lam[:, None, None]
    for k in range(dim):
        Et[:, k, k] = lam + 2 * mu
    for k in range(dim, ns):
        Et[:, k, k] = 2 * mu
    p = 2
    iso, ani = sdg.Context(0), sdg.Context(0)
    iso.setup(mesh.xyz, mesh.elem, mesh.period, p, 1, sdg.SDG_SCHEME_STDG, 0.01, lam, mu, rho, sdg.SDG_PREC_F64)
    ani.setup_anisotropic(mesh.xyz, mesh.elem, mesh.period, p, 1, sdg.SDG_SCHEME_STDG, 0.01, Et, rho,
                          sdg.SDG_PREC_F64)
    rng = np.random.default_rng(43)
    v = rng.standard_normal(iso.sizes["n_vel_slab"])
    iso.set_operator_variant(4)
    ref = _apply(iso, v, sdg.SDG_PREC_F64)
    for var in ((3, 4, 8) if dim == 3 else (3, 4)):
        ani.set_operator_variant(var)
        err = rel(_apply(ani, v, sdg.SDG_PREC_F64), ref)
        assert err <= 1e-14, (var, err)
    iso.close()
    ani.close()


def test_anisotropic_batched_columns_and_refusals():
    """Batched applies use the column grid (the matrix-core kernel applies
    the isotropic law only and is refused), match single-column applies, and
    the adjoint step is refused; a stiffness that breaks the major symmetry
    or is not positive definite is rejected."""
    import torch
    import paper_1802_04516_amd as sdg
    mesh = synth.kuhn_cube(3, periodic=True)
    Et, rho = synth.anisotropic_material(mesh.n_elem, 3, seed=51)
    ctx = sdg.Context(0)
    ctx.setup_anisotropic(mesh.xyz, mesh.elem, mesh.period, 2, 0, sdg.SDG_SCHEME_CN, 0.01, Et, rho,
                          sdg.SDG_PREC_F64, max_rhs=4)
    with pytest.raises(sdg.SdgError) as ei:
        ctx.set_batched_variant(1)
    assert ei.value.code == sdg.SDG_EUNSUPPORTED
    n = ctx.sizes["n_vel_slab"]
    rng = np.random.default_rng(52)
    V = rng.standard_normal((4, n))
    Y = _apply(ctx, V.ravel(), sdg.SDG_PREC_F64, n_rhs=4).reshape(4, n)
    for k in range(4):
        assert rel(Y[k], _apply(ctx, V[k], sdg.SDG_PREC_F64)) <= 1e-15
    ne, nphi, nsig, npsi, nf = (ctx.sizes[k] for k in ("n_elem", "n_phi", "n_sigma", "n_psi", "n_face"))
    z = lambda m: torch.zeros(m, dtype=torch.float64, device="cuda")
    with pytest.raises(sdg.SdgError) as ei:
        ctx.adjoint_step(z(ne * 3 * nphi), z(n), z(ne * 3 * nphi), z(nf * nsig * npsi), z(3 * ne),
                         opts=sdg.SolveOpts(sdg.SDG_SOLVER_AUTO, sdg.SDG_PREC_F64, 1e-12, 100, 30, 5, 10, 1e-5,
                                            sdg.SDG_PRECOND_MASS))
    assert ei.value.code == sdg.SDG_EUNSUPPORTED
    bad = Et.copy()
    bad[0, 0, 5] += 0.1   # E~ W^-1 no longer symmetric
    with pytest.raises(sdg.SdgError) as ei:
        sdg.sdg_set_material_anisotropic(ctx.h, bad, rho)
    assert ei.value.code == sdg.SDG_EINVAL
    neg = -Et
    sdg.sdg_set_material_anisotropic(ctx.h, neg, rho)
    with pytest.raises(sdg.SdgError) as ei:
        sdg.sdg_assemble(ctx.h, sdg.SDG_PREC_F64)
    assert ei.value.code == sdg.SDG_EINVAL
    ctx.close()
