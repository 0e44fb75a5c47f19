"""Curved boundary elements on the GPU (Section 3: sub-/iso-parametric maps):
a jittered disk whose boundary triangles carry geometry of degree q, free
surface on the curved boundary, against the oracle with the same geometry.

Bars as for straight meshes: operator 1e-12 (FP32 2e-6), step 1e-11,
energy 1e-13, projection 1e-12.
"""
import numpy as np
import pytest

import synth
from gpu_cases import rel
from oracle.assemble import Blocks
from oracle.mesh import Topology
from oracle.slab import Slab
from oracle import waves

pytestmark = pytest.mark.gpu

CCASES = {
    # name: (rings, p, p_gamma, scheme, dt, q)
    "disk_cn_p2q2": (4, 2, 0, "cn", 0.01, 2),
    "disk_stdg_p3q2": (3, 3, 2, "stdg", 0.01, 2),
    "disk_stdg_p2q3": (3, 2, 1, "stdg", 0.02, 3),
}


def cbuild(name):
    import paper_1802_04516_amd as sdg
    n, p, pg, scheme, dt, q = CCASES[name]
    m = synth.disk_mesh(n, q=q, jitter=0.15, seed=51)
    lam, mu, rho = synth.lognormal_material(m.n_elem, sigma=0.2, seed=52)
    ctx = sdg.Context(0)
    sizes = ctx.setup_curved(m.xyz, m.elem, m.meta["curved"], p, pg,
                             sdg.SDG_SCHEME_CN if scheme == "cn" else sdg.SDG_SCHEME_STDG, dt, lam, mu, rho,
                             sdg.SDG_PREC_F64 | sdg.SDG_PREC_F32 | sdg.SDG_ASSEMBLE_BLOCK_PRECOND
                             | sdg.SDG_ASSEMBLE_PATCH_PRECOND)
    B = Blocks(Topology(m.xyz, m.elem, None), p, lam, mu, rho, curved=m.meta["curved"])
    return dict(name=name, mesh=m, ctx=ctx, sizes=sizes, B=B, slab=Slab(B, pg, dt, scheme), p=p, pg=pg,
                scheme=scheme, dt=dt)


@pytest.fixture(scope="module", params=sorted(CCASES))
def ccase(request):
    c = cbuild(request.param)
    c["S"] = c["slab"].schur()
    yield c
    c["ctx"].close()


def _gpu(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _canon(B, s_raw):
    return np.stack([B.to_canonical(j, s_raw[j]) for j in range(B.topo.n_face)])


def test_curved_apply_every_variant(ccase):
    import torch
    import paper_1802_04516_amd as sdg
    ctx, S = ccase["ctx"], ccase["S"]
    v = np.random.default_rng(61).standard_normal(S.shape[0])
    ref = S @ v
    for var in range(sdg.N_VARIANTS):
        if var == 8:
            continue  # the compressed operator is 3D
        ctx.set_operator_variant(var)
        for prec, bar in ((sdg.SDG_PREC_F64, 1e-12), (sdg.SDG_PREC_F32, 2e-6)):
            vt = _gpu(v)
            yt = torch.empty_like(vt)
            ctx.apply(vt, yt, prec)
            torch.cuda.synchronize()
            err = rel(yt.cpu().numpy(), ref)
            assert err <= bar, (var, prec, err)
    ctx.set_operator_variant(-1)


def test_curved_steps_match_oracle(ccase):
    """Two steps with each preconditioner the scheme takes, from a random
    state, against the oracle's coupled LU step."""
    import torch
    import paper_1802_04516_amd as sdg
    B, slab, ctx = ccase["B"], ccase["slab"], ccase["ctx"]
    cn = ccase["scheme"] == "cn"
    pcs = [sdg.SDG_PRECOND_MASS, sdg.SDG_PRECOND_BLOCK] + ([] if cn else [sdg.SDG_PRECOND_PATCH])
    for pc in pcs:
        rng = np.random.default_rng(7)
        v = rng.standard_normal((B.topo.n_elem, 2, B.nphi))
        s = 0.1 * rng.standard_normal((B.topo.n_face, 3, B.npsi))
        vg, sg = _gpu(v), _gpu(_canon(B, s))
        for n in range(2):
            o = sdg.SolveOpts(sdg.SDG_SOLVER_AUTO, sdg.SDG_PREC_F64, 1e-13, 4000, 30, 5, 10, 1e-5, pc)
            info = ctx.step(vg, sg, None, opts=o)
            _, _, v, s = slab.step(v, s)
            ev, es = rel(vg.cpu().numpy(), v), rel(sg.cpu().numpy(), _canon(B, s))
            print(f"{ccase['name']} precond {pc} step {n}: {info['iterations']} its, v {ev:.2e} sigma {es:.2e}")
            assert ev <= 1e-11 and es <= 1e-11
        torch.cuda.synchronize()
    # FP32 operator inside FP64 refinement
    rng = np.random.default_rng(8)
    v = rng.standard_normal((B.topo.n_elem, 2, B.nphi))
    s = 0.1 * rng.standard_normal((B.topo.n_face, 3, B.npsi))
    vg, sg = _gpu(v), _gpu(_canon(B, s))
    o = sdg.SolveOpts(sdg.SDG_SOLVER_AUTO, sdg.SDG_PREC_F32, 1e-12, 4000, 30, 5, 20, 1e-5, sdg.SDG_PRECOND_BLOCK)
    ctx.step(vg, sg, None, opts=o)
    _, _, v, s = slab.step(v, s)
    assert rel(vg.cpu().numpy(), v) <= 1e-11 and rel(sg.cpu().numpy(), _canon(B, s)) <= 1e-11


def test_curved_energy(ccase):
    import paper_1802_04516_amd as sdg
    B, slab, ctx = ccase["B"], ccase["slab"], ccase["ctx"]
    rng = np.random.default_rng(3)
    v = rng.standard_normal((B.topo.n_elem, 2, B.nphi))
    s = 0.1 * rng.standard_normal((B.topo.n_face, 3, B.npsi))
    vg, sg = _gpu(v), _gpu(_canon(B, s))
    E0 = ctx.energy(vg, sg)
    ref = slab.energy(v, s)
    assert abs(E0 - ref) <= 1e-13 * ref, (E0, ref)
    if ccase["scheme"] == "cn":
        o = sdg.SolveOpts(sdg.SDG_SOLVER_CG, sdg.SDG_PREC_F64, 1e-15, 8000, 30, 5, 10, 1e-5, sdg.SDG_PRECOND_BLOCK)
        for _ in range(3):
            ctx.step(vg, sg, None, opts=o)
        assert abs(ctx.energy(vg, sg) - E0) <= 1e-12 * E0


class _Linear:
    """A linear plane-wave-like field (data only): velocity and Voigt
    stress linear in x, exact in every discrete space of degree >= 1."""

    def velocity(self, x, t):
        x = np.atleast_2d(x)
        return np.stack([0.3 + 0.5 * x[:, 0] - 0.2 * x[:, 1], -0.1 + 0.4 * x[:, 1]], axis=1)

    def stress_voigt(self, x, t):
        x = np.atleast_2d(x)
        return np.stack([1.0 + x[:, 0], 0.5 - x[:, 1], 0.2 * x[:, 0] + 0.3 * x[:, 1]], axis=1)


def test_curved_projection_matches_oracle(ccase):
    """L2 projection of initial data on the curved mesh against the oracle's
    (linear data: both projections are exact to rounding)."""
    B, ctx = ccase["B"], ccase["ctx"]
    w = _Linear()
    vg, sg = ctx.project_state(lambda x: w.velocity(x, 0.0), lambda x: w.stress_voigt(x, 0.0))
    v, s = waves.project(B, w, 0.0, extra_degree=2)
    assert rel(vg.cpu().numpy(), v) <= 1e-12
    assert rel(sg.cpu().numpy(), _canon(B, s)) <= 1e-12


def test_curved_source_and_sampling():
    """A point source inside a curved boundary element and sampling there
    (points located by Newton on the element map)."""
    import torch
    import paper_1802_04516_amd as sdg
    c = cbuild("disk_stdg_p3q2")
    B, slab, ctx = c["B"], c["slab"], c["ctx"]
    ids = c["mesh"].meta["curved"][0]
    e = int(ids[3])
    pos = B.maps[e].x(np.array([[0.2, 0.1]]))[0]           # a point near the curved edge
    assert B.locate(pos) == e
    ctx.set_sources(pos[None, :], np.array([[0.0, 1.0]]))
    v = np.zeros((B.topo.n_elem, 2, B.nphi))
    s = np.zeros((B.topo.n_face, 3, B.npsi))
    vg, sg = _gpu(v), _gpu(_canon(B, s))
    amp = np.array([[1.0, -0.5, 0.25]])
    o = sdg.SolveOpts(sdg.SDG_SOLVER_AUTO, sdg.SDG_PREC_F64, 1e-13, 4000, 30, 5, 10, 1e-5, sdg.SDG_PRECOND_BLOCK)
    ctx.step(vg, sg, amp.ravel(), opts=o)
    src = dict(pos=pos[None, :], dir=np.array([[0.0, 1.0]]), amp=amp)
    _, _, v1, s1 = slab.step(v, s, src)
    assert rel(vg.cpu().numpy(), v1) <= 1e-11
    pts = np.vstack([pos, B.maps[e].x(np.array([[0.05, 0.9]]))[0]])
    out = torch.empty(pts.shape[0] * 2, dtype=torch.float64, device="cuda")
    sdg.sdg_sample_velocity(ctx.h, vg, pts, out)
    torch.cuda.synchronize()
    ref = np.stack([B.velocity_at(v1[B.locate(x)], B.locate(x), x[None, :])[0] for x in pts])
    assert np.allclose(out.cpu().numpy().reshape(ref.shape), ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())
    ctx.close()


def test_curved_refusals():
    """3D, periodic meshes and mesh batches take no curved elements; a
    curved face shared with another element is rejected; the adjoint step
    refuses a curved mesh."""
    import torch
    import paper_1802_04516_amd as sdg
    m = synth.disk_mesh(3, q=2)
    ids, nodes = m.meta["curved"]
    ctx = sdg.Context(0)
    k3 = synth.kuhn_cube(2, periodic=False)
    sdg.sdg_set_mesh(ctx.h, k3.xyz, k3.elem, None)
    with pytest.raises(sdg.SdgError) as ei:
        sdg.sdg_set_curved_elements(ctx.h, ids[:1], nodes[:1])
    assert ei.value.code == sdg.SDG_EUNSUPPORTED
    sq = synth.split_square(3, periodic=True)
    sdg.sdg_set_mesh(ctx.h, sq.xyz, sq.elem, sq.period)
    with pytest.raises(sdg.SdgError) as ei:
        sdg.sdg_set_curved_elements(ctx.h, ids[:1], nodes[:1])
    assert ei.value.code == sdg.SDG_EUNSUPPORTED
    # bend an interior face: move the node of an interior edge
    bad = nodes.copy()
    e0 = int(ids[0])
    tri = m.elem[e0]
    ring_out = [np.hypot(*m.xyz[v]) > 0.999 for v in tri]
    # node 4 of degree 2 lies on edge (1, 2), node 3 on edge (2, 0), node 1 on edge (0, 1)
    interior_node = {(1, 2): 4, (0, 2): 3, (0, 1): 1}
    for (a, b), k in interior_node.items():
        if not (ring_out[a] and ring_out[b]):
            bad[0, k] += 0.01
            break
    lam, mu, rho = synth.homogeneous_material(m.n_elem)
    sdg.sdg_set_mesh(ctx.h, m.xyz, m.elem, None)
    sdg.sdg_set_curved_elements(ctx.h, ids, bad)
    sdg.sdg_set_discretization(ctx.h, 2, 0, sdg.SDG_SCHEME_CN, 0.01)
    sdg.sdg_set_material(ctx.h, lam, mu, rho)
    with pytest.raises(sdg.SdgError) as ei:
        sdg.sdg_assemble(ctx.h, sdg.SDG_PREC_F64)
    assert ei.value.code == sdg.SDG_EMESH
    ctx.close()
    c = cbuild("disk_cn_p2q2")
    sz = c["sizes"]
    z = lambda n: torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(sdg.SdgError) as ei:
        c["ctx"].adjoint_step(z(sz["n_vel_state"]), z(sz["n_vel_slab"]), z(sz["n_vel_state"]),
                              z(sz["n_stress_state"]), z(3 * sz["n_elem"]))
    assert ei.value.code == sdg.SDG_EUNSUPPORTED
    c["ctx"].close()
