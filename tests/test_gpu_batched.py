"""Batched right-hand sides and mesh batches: several independent systems
solved in shared launches, each held to the single-system oracle bar.

Batched columns: column r of a batched step carries source r % n_src and its
own old state; each column is compared with the oracle's step of that
column alone (<= 1e-11 relative L2, Krylov rtol 1e-13), and the batched
operator apply with the single-column apply (bit for bit: the same kernels
on offset pointers) and with the oracle's Schur complement.

Mesh batches: ragged meshes concatenated by the library, one Krylov process
per mesh; each mesh's part of the state is compared with the oracle on that
mesh alone.
"""
import numpy as np
import pytest

import synth
from gpu_cases import material, rel
from oracle.assemble import Blocks
from oracle.mesh import Topology
from oracle.slab import Slab

pytestmark = pytest.mark.gpu


def _gpu(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _poison_freed_device_memory(nbytes=1 << 30):
    """Leave NaN bit patterns in device memory handed back to the driver, so
    that the library's next workspace allocations are likely to start from
    NaN: a solver that reads workspace values it never wrote (say a zero
    coefficient times a stale basis vector) then returns NaN."""
    import torch
    t = torch.full((nbytes // 8,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    del t
    torch.cuda.empty_cache()


def _canon(B, s_raw):
    return np.stack([B.to_canonical(j, s_raw[j]) for j in range(B.topo.n_face)])


def _opts(rtol=1e-13, precision=None, precond=None, max_iter=3000):
    import paper_1802_04516_amd as sdg
    return sdg.SolveOpts(sdg.SDG_SOLVER_AUTO, precision or sdg.SDG_PREC_F64, rtol, max_iter, 30, 5, 20, 1e-5,
                         sdg.SDG_PRECOND_MASS if precond is None else precond)


def _amps(slab, scheme, dt, n, n_src, scale):
    t = np.array([(n + 0.5) * dt]) if scheme == "cn" else n * dt + slab.tb.tau * dt
    return np.stack([scale[s] * synth.ricker(t, 10.0, 0.02) for s in range(n_src)])


BATCH_CASES = {
    # name: (mesh, p, p_gamma, scheme, dt, material, columns, preconditioner)
    "stdg_p3pg3": (lambda: synth.split_square(6, jitter=0.2, seed=2001), 3, 3, "stdg", 2.5e-3, "layered", 5, "block"),
    "stdg_p2pg1": (lambda: synth.split_square(5, jitter=0.1, seed=9), 2, 1, "stdg", 0.01, "lognormal", 3, "mass"),
    "cn_p2": (lambda: synth.split_square(5, periodic=True, jitter=0.1, seed=4), 2, 0, "cn", 0.01, "lognormal", 4,
              "mass"),
}


@pytest.fixture(scope="module", params=sorted(BATCH_CASES))
def bcase(request):
    import paper_1802_04516_amd as sdg
    mk, p, pg, scheme, dt, matkind, R, pc = BATCH_CASES[request.param]
    mesh = mk()
    lam, mu, rho = material(matkind, mesh)
    ctx = sdg.Context(0)
    sizes = ctx.setup(mesh.xyz, mesh.elem, mesh.period, p, pg,
                      sdg.SDG_SCHEME_CN if scheme == "cn" else sdg.SDG_SCHEME_STDG, dt, lam, mu, rho,
                      sdg.SDG_PREC_F64 | sdg.SDG_PREC_F32 | sdg.SDG_ASSEMBLE_BLOCK_PRECOND, max_rhs=R)
    B = Blocks(Topology(mesh.xyz, mesh.elem, mesh.period), p, lam, mu, rho)
    slab = Slab(B, pg, dt, scheme)
    yield dict(name=request.param, mesh=mesh, ctx=ctx, sizes=sizes, B=B, slab=slab, scheme=scheme, dt=dt, R=R,
               precond=sdg.SDG_PRECOND_BLOCK if pc == "block" else sdg.SDG_PRECOND_MASS)
    ctx.close()


@pytest.mark.parametrize("bvariant", [0, 1, 2])
def test_batched_apply_matches_columns_and_oracle(bcase, bvariant):
    """Batched applies against the single-column apply and the oracle's
    Schur complement.  The column grid (bvariant 0) runs the single-column
    kernels on offset pointers and is equal bit for bit; the matrix-core
    kernel (1, 2) sums in another order: FP64 within 1e-13 of the single
    apply, FP32 (v_mfma_f32_16x16x4, FP32 face slots) within 1e-6 of it,
    and both within the usual bars of the oracle."""
    import torch
    import paper_1802_04516_amd as sdg
    ctx, R, n = bcase["ctx"], bcase["R"], bcase["sizes"]["n_vel_slab"]
    S = bcase["slab"].schur()
    rng = np.random.default_rng(77)
    V = rng.standard_normal((R, n))
    old = ctx.sizes["op_bvariant"]
    ctx.set_batched_variant(bvariant)
    try:
        for prec, tol in ((sdg.SDG_PREC_F64, 1e-12), (sdg.SDG_PREC_F32, 2e-6)):
            vb, yb = _gpu(V), torch.empty(R * n, dtype=torch.float64, device="cuda")
            ctx.apply(vb, yb, prec, n_rhs=R)
            ys = torch.empty(n, dtype=torch.float64, device="cuda")
            for r in range(R):
                ctx.apply(_gpu(V[r]), ys, prec)
                col = yb[r * n:(r + 1) * n]
                if bvariant == 0:
                    assert torch.equal(ys, col), f"column {r} differs from the single apply"
                else:
                    assert rel(col.cpu().numpy(), ys.cpu().numpy()) <= (1e-6 if prec == sdg.SDG_PREC_F32 else 1e-13)
                assert rel(col.cpu().numpy(), S @ V[r]) <= tol
        yt = torch.empty(R * n, dtype=torch.float64, device="cuda")
        ctx.apply_adjoint(_gpu(V), yt, n_rhs=R)
        for r in range(R):
            assert rel(yt[r * n:(r + 1) * n].cpu().numpy(), S.T @ V[r]) <= 1e-12
        # a partial last tile: fewer columns than the workgroup width
        if R > 1:
            for prec, tol in ((sdg.SDG_PREC_F64, 1e-12), (sdg.SDG_PREC_F32, 2e-6)):
                vb, yb = _gpu(V[:R - 1]), torch.empty((R - 1) * n, dtype=torch.float64, device="cuda")
                ctx.apply(vb, yb, prec, n_rhs=R - 1)
                for r in range(R - 1):
                    assert rel(yb[r * n:(r + 1) * n].cpu().numpy(), S @ V[r]) <= tol
    finally:
        ctx.set_batched_variant(old)


@pytest.mark.parametrize("variant", [3, 6])
def test_column_grid_with_persistent_and_lane_reduced_face_kernels(bcase, variant):
    """The column grid (grid y = column) of the persistent face kernel
    (variant 3, whose x grid walks chunks) and of the lane-reduced one
    (variant 6) gives every column bit for bit its single-column apply."""
    import torch
    import paper_1802_04516_amd as sdg
    ctx, R, n = bcase["ctx"], bcase["R"], bcase["sizes"]["n_vel_slab"]
    V = np.random.default_rng(78).standard_normal((R, n))
    old = ctx.sizes["op_bvariant"]
    ctx.set_batched_variant(0)
    ctx.set_operator_variant(variant)
    try:
        for prec in (sdg.SDG_PREC_F64, sdg.SDG_PREC_F32):
            yb = torch.empty(R * n, dtype=torch.float64, device="cuda")
            ctx.apply(_gpu(V), yb, prec, n_rhs=R)
            ys = torch.empty(n, dtype=torch.float64, device="cuda")
            for r in range(R):
                ctx.apply(_gpu(V[r]), ys, prec)
                assert torch.equal(ys, yb[r * n:(r + 1) * n]), f"column {r} differs from the single apply"
    finally:
        ctx.set_operator_variant(-1)
        ctx.set_batched_variant(old)


@pytest.mark.parametrize("precision", ["f64", "f32ir", "f64_cgs2"])
def test_batched_steps_match_oracle_per_column(bcase, precision):
    """Batched columns against the oracle column by column; f64_cgs2 runs the
    multi-system GMRES with both Gram-Schmidt projections within the step
    (SDG_SOLVE_CGS2) instead of the default delayed one."""
    import paper_1802_04516_amd as sdg
    ctx, R, B, slab = bcase["ctx"], bcase["R"], bcase["B"], bcase["slab"]
    ne, nf = B.topo.n_elem, B.topo.n_face
    rng = np.random.default_rng(5 + R)
    n_src = 2
    pos = np.array([[0.31, 0.42], [0.67, 0.58]])
    dirs = np.array([[0.0, 1.0], [0.6, 0.8]])
    ctx.set_sources(pos, dirs)
    scale = np.array([1.0, -0.7])
    # column states: random for r < R-1, the last column starts at rest
    v0 = [0.3 * rng.standard_normal((ne, 2, B.nphi)) for _ in range(R - 1)] + [np.zeros((ne, 2, B.nphi))]
    s0 = [0.1 * rng.standard_normal((nf, 3, B.npsi)) for _ in range(R - 1)] + [np.zeros((nf, 3, B.npsi))]
    vg = _gpu(np.stack(v0))
    sg = _gpu(np.stack([_canon(B, s) for s in s0]))
    prec = sdg.SDG_PREC_F32 if precision == "f32ir" else sdg.SDG_PREC_F64
    vo, so = [v.copy() for v in v0], [s.copy() for s in s0]
    for n in range(3):
        amps = _amps(slab, bcase["scheme"], bcase["dt"], n, n_src, scale)
        o = _opts(precision=prec, precond=bcase["precond"])
        if precision == "f64_cgs2":
            o.flags = sdg.SDG_SOLVE_CGS2
        info = ctx.step(vg, sg, amps.ravel(), n_rhs=R, opts=o)
        V = vg.cpu().numpy().reshape(R, -1)
        Sg = sg.cpu().numpy().reshape(R, -1)
        worst = 0.0
        for r in range(R):
            src = dict(pos=pos[r % n_src:r % n_src + 1], dir=dirs[r % n_src:r % n_src + 1],
                       amp=amps[r % n_src:r % n_src + 1])
            _, _, vo[r], so[r] = slab.step(vo[r], so[r], src)
            worst = max(worst, rel(V[r], vo[r]), rel(Sg[r], _canon(B, so[r])))
        print(f"{bcase['name']} {precision} step {n}: worst column err {worst:.2e} iters {info['iterations']} "
              f"refinements {info['refinements']} rel res {info['rel_residual']:.2e}")
        assert worst <= 1e-11


def test_batched_energy_and_limits(bcase):
    import torch
    import paper_1802_04516_amd as sdg
    ctx, R, B = bcase["ctx"], bcase["R"], bcase["B"]
    rng = np.random.default_rng(3)
    ne, nf = B.topo.n_elem, B.topo.n_face
    v = rng.standard_normal((R, ne, 2, B.nphi))
    s = rng.standard_normal((R, nf, 3, B.npsi))
    e = ctx.energy(_gpu(v), _gpu(s), n_rhs=R)
    for r in range(R):
        e1 = ctx.energy(_gpu(v[r]), _gpu(s[r]))
        assert e[r] == e1
    n = bcase["sizes"]["n_vel_slab"]
    L = sdg.lib()
    x = torch.zeros((R + 1) * n, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    rc = L.sdg_apply_velocity_operator(ctx.h, sdg._dev(x), sdg._dev(y), R + 1, sdg.SDG_PREC_F64, None)
    assert rc == sdg.SDG_EINVAL


MESH_BATCH = [
    # ragged sizes: 18, 50, 32 triangles
    (lambda: synth.split_square(3, jitter=0.1, seed=41), 0.02),
    (lambda: synth.split_square(5, jitter=0.2, seed=42), 0.01),
    (lambda: synth.split_square(4, seed=43), 0.0),
]


@pytest.mark.parametrize("scheme,p,pg,precision", [("stdg", 2, 2, "f64"), ("stdg", 3, 1, "f32ir"),
                                                    ("cn", 2, 0, "f64")])
def test_mesh_batch_step_matches_oracle_per_mesh(scheme, p, pg, precision):
    import paper_1802_04516_amd as sdg
    meshes = [mk() for mk, _ in MESH_BATCH]
    mats = [synth.lognormal_material(m.n_elem, sigma=0.2, seed=100 + q) for q, m in enumerate(meshes)]
    lam, mu, rho = (np.concatenate([mt[i] for mt in mats]) for i in range(3))
    dt = 0.01
    ctx = sdg.Context(0)
    sizes = ctx.setup_batch([(m.xyz, m.elem) for m in meshes], p, pg,
                            sdg.SDG_SCHEME_CN if scheme == "cn" else sdg.SDG_SCHEME_STDG, dt, lam, mu, rho,
                            sdg.SDG_PREC_F64 | sdg.SDG_PREC_F32 | sdg.SDG_ASSEMBLE_BLOCK_PRECOND)
    slabs = [Slab(Blocks(Topology(m.xyz, m.elem, None), p, *mt), pg, dt, scheme) for m, mt in zip(meshes, mats)]
    # faces of the concatenated mesh are contiguous per mesh, in each mesh's own order
    left = ctx.face_table()[0]
    eoff = ctx.mesh_elem_off
    foff = np.searchsorted(left, eoff)
    for q, S in enumerate(slabs):
        assert foff[q + 1] - foff[q] == S.nf
    pos = np.array([[0.37, 0.61], [0.52, 0.44], [0.7, 0.3]])
    dirs = np.array([[0.0, 1.0], [1.0, 0.0], [0.6, 0.8]])
    scale = np.array([1.0, 0.5, -0.8])
    ctx.set_mesh_sources(pos, dirs, np.arange(3, dtype=np.int32))
    rng = np.random.default_rng(8)
    v0 = [0.2 * rng.standard_normal((m.n_elem, 2, S.nphi)) * (q != 2) for q, (m, S) in enumerate(zip(meshes, slabs))]
    s0 = [np.zeros((S.nf, 3, S.npsi)) for S in slabs]
    vg = _gpu(np.concatenate([v.ravel() for v in v0]))
    sg = _gpu(np.concatenate([np.stack([S.B.to_canonical(j, s[j]) for j in range(S.nf)]).ravel()
                              for S, s in zip(slabs, s0)]))
    prec = sdg.SDG_PREC_F64 if precision == "f64" else sdg.SDG_PREC_F32
    ng = pg + 1
    vo, so = [v.copy() for v in v0], [s.copy() for s in s0]
    nvs = 2 * slabs[0].nphi
    nss = 3 * slabs[0].npsi
    for n in range(3):
        amps = _amps(slabs[0], scheme, dt, n, 3, scale)
        info = ctx.step(vg, sg, amps.ravel(), opts=_opts(precision=prec, precond=sdg.SDG_PRECOND_BLOCK))
        V = vg.cpu().numpy()
        Sg = sg.cpu().numpy()
        worst = 0.0
        for q, S in enumerate(slabs):
            src = dict(pos=pos[q:q + 1], dir=dirs[q:q + 1], amp=amps[q:q + 1])
            _, _, vo[q], so[q] = S.step(vo[q], so[q], src)
            vq = V[eoff[q] * nvs:eoff[q + 1] * nvs]
            sq = Sg[foff[q] * nss:foff[q + 1] * nss]
            worst = max(worst, rel(vq, vo[q]), rel(sq, np.stack([S.B.to_canonical(j, so[q][j]) for j in range(S.nf)])))
        print(f"mesh batch {scheme} p={p} pg={pg} {precision} step {n}: worst mesh err {worst:.2e} "
              f"iters {info['iterations']} rel res {info['rel_residual']:.2e}")
        assert worst <= 1e-11
    assert sizes["n_elem"] == sum(m.n_elem for m in meshes)
    # energy of the batch: one value per mesh (Section 5.2)
    e = ctx.energy(vg, sg)
    assert len(e) == len(meshes)
    for q, S in enumerate(slabs):
        eo = S.energy(vo[q], so[q])
        assert abs(e[q] - eo) <= 1e-11 * abs(eo), (q, e[q], eo)
    ctx.close()


GRAPH_CASES = {
    # name: (meshes, p, p_gamma, scheme, columns)
    "mesh_batch_stdg": ([m for m, _ in MESH_BATCH], 2, 2, "stdg", 1),
    "single_stdg_p3": ([lambda: synth.split_square(6, jitter=0.2, seed=2001)], 3, 3, "stdg", 1),
    "batched_cn": ([lambda: synth.split_square(5, jitter=0.1, seed=4)], 2, 0, "cn", 3),
}


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32_ir"])
@pytest.mark.parametrize("name", sorted(GRAPH_CASES))
def test_graph_replays_match_eager_steps_and_oracle(name, fp32):
    """The step recorded in HIP graphs is replayed for several steps with
    other work and synchronisations in between; every replayed step is
    checked against the same step run eagerly and against the oracle.  With
    fp32_ir both run the FP32 operator inside FP64 refinement, the graph
    with its per-system outer tests on the device.  The context is created
    after NaN has been left in freed device memory, and every result must be
    finite: a system that converges within a recorded part of a cycle must
    not pick up basis vectors it never wrote."""
    import torch
    import paper_1802_04516_amd as sdg
    mks, p, pg, scheme, R = GRAPH_CASES[name]
    meshes = [mk() for mk in mks]
    mats = [synth.lognormal_material(m.n_elem, sigma=0.2, seed=200 + q) for q, m in enumerate(meshes)]
    lam, mu, rho = (np.concatenate([mt[i] for mt in mats]) for i in range(3))
    dt = 0.01
    sch = sdg.SDG_SCHEME_CN if scheme == "cn" else sdg.SDG_SCHEME_STDG
    prc = sdg.SDG_PREC_F64 | sdg.SDG_ASSEMBLE_BLOCK_PRECOND | (sdg.SDG_PREC_F32 if fp32 else 0)
    _poison_freed_device_memory()
    ctx = sdg.Context(0)
    if len(meshes) > 1:
        ctx.setup_batch([(m.xyz, m.elem) for m in meshes], p, pg, sch, dt, lam, mu, rho, prc)
        ctx.set_mesh_sources(np.array([[0.37, 0.61], [0.52, 0.44], [0.7, 0.3]]), np.array([[0.0, 1.0]] * 3),
                             np.arange(3, dtype=np.int32))
        n_src = 3
    else:
        ctx.setup(meshes[0].xyz, meshes[0].elem, None, p, pg, sch, dt, lam, mu, rho, prc, max_rhs=R)
        ctx.set_sources(np.array([[0.41, 0.57], [0.6, 0.35], [0.25, 0.3]][:R]), np.array([[0.0, 1.0]] * R))
        n_src = R
    slabs = [Slab(Blocks(Topology(m.xyz, m.elem, None), p, *mt), pg, dt, scheme) for m, mt in zip(meshes, mats)]
    sz = ctx.sizes
    rng = np.random.default_rng(13)
    v0 = 0.2 * rng.standard_normal(sz["n_vel_state"] * R)
    s0 = np.zeros(sz["n_stress_state"] * R)
    vg, sg = _gpu(v0), _gpu(s0)          # graph-mode state
    ve, se = _gpu(v0), _gpu(s0)          # eager state
    pr = sdg.SDG_PREC_F32 if fp32 else sdg.SDG_PREC_F64
    opts_g = _opts(precision=pr, precond=sdg.SDG_PRECOND_BLOCK)
    opts_g.flags = sdg.SDG_SOLVE_GRAPH
    opts_e = _opts(precision=pr, precond=sdg.SDG_PRECOND_BLOCK)
    scratch_v = torch.randn(sz["n_vel_slab"], dtype=torch.float64, device="cuda")
    scratch_y = torch.empty_like(scratch_v)
    for n in range(4):
        amps = _amps(slabs[0], scheme, dt, n, n_src, np.linspace(1.0, -0.5, n_src))
        # the eager step starts from the graph path's state so both see the same input
        ve.copy_(vg)
        se.copy_(sg)
        vin = vg.cpu().numpy()
        sin = sg.cpu().numpy()
        info_g = ctx.step(vg, sg, amps.ravel(), n_rhs=R, opts=opts_g)
        ctx.apply(scratch_v, scratch_y)          # eager work between replays
        torch.cuda.synchronize()
        info_e = ctx.step(ve, se, amps.ravel(), n_rhs=R, opts=opts_e)
        d_ge = max(rel(vg.cpu().numpy(), ve.cpu().numpy()), rel(sg.cpu().numpy(), se.cpu().numpy()))
        # oracle, per mesh / column, from the same input
        worst = 0.0
        if len(meshes) > 1:
            nvs, nss = 2 * slabs[0].nphi, 3 * slabs[0].npsi
            eoff = ctx.mesh_elem_off
            left = ctx.face_table()[0]
            foff = np.searchsorted(left, eoff)
            for q, S in enumerate(slabs):
                vq = vin[eoff[q] * nvs:eoff[q + 1] * nvs].reshape(S.ne, S.d, S.nphi)
                sq = sin[foff[q] * nss:foff[q + 1] * nss].reshape(S.nf, S.nsig, S.npsi)
                sraw = np.stack([S.B.from_canonical(j, sq[j]) for j in range(S.nf)])
                src = dict(pos=np.array([[0.37, 0.61], [0.52, 0.44], [0.7, 0.3]])[q:q + 1],
                           dir=np.array([[0.0, 1.0]]), amp=amps[q:q + 1])
                _, _, v1, s1 = S.step(vq, sraw, src)
                worst = max(worst, rel(vg.cpu().numpy()[eoff[q] * nvs:eoff[q + 1] * nvs], v1),
                            rel(sg.cpu().numpy()[foff[q] * nss:foff[q + 1] * nss],
                                np.stack([S.B.to_canonical(j, s1[j]) for j in range(S.nf)])))
        else:
            S = slabs[0]
            pos = np.array([[0.41, 0.57], [0.6, 0.35], [0.25, 0.3]])
            for r in range(R):
                vq = vin.reshape(R, -1)[r].reshape(S.ne, S.d, S.nphi)
                sq = sin.reshape(R, -1)[r].reshape(S.nf, S.nsig, S.npsi)
                sraw = np.stack([S.B.from_canonical(j, sq[j]) for j in range(S.nf)])
                src = dict(pos=pos[r:r + 1], dir=np.array([[0.0, 1.0]]), amp=amps[r:r + 1])
                _, _, v1, s1 = S.step(vq, sraw, src)
                worst = max(worst, rel(vg.cpu().numpy().reshape(R, -1)[r], v1),
                            rel(sg.cpu().numpy().reshape(R, -1)[r],
                                np.stack([S.B.to_canonical(j, s1[j]) for j in range(S.nf)])))
        print(f"{name} {'fp32_ir' if fp32 else 'fp64'} step {n}: graph vs eager {d_ge:.2e}, vs oracle "
              f"{worst:.2e}, iters graph {info_g['iterations']} eager {info_e['iterations']}, refinements "
              f"graph {info_g['refinements']} eager {info_e['refinements']}")
        assert np.isfinite(vg.cpu().numpy()).all() and np.isfinite(sg.cpu().numpy()).all()
        assert d_ge <= 1e-11 and worst <= 1e-11
        assert info_g["rel_residual"] <= 1e-13
    ctx.close()
