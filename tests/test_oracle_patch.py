"""The patch rows used by the full-size GPU parity tests equal the rows of
the whole-mesh oracle (locality of the velocity Schur complement: the
stress mass of eq. MD_2 is block diagonal over the faces)."""
import numpy as np
import pytest

import synth
from oracle.assemble import Blocks
from oracle.mesh import Topology
from oracle.slab import Slab
from patch import Patch, face_codes

MESHES = {
    # free surface with jitter at the full-size 2D degrees; periodic 3D (seam faces)
    "2d_free_p3pg3": (lambda: synth.split_square(4, jitter=0.2, seed=2001), 3, 3, 2.5e-3, "stdg", "layered"),
    "3d_periodic_cn_p2": (lambda: synth.kuhn_cube(3, periodic=True), 2, 0, 0.01, "cn", "lognormal"),
    "2d_periodic_cn_p1": (lambda: synth.split_square(4, periodic=True, jitter=0.1, seed=5), 1, 0, 0.01, "cn",
                          "lognormal"),
}


def _material(kind, mesh):
    if kind == "layered":
        return synth.layered_material(mesh.centroids(), sigma=0.1, seed=2002)
    return synth.lognormal_material(mesh.n_elem, sigma=0.2, seed=17)


@pytest.fixture(scope="module", params=sorted(MESHES))
def whole(request):
    mk, p, pg, dt, scheme, mat = MESHES[request.param]
    mesh = mk()
    lam, mu, rho = _material(mat, mesh)
    topo = Topology(mesh.xyz, mesh.elem, mesh.period)
    B = Blocks(topo, p, lam, mu, rho)
    slab = Slab(B, pg, dt, scheme)
    return dict(mesh=mesh, p=p, pg=pg, dt=dt, scheme=scheme, mat=(lam, mu, rho), B=B, slab=slab,
                S=slab.schur())


def _patch(w, i):
    return Patch(w["mesh"], i, w["p"], w["pg"], w["dt"], w["scheme"], *w["mat"])


def test_face_codes_follow_oracle_face_order(whole):
    topo = whole["B"].topo
    d = topo.dim
    ref = [F.left * (d + 1) + F.lf for F in topo.faces]
    assert np.array_equal(face_codes(whole["mesh"].elem), ref)


def test_patch_schur_rows_and_columns_equal_whole_mesh(whole):
    slab, S = whole["slab"], whole["S"]
    ne = slab.ne
    blk = slab.ng * slab.d * slab.nphi
    rng = np.random.default_rng(41)
    v = rng.standard_normal(slab.nv)
    ref_row = (S @ v).reshape(ne, blk)
    ref_col = (S.T @ v).reshape(ne, blk)
    for i in sorted({0, ne - 1, *rng.choice(ne, 4, replace=False).tolist()}):
        P = _patch(whole, i)
        Sp = P.slab.schur()
        scale = np.abs(ref_row[i]).max()
        assert np.abs(P.schur_row(v, Sp) - ref_row[i]).max() <= 1e-13 * scale, i
        assert np.abs(P.schur_col(v, Sp) - ref_col[i]).max() <= 1e-13 * np.abs(ref_col[i]).max(), i


def test_patch_coupled_residual_vanishes_at_whole_mesh_solution(whole):
    B, slab = whole["B"], whole["slab"]
    rng = np.random.default_rng(43)
    v_old = rng.standard_normal((slab.ne, slab.d, slab.nphi))
    s_old = rng.standard_normal((slab.nf, slab.nsig, slab.npsi))
    v, s, _, _ = slab.step(v_old, s_old)
    can = lambda j, x: B.to_canonical(j, x)  # noqa: E731
    s_can = np.stack([can(j, s[j].reshape(-1, slab.npsi)) for j in range(slab.nf)])
    s_old_can = np.stack([can(j, s_old[j]) for j in range(slab.nf)])
    codes = face_codes(whole["mesh"].elem)
    b_full = slab.rhs(v_old, s_old)
    blk = slab.ng * slab.d * slab.nphi
    for i in sorted({0, slab.ne - 1, *rng.choice(slab.ne, 3, replace=False).tolist()}):
        P = _patch(whole, i)
        rv, bv, faces = P.coupled_residual(v, s_can, v_old, s_old_can, codes)
        assert np.abs(bv - b_full[i * blk:(i + 1) * blk]).max() <= 1e-13 * np.abs(bv).max()
        assert np.linalg.norm(rv) <= 1e-11 * np.linalg.norm(bv), i
        for rs, bs in faces:
            assert np.linalg.norm(rs) <= 1e-11 * np.linalg.norm(bs), i
    # a wrong state is seen: perturb one stress DOF of a face of element 0
    P = _patch(whole, 0)
    g = P.global_faces(codes)[0]
    bad = s_can.copy()
    bad[g].flat[0] += 1e-3 * np.abs(bad[g]).max()
    rv, bv, faces = P.coupled_residual(v, bad, v_old, s_old_can, codes)
    assert np.linalg.norm(rv) > 1e-8 * np.linalg.norm(bv)
