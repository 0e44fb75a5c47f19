"""Host-side set-up code of the library (no GPU), against the oracle.

tests/host/dual_basis.cpp compiles the library's set-up source on the host
and writes the canonical dual basis of every face at given points.  The
canonical basis is the Gram-Schmidt orthonormalisation over the dual element
of the raw sequence (Section 3, the stress basis of the dual mesh): the
library builds it from Legendre products by Householder QR, the oracle from
monomials by a Cholesky factor of the Gram matrix.  Both span the same
nested spaces with positive leading coefficients, so the functions must
agree; a wrong frame, ordering or orthonormalisation in either shows up.
The harness also writes the library's face table, which must follow the
oracle's face numbering, its coupling blocks, which must be the oracle's D
(eq. MD_3) mapped to the canonical basis, and its dual material, element
mass and time basis.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from oracle.assemble import Blocks
from oracle.basis import TimeBasis
from oracle.mesh import Topology

HERE = os.path.dirname(os.path.abspath(__file__))
HIP_INCLUDE = "/opt/rocm/include"

MESHES = {
    # name: (mesh, p, periodic, p_gamma)
    "2d_free_p3": (lambda: synth.split_square(3, jitter=0.2, seed=5), 3, False, 3),
    "2d_periodic_p2": (lambda: synth.split_square(4, periodic=True, jitter=0.1, seed=6), 2, True, 1),
    "3d_free_p2": (lambda: synth.kuhn_cube(2, periodic=False), 2, False, 2),
    "3d_periodic_p1": (lambda: synth.kuhn_cube(3, periodic=True), 1, True, 0),
    "3d_free_p4": (lambda: synth.kuhn_cube(2, periodic=False), 4, False, 0),
}


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(os.path.join(HIP_INCLUDE, "hip", "hip_runtime.h")):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path_factory.mktemp("host") / "dual_basis")
    subprocess.run([gxx, "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", f"-I{HIP_INCLUDE}", "-w",
                    os.path.join(HERE, "host", "dual_basis.cpp"), "-o", exe, "-lpthread"], check=True)
    return exe


@pytest.mark.parametrize("name", sorted(MESHES))
def test_library_dual_basis_equals_oracle_gram_schmidt(harness, tmp_path, name):
    mk, p, periodic, pg = MESHES[name]
    mesh = mk()
    elem = np.asarray(mesh.elem, dtype=np.int64)
    xyz = np.asarray(mesh.xyz, dtype=np.float64)
    d = elem.shape[1] - 1
    lam, mu, rho = synth.lognormal_material(elem.shape[0], sigma=0.3, seed=31)
    mfile, pfile, ofile = tmp_path / "mesh.bin", tmp_path / "pts.bin", tmp_path / "out.bin"
    with open(mfile, "wb") as f:
        np.array([d, xyz.shape[0], elem.shape[0], p, int(periodic), pg], dtype=np.int64).tofile(f)
        xyz.tofile(f)
        elem.tofile(f)
        for a in (lam, mu, rho):
            np.asarray(a, dtype=np.float64).tofile(f)
    topo = Topology(mesh.xyz, mesh.elem, mesh.period)
    B = Blocks(topo, p, lam, mu, rho)
    # points: the centroids of the two sub-simplices and of the face
    pts = []
    for j, F in enumerate(topo.faces):
        tl = topo.sub_simplex(j, 0).mean(axis=0)
        tr = topo.sub_simplex(j, 1).mean(axis=0) if F.right >= 0 else 0.5 * (tl + F.X.mean(axis=0))
        pts.append([tl, tr, F.X.mean(axis=0)])
    pts = np.asarray(pts, dtype=np.float64)
    K = pts.shape[1]
    with open(pfile, "wb") as f:
        np.array([K], dtype=np.int64).tofile(f)
        pts.tofile(f)
    ffile, bfile, dfile = tmp_path / "faces.bin", tmp_path / "blocks.bin", tmp_path / "data.bin"
    subprocess.run([harness, str(mfile), str(pfile), str(ofile), str(ffile), str(bfile), str(dfile)], check=True)
    # the face table (numbering by left element and local face, sides)
    faces = np.fromfile(ffile, dtype=np.int32).reshape(-1, 4)
    assert np.array_equal(faces, [[F.left, F.lf, F.right, F.rf] for F in topo.faces])
    got = np.fromfile(ofile, dtype=np.float64).reshape(topo.n_face, K, B.npsi)
    worst = 0.0
    for j in range(topo.n_face):
        raw = B.duals[j].eval(pts[j])                       # (K, npsi)
        ref = np.linalg.solve(B.L[j], raw.T).T              # canonical = L^-1 raw
        err = np.abs(got[j] - ref).max() / np.abs(ref).max()
        worst = max(worst, err)
    print(f"{name}: {topo.n_face} faces, worst relative difference {worst:.2e}")
    # degree 4 on tetrahedra: Gram matrices of cond 1e8, two QR-based
    # orthonormalisations of different raw sequences agree to ~1e-11
    p4 = d == 3 and p == 4
    assert worst <= (1e-10 if p4 else 1e-9)
    # the coupling blocks D (eq. MD_3) in the canonical basis: D_can = D_raw L^-T
    Dt = np.fromfile(bfile, dtype=np.float64).reshape(topo.n_face, 2, B.nphi, d, B.npsi)
    worst_d = 0.0
    for j, F in enumerate(topo.faces):
        for side in range(2):
            if side == 1 and F.right < 0:
                assert not Dt[j, 1].any()
                continue
            ref = np.linalg.solve(B.L[j], B.D[j][side].reshape(-1, B.npsi).T).T.reshape(B.nphi, d, B.npsi)
            worst_d = max(worst_d, np.abs(Dt[j, side] - ref).max() / np.abs(ref).max())
    print(f"{name}: worst relative difference of the coupling blocks {worst_d:.2e}")
    assert worst_d <= (1e-10 if p4 else 1e-11)
    # dual material (volume-weighted Lame parameters), element mass rho |J| M_ref
    # against the oracle's rho M_bar, and the time basis (Section 4)
    nf, ne, nphi, ng = topo.n_face, topo.n_elem, B.nphi, pg + 1
    data = np.fromfile(dfile, dtype=np.float64)
    sizes = [2 * nf, ne, nphi * nphi, ng, ng, ng, ng, ng * ng]
    assert data.size == sum(sizes)
    face_lm, elem_w, Mref, tau, w, e0, e1, T = np.split(data, np.cumsum(sizes)[:-1])
    face_lm = face_lm.reshape(nf, 2)
    assert np.allclose(face_lm[:, 0], B.lam_j, rtol=1e-13, atol=0)
    assert np.allclose(face_lm[:, 1], B.mu_j, rtol=1e-13, atol=0)
    Mref = Mref.reshape(nphi, nphi)
    for e in range(ne):
        ref = B.rho[e] * B.Mbar[e]
        assert np.abs(elem_w[e] * Mref - ref).max() <= 1e-12 * np.abs(ref).max(), e
    tb = TimeBasis(pg)
    for got_, ref_ in ((tau, tb.tau), (w, tb.w), (e0, tb.e0), (e1, tb.e1), (T, tb.T.ravel())):
        assert np.allclose(got_, ref_, rtol=0, atol=1e-13)


@pytest.fixture(scope="module")
def proj_harness(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(os.path.join(HIP_INCLUDE, "hip", "hip_runtime.h")):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path_factory.mktemp("host") / "projection")
    subprocess.run([gxx, "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", f"-I{HIP_INCLUDE}", "-w",
                    os.path.join(HERE, "host", "projection.cpp"), "-o", exe, "-lpthread"], check=True)
    return exe


class _PolyField:
    """A random polynomial field of total degree q: velocity (dim components)
    and Voigt stress (n_sigma components)."""

    def __init__(self, dim, q, seed):
        rng = np.random.default_rng(seed)
        self.exps = [e for e in np.ndindex(*([q + 1] * dim)) if sum(e) <= q]
        self.cv = rng.standard_normal((len(self.exps), dim))
        self.cs = rng.standard_normal((len(self.exps), dim * (dim + 1) // 2))

    def _mono(self, x):
        x = np.atleast_2d(x)
        return np.stack([np.prod(x ** np.array(e)[None, :], axis=1) for e in self.exps], axis=1)

    def velocity(self, x, t=0.0):
        return self._mono(x) @ self.cv

    def stress_voigt(self, x, t=0.0):
        return self._mono(x) @ self.cs


@pytest.mark.parametrize("name", sorted(MESHES))
def test_library_projection_of_initial_data_equals_oracle(proj_harness, tmp_path, name):
    """The library's L2 projection of initial data (velocity per element,
    stress per dual element in the canonical basis) equals the oracle's, for
    polynomial data of degree p + 1 (outside the discrete spaces, integrated
    exactly by both rules).  On a free-surface dual element only T_{l,j}
    carries weight."""
    from oracle import waves
    mk, p, periodic, pg = MESHES[name]
    mesh = mk()
    elem = np.asarray(mesh.elem, dtype=np.int64)
    xyz = np.asarray(mesh.xyz, dtype=np.float64)
    d = elem.shape[1] - 1
    lam, mu, rho = synth.lognormal_material(elem.shape[0], sigma=0.3, seed=31)
    mfile = tmp_path / "mesh.bin"
    with open(mfile, "wb") as f:
        np.array([d, xyz.shape[0], elem.shape[0], p, int(periodic), pg], dtype=np.int64).tofile(f)
        xyz.tofile(f)
        elem.tofile(f)
        for a in (lam, mu, rho):
            np.asarray(a, dtype=np.float64).tofile(f)
    topo = Topology(mesh.xyz, mesh.elem, mesh.period)
    B = Blocks(topo, p, lam, mu, rho)
    field = _PolyField(d, p + 1, seed=5)
    v_ref, s_raw = waves.project(B, field, 0.0)
    s_ref = np.stack([B.to_canonical(j, s_raw[j]) for j in range(topo.n_face)])
    psi_deg = 2 * p if d == 2 else p
    for which, ref, fn in ((0, v_ref, field.velocity), (1, s_ref, field.stress_voigt)):
        pfile, vfile, ofile = tmp_path / f"p{which}.bin", tmp_path / f"v{which}.bin", tmp_path / f"o{which}.bin"
        # exact for the data of degree p + 1 times a basis function: one above the lowest degree
        deg = str((2 * p if which == 0 else psi_deg + p) + 1)
        subprocess.run([proj_harness, str(mfile), "0", str(which), deg, str(pfile)], check=True)
        raw = np.fromfile(pfile, dtype=np.float64)
        nq = int(np.frombuffer(raw[:1].tobytes(), dtype=np.int64)[0])
        ncell = topo.n_elem if which == 0 else topo.n_face
        pts = raw[1:1 + ncell * nq * d].reshape(ncell, nq, d)
        wts = raw[1 + ncell * nq * d:].reshape(ncell, nq)
        # the weights integrate the cell volumes: |T_e|, or |R_j| = |T_{l,j}| + |T_{r,j}|
        vol = np.array([topo.volume(e) for e in range(ncell)]) if which == 0 else B.vol_sub.sum(axis=1)
        assert np.allclose(wts.sum(axis=1), vol, rtol=1e-13, atol=0)
        np.ascontiguousarray(fn(pts.reshape(-1, d))).tofile(vfile)
        subprocess.run([proj_harness, str(mfile), "1", str(which), deg, str(vfile), str(ofile)], check=True)
        got = np.fromfile(ofile, dtype=np.float64).reshape(ref.shape)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"{name} which={which}: {nq} points per cell, max rel difference {err:.2e}")
        assert err <= (1e-10 if (d == 3 and p == 4) else 1e-11)


@pytest.mark.parametrize("name,p", [("periodic_p2", 2), ("free_p1", 1), ("free_jitter_p2", 2),
                                    ("free_jitter_p3", 3)])
def test_compressed_3d_operator_rebuilds_the_blocks(tmp_path, name, p):
    """The compressed 3D operator (per face side: the change of basis C from
    the canonical dual basis to a reference basis of P_p on the element's
    reference sub-simplex, and the face-term and Jacobian coefficients; per
    local face: reference tables) rebuilds every stored block of eq. (MD_3)."""
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(os.path.join(HIP_INCLUDE, "hip", "hip_runtime.h")):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path / "compressed")
    subprocess.run([gxx, "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", f"-I{HIP_INCLUDE}", "-w",
                    os.path.join(HERE, "host", "compressed.cpp"), "-o", exe, "-lpthread"], check=True)
    if name == "periodic_p2":
        mesh, periodic = synth.kuhn_cube(3, periodic=True), True
    elif name == "free_p1":
        mesh, periodic = synth.kuhn_cube(2, periodic=False), False
    else:
        mesh = synth.kuhn_cube(2, periodic=False)
        rng = np.random.default_rng(7)
        xyz = mesh.xyz + rng.uniform(-0.08, 0.08, mesh.xyz.shape) * (mesh.xyz > 0) * (mesh.xyz < 1)
        mesh = synth.Mesh(xyz=xyz, elem=mesh.elem, period=None)
        periodic = False
    elem = np.asarray(mesh.elem, dtype=np.int64)
    xyz = np.asarray(mesh.xyz, dtype=np.float64)
    lam, mu, rho = synth.lognormal_material(elem.shape[0], sigma=0.3, seed=31)
    mfile = tmp_path / "mesh.bin"
    with open(mfile, "wb") as f:
        np.array([3, xyz.shape[0], elem.shape[0], p, int(periodic), 0], dtype=np.int64).tofile(f)
        xyz.tofile(f)
        elem.tofile(f)
        for a in (lam, mu, rho):
            np.asarray(a, dtype=np.float64).tofile(f)
    out = subprocess.run([exe, str(mfile)], check=True, capture_output=True, text=True).stdout
    err = float(out.split()[0])
    print(f"{name}: largest difference of the rebuilt blocks {err:.2e} of the largest entry")
    # rounding of the factored sum grows with the degree (2.8e-13 at p = 2,
    # 4.1e-12 at p = 3 on the jittered mesh)
    assert err <= (1e-12 if p <= 2 else 1e-11)


@pytest.fixture(scope="module")
def curved_harness(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(os.path.join(HIP_INCLUDE, "hip", "hip_runtime.h")):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path_factory.mktemp("host") / "curved")
    subprocess.run([gxx, "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", f"-I{HIP_INCLUDE}", "-w",
                    os.path.join(HERE, "host", "curved.cpp"), "-o", exe, "-lpthread"], check=True)
    return exe


@pytest.mark.parametrize("p,q", [(2, 2), (3, 2), (2, 3)])
def test_library_curved_elements_equal_oracle(curved_harness, tmp_path, p, q):
    """Curved boundary elements (Section 3 maps): the library's coupling
    blocks in the canonical basis, element masses, volume fractions and
    barycentres against the oracle's, on a jittered disk whose boundary
    triangles carry geometry of degree q."""
    m = synth.disk_mesh(3, q=q, jitter=0.15, seed=41)
    ids, nodes = m.meta["curved"]
    lam, mu, rho = synth.lognormal_material(m.n_elem, sigma=0.3, seed=42)
    mfile, ofile = tmp_path / "mesh.bin", tmp_path / "out.bin"
    with open(mfile, "wb") as f:
        np.array([m.n_vert, m.n_elem, p, 1, q, len(ids)], dtype=np.int64).tofile(f)
        np.asarray(m.xyz, np.float64).tofile(f)
        np.asarray(m.elem, np.int64).tofile(f)
        for a in (lam, mu, rho):
            np.asarray(a, np.float64).tofile(f)
        np.asarray(ids, np.int64).tofile(f)
        np.asarray(nodes, np.float64).tofile(f)
    subprocess.run([curved_harness, str(mfile), str(ofile)], check=True)
    topo = Topology(m.xyz, m.elem, None)
    B = Blocks(topo, p, lam, mu, rho, curved=(ids, nodes))
    nf, ne, nphi, npsi = topo.n_face, topo.n_elem, B.nphi, B.npsi
    data = np.fromfile(ofile, dtype=np.float64)
    sizes = [nf * 2 * nphi * 2 * npsi, ne * nphi * nphi, nf * 2, ne * 2]
    assert data.size == sum(sizes)
    Dt, mass, wt, bary = np.split(data, np.cumsum(sizes)[:-1])
    Dt = Dt.reshape(nf, 2, nphi, 2, npsi)
    worst = 0.0
    for j, F in enumerate(topo.faces):
        for s in range(len(B.D[j])):
            ref = np.linalg.solve(B.L[j], B.D[j][s].reshape(-1, npsi).T).T.reshape(nphi, 2, npsi)
            worst = max(worst, np.abs(Dt[j, s] - ref).max() / np.abs(ref).max())
    print(f"p={p} q={q}: worst relative difference of the coupling blocks {worst:.2e}")
    assert worst <= 1e-11
    mass = mass.reshape(ne, nphi, nphi)
    for e in range(ne):
        ref = B.rho[e] * B.Mbar[e]
        assert np.abs(mass[e] - ref).max() <= 1e-12 * np.abs(ref).max(), e
    vt = B.vol_sub.sum(axis=1, keepdims=True)
    assert np.allclose(wt.reshape(nf, 2), B.vol_sub / vt, rtol=0, atol=1e-13)
    assert np.allclose(bary.reshape(ne, 2), B.bary, rtol=0, atol=1e-14)
