"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed
forms of integrals, polynomial reproduction, the symmetry / positive
definiteness theorems of Section 5.1, the energy results of Section 5.2
(eqs. stsum4 and SP3F), the plane-wave eigenstructure of Section 6.2 and the
reductions stated with eq. (NM25.cn).
"""
import math

import numpy as np
import pytest

import synth
from oracle import quad, waves
from oracle.assemble import Blocks, locate
from oracle.basis import LagrangeBasis, TimeBasis, phys_basis
from oracle.mesh import Topology
from oracle.slab import Slab


def _blocks(mesh, p, mat=None):
    topo = Topology(mesh.xyz, mesh.elem, mesh.period)
    lam, mu, rho = mat if mat is not None else synth.homogeneous_material(mesh.n_elem)
    return Blocks(topo, p, lam, mu, rho)


# ------------------------------------------------------------------ quadrature

@pytest.mark.parametrize("dim,deg", [(1, 9), (2, 8), (2, 16), (3, 6), (3, 9)])
def test_quadrature_exact_on_monomials(dim, deg):
    """int over the reference simplex of x^a = prod(a_i!) / (|a| + dim)!"""
    pts, w = quad.reference_rule(dim, deg)
    for a in np.ndindex(*([deg + 1] * dim)):
        if sum(a) > deg:
            continue
        exact = np.prod([math.factorial(k) for k in a]) / math.factorial(sum(a) + dim)
        got = np.sum(w * np.prod(pts ** np.array(a)[None, :], axis=1))
        assert abs(got - exact) <= 1e-14 * max(1.0, exact) + 1e-16


def test_quadrature_physical_simplex_volume_and_face_length():
    V = np.array([[0.1, 0.2], [1.3, 0.4], [0.2, 1.7]])
    _, w = quad.simplex_rule(V, 3)
    area = 0.5 * abs(np.linalg.det((V[1:] - V[0]).T))
    assert abs(w.sum() - area) < 1e-14
    _, w = quad.simplex_rule(V[:2], 3)
    assert abs(w.sum() - np.linalg.norm(V[1] - V[0])) < 1e-14


# ------------------------------------------------------------------ bases

@pytest.mark.parametrize("dim,p", [(2, 1), (2, 3), (2, 4), (3, 2), (3, 3)])
def test_lagrange_basis_nodal_and_reproducing(dim, p):
    lb = LagrangeBasis(dim, p)
    assert np.allclose(lb.eval(lb.nodes), np.eye(lb.n), atol=1e-12)
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1 / dim, size=(20, dim))
    assert np.allclose(lb.eval(x).sum(axis=1), 1.0, atol=1e-13)
    # interpolation reproduces an arbitrary polynomial of degree p
    coef = rng.standard_normal(len(lb.exps))
    f = lambda y: sum(c * np.prod(y ** np.array(e)[None, :], axis=1) for c, e in zip(coef, lb.exps))
    assert np.allclose(lb.eval(x) @ f(lb.nodes), f(x), atol=1e-11)
    assert lb.n == math.comb(p + dim, dim)


@pytest.mark.parametrize("pg", [0, 1, 2, 3])
def test_time_matrix_closed_forms(pg):
    """T u-hat for u = 1 is g(0) and for u = t is the weight vector (both
    from T_ab = g_a(1) g_b(1) - int g_a' g_b = g_a(0)g_b(0) + int g_a g_b');
    T + T^T = g(1)g(1)^T + g(0)g(0)^T (integration by parts)."""
    tb = TimeBasis(pg)
    assert np.allclose(tb.T @ np.ones(tb.n), tb.e0, atol=1e-13)
    if pg >= 1:  # u = t is representable only for p_gamma >= 1
        assert np.allclose(tb.T @ tb.tau, tb.w, atol=1e-13)
    assert np.allclose(tb.T + tb.T.T, np.outer(tb.e1, tb.e1) + np.outer(tb.e0, tb.e0), atol=1e-13)
    assert abs(tb.w.sum() - 1.0) < 1e-15
    if pg == 0:
        assert np.allclose(tb.T, [[1.0]])
    # eigenvalues have positive real part (energy stability of the time slab)
    assert np.all(np.linalg.eigvals(tb.T).real > 0)


def _split_simplex(V):
    """The 2^k simplices of one midpoint (red) refinement of the simplex with
    vertex rows V: corner pieces plus the interior ones (k = 2: 4 triangles,
    k = 3: 8 tetrahedra via the 0-5 diagonal of the inner octahedron)."""
    V = np.asarray(V, float)
    k = V.shape[0] - 1
    mid = {(a, b): 0.5 * (V[a] + V[b]) for a in range(k + 1) for b in range(k + 1)}
    P = lambda a, b: mid[(min(a, b), max(a, b))]
    if k == 2:
        return [np.array([V[0], P(0, 1), P(0, 2)]), np.array([V[1], P(0, 1), P(1, 2)]),
                np.array([V[2], P(0, 2), P(1, 2)]), np.array([P(0, 1), P(1, 2), P(0, 2)])]
    m01, m02, m03, m12, m13, m23 = P(0, 1), P(0, 2), P(0, 3), P(1, 2), P(1, 3), P(2, 3)
    return [np.array([V[0], m01, m02, m03]), np.array([V[1], m01, m12, m13]),
            np.array([V[2], m02, m12, m23]), np.array([V[3], m03, m13, m23]),
            np.array([m01, m02, m03, m23]), np.array([m01, m02, m12, m23]),
            np.array([m01, m03, m13, m23]), np.array([m01, m12, m13, m23])]


@pytest.mark.parametrize("case", ["2d_free_jitter", "2d_periodic", "3d_free", "3d_periodic"])
def test_canonical_dual_basis_is_gram_schmidt_of_raw_sequence(case):
    """The canonical dual basis (raw monomials times the inverse transposed
    Cholesky factor of the oracle's Gram matrix M_j) equals modified
    Gram-Schmidt of the raw sequence, run on its own inner product: a
    quadrature over a midpoint refinement of each sub-simplex T_{i,j} of the
    dual element, with a rule of another degree.  A Gram matrix that missed a
    sub-simplex, a transposed or non-inverted factor, or a wrong raw order
    fails this."""
    p = 2
    mesh = {"2d_free_jitter": lambda: synth.split_square(3, jitter=0.2, seed=3),
            "2d_periodic": lambda: synth.split_square(3, periodic=True, jitter=0.1, seed=4),
            "3d_free": lambda: synth.kuhn_cube(2, periodic=False),
            "3d_periodic": lambda: synth.kuhn_cube(3)}[case]()
    B = _blocks(mesh, p)
    psi_deg = 2 * p if B.dim == 2 else p
    rng = np.random.default_rng(0)
    faces = rng.choice(B.topo.n_face, size=min(B.topo.n_face, 12), replace=False)
    for j in faces:
        F = B.topo.faces[j]
        pts, wts = [], []
        for side in ([0] if F.right < 0 else [0, 1]):
            for piece in _split_simplex(B.topo.sub_simplex(j, side)):
                x, w = quad.simplex_rule(piece, 2 * psi_deg + 3)
                pts.append(x)
                wts.append(w)
        x, w = np.vstack(pts), np.concatenate(wts)
        raw = B.duals[j].eval(x)
        Q = np.zeros_like(raw)
        for m in range(B.npsi):
            f = raw[:, m].copy()
            for k in range(m):
                f -= np.sum(w * f * Q[:, k]) * Q[:, k]
            Q[:, m] = f / np.sqrt(np.sum(w * f * f))
        canon = raw @ np.linalg.inv(B.L[j]).T
        scale = np.abs(Q).max()
        assert np.abs(canon - Q).max() <= 1e-9 * scale, (case, j, np.abs(canon - Q).max())
        assert B.npsi == ((p + 1) ** 2 if B.dim == 2 else math.comb(p + 3, 3))


# ------------------------------------------------------------------ blocks

@pytest.mark.parametrize("case", ["periodic", "free_jitter", "3d"])
def test_qtilde_is_minus_d_transpose(case):
    """Q~_{i,j} = -D_{i,j}^T (Section 5.1), with Q~ assembled from its own
    definition (eq. qtilde), not from D."""
    if case == "periodic":
        B = _blocks(synth.split_square(3, periodic=True), 2)
    elif case == "free_jitter":
        B = _blocks(synth.split_square(3, jitter=0.2, seed=5), 2)
    else:
        B = _blocks(synth.kuhn_cube(2, periodic=False), 2)
    for j in range(B.topo.n_face):
        for s in range(len(B.D[j])):
            Dt = np.transpose(B.D[j][s], (2, 1, 0))
            assert np.allclose(B.Qt[j][s], -Dt, atol=1e-13, rtol=0)


def _poly_field(dim, p, rng):
    """A random vector polynomial of degree p and its gradient."""
    exps = [e for e in np.ndindex(*([p + 1] * dim)) if sum(e) <= p]
    C = rng.standard_normal((dim, len(exps)))

    def val(x):
        mons = np.stack([np.prod(x ** np.array(e)[None, :], axis=1) for e in exps], axis=1)
        return mons @ C.T

    def grad(x):  # (npts, c, l) = d_l v_c
        out = np.zeros((x.shape[0], dim, dim))
        for q, e in enumerate(exps):
            for l in range(dim):
                if e[l] == 0:
                    continue
                ee = list(e)
                ee[l] -= 1
                d = e[l] * np.prod(x ** np.array(ee)[None, :], axis=1)
                out[:, :, l] += np.outer(d, C[:, q])
        return out
    return val, grad


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_patch_test_discrete_gradient_exact(dim, p):
    """For a continuous polynomial velocity of degree p the stress update
    M_j^{-1} sum_i Q~_{i,j} v_i equals grad v exactly (interior and
    free-surface faces alike)."""
    rng = np.random.default_rng(7)
    mesh = synth.split_square(4, jitter=0.2, seed=9) if dim == 2 else synth.kuhn_cube(2, periodic=False)
    B = _blocks(mesh, p)
    val, grad = _poly_field(dim, p, rng)
    v = np.zeros((B.topo.n_elem, dim, B.nphi))
    for e in range(B.topo.n_elem):
        V = B.topo.V[e]
        nodes = V[0] + B.lb.nodes @ (V[1:] - V[0])
        v[e] = val(nodes).T
    for j, F in enumerate(B.topo.faces):
        sides = [F.left] if F.right < 0 else [F.left, F.right]
        g = sum(np.einsum("mlk,ck->mcl", B.Qt[j][s], v[e]) for s, e in enumerate(sides))
        gh = np.linalg.solve(B.M[j], g.reshape(B.npsi, -1)).reshape(B.npsi, dim, dim)
        for s in range(len(sides)):
            x, _ = quad.simplex_rule(B.topo.sub_simplex(j, s), 3)
            got = np.einsum("qm,mcl->qcl", B.duals[j].eval(x), gh)
            assert np.allclose(got, grad(x), atol=1e-10)


def test_divergence_patch_test():
    """For a stress field that is one global polynomial of degree p,
    sum_j D_{i,j} . sigma_j = int_{T_i} phi grad.sigma (Section 4, eq. NM10)."""
    rng = np.random.default_rng(11)
    p, dim = 2, 2
    B = _blocks(synth.split_square(3, jitter=0.15, seed=4), p)
    exps = [e for e in np.ndindex(p + 1, p + 1) if sum(e) <= p]
    C = rng.standard_normal((3, len(exps)))

    def sig(x):
        return np.stack([np.prod(x ** np.array(e)[None, :], axis=1) for e in exps], 1) @ C.T

    def div(x):  # (npts, c): d_l sigma_{c l}
        vo = [[0, 2], [2, 1]]
        out = np.zeros((x.shape[0], 2))
        for q, e in enumerate(exps):
            for l in range(2):
                if e[l] == 0:
                    continue
                ee = list(e)
                ee[l] -= 1
                d = e[l] * np.prod(x ** np.array(ee)[None, :], axis=1)
                for c in range(2):
                    out[:, c] += d * C[vo[c][l], q]
        return out
    # raw stress DOFs by L2 projection onto each dual element (exact: P_p in Q_p)
    s_raw = []
    for j, F in enumerate(B.topo.faces):
        rhs = 0
        for side in ([0] if F.right < 0 else [0, 1]):
            x, w = quad.simplex_rule(B.topo.sub_simplex(j, side), 3 * p + 2)
            pv = B.duals[j].eval(x)
            rhs = rhs + (pv * w[:, None]).T @ sig(x)
        s_raw.append(np.linalg.solve(B.M[j], rhs).T)
    vo = np.array([[0, 2], [2, 1]])
    for e in range(B.topo.n_elem):
        # free-surface faces drop the boundary integral; compare interior elements only
        if any(B.topo.faces[j].right < 0 for j in B.topo.elem_faces[e]):
            continue
        got = np.zeros((2, B.nphi))
        for f, j in enumerate(B.topo.elem_faces[e]):
            F = B.topo.faces[j]
            s = 0 if F.left == e else 1
            Dm = B.D[j][s]
            for c in range(2):
                for l in range(2):
                    got[c] += Dm[:, l, :] @ s_raw[j][vo[c, l]]
        x, w = quad.simplex_rule(B.topo.V[e], 2 * p)
        phi, _ = phys_basis(B.lb, B.maps[e], x)
        ref = ((phi * w[:, None]).T @ div(x)).T
        assert np.allclose(got, ref, atol=1e-11)


def test_constant_velocity_in_kernel_periodic():
    """Constant velocity has zero gradient, so K 1 = 0 on a periodic mesh."""
    B = _blocks(synth.split_square(4, periodic=True, jitter=0.1, seed=2), 2)
    S = Slab(B, 0, 0.1, "stdg")
    Sch = S.schur()
    Mv = S.A[:S.nv, :S.nv]
    for c in range(2):
        one = np.zeros((B.topo.n_elem, 1, 2, B.nphi))
        one[:, :, c, :] = 1.0
        r = (Sch - Mv) @ one.ravel()
        assert np.abs(r).max() < 1e-12 * abs(Sch).max()


def test_rigid_rotation_in_kernel_free_surface():
    """An infinitesimal rotation v = (-y, x) has skew gradient, zero strain
    rate and hence no stress: K v = 0 on a free-surface mesh."""
    B = _blocks(synth.split_square(4, jitter=0.2, seed=3), 1)
    S = Slab(B, 0, 0.1, "stdg")
    K = S.schur() - S.A[:S.nv, :S.nv]
    v = np.zeros((B.topo.n_elem, 1, 2, B.nphi))
    for e in range(B.topo.n_elem):
        V = B.topo.V[e]
        nodes = V[0] + B.lb.nodes @ (V[1:] - V[0])
        v[e, 0, 0] = -nodes[:, 1]
        v[e, 0, 1] = nodes[:, 0]
    assert np.abs(K @ v.ravel()).max() < 1e-12 * abs(K).max()


# ------------------------------------------------------------------ theorems

@pytest.mark.parametrize("hetero", [False, True])
def test_cn_schur_symmetric_positive_definite(hetero):
    """Section 5.1: the CN velocity matrix is symmetric and positive definite
    (proved for homogeneous material; observed for heterogeneous)."""
    w = synth.workload("c1")
    mat = synth.lognormal_material(w["mesh"].n_elem, sigma=0.3, seed=4) if hetero else None
    B = _blocks(w["mesh"], 1, mat)
    S = Slab(B, 0, 0.01, "cn").schur().toarray()
    assert np.linalg.norm(S - S.T) <= 1e-14 * np.linalg.norm(S)
    assert np.linalg.eigvalsh(0.5 * (S + S.T)).min() > 0


def test_cn_is_euler_with_quarter_coupling():
    """With p_gamma = 0 the DG-in-time slab is implicit Euler, A = rho Mbar +
    dt^2 K; Crank-Nicolson gives rho Mbar + dt^2 K / 4 (eq. velocity.sys.cn)."""
    B = _blocks(synth.split_square(3, periodic=True), 1)
    S_ie = Slab(B, 0, 0.02, "stdg")
    S_cn = Slab(B, 0, 0.02, "cn")
    Mv = S_ie.A[:S_ie.nv, :S_ie.nv]
    K_ie = (S_ie.schur() - Mv).toarray()
    K_cn = (S_cn.schur() - Mv).toarray()
    assert np.allclose(K_cn, K_ie / 4, atol=1e-15 * abs(K_ie).max())


def test_cn_energy_conservation_c1():
    """Section 5.2, eq. (SP3F): CN conserves energy exactly (drift <= 1e-12)."""
    w = synth.workload("c1")
    B = _blocks(w["mesh"], 1)
    S = Slab(B, 0, w["dt"], "cn")
    v, s = waves.project(B, waves.PlaneWave2D(waves=("p",)), 0.0)
    E0 = S.energy(v, s)
    for _ in range(w["steps"]):
        _, _, v, s = S.step(v, s)
    assert abs(S.energy(v, s) - E0) <= 1e-12 * E0


@pytest.mark.parametrize("pg", [1, 2])
def test_stdg_energy_dissipation_identity(pg):
    """Section 5.2, eq. (stsum4): E^{n+1} - E^n + jump terms = 0 exactly, for
    piecewise-constant heterogeneous material on a free-surface mesh."""
    mesh = synth.split_square(3, jitter=0.2, seed=6)
    mat = synth.lognormal_material(mesh.n_elem, sigma=0.3, seed=8)
    B = _blocks(mesh, 1, mat)
    S = Slab(B, pg, 0.05, "stdg")
    rng = np.random.default_rng(0)
    v = rng.standard_normal((B.topo.n_elem, 2, B.nphi))
    s = rng.standard_normal((B.topo.n_face, 3, B.npsi)) * 0.1
    E0 = S.energy(v, s)
    for _ in range(3):
        vs, ss, v1, s1 = S.step(v, s)
        E1 = S.energy(v1, s1)
        J = S.jump_energy(vs, ss, v, s)
        assert abs(E1 - E0 + J) <= 1e-12 * E0
        assert E1 <= E0 * (1 + 1e-14)
        v, s, E0 = v1, s1, E1


# ------------------------------------------------------------------ waves

@pytest.mark.parametrize("kind", ["p", "s"])
def test_plane_wave_solves_the_pde(kind):
    """The 2D plane waves of eq. (NT2.2) (with unit n) satisfy
    sigma_t - E grad v = 0 and rho v_t - div sigma = 0 (central differences)."""
    lam, mu, rho = 2.0, 1.0, 1.0
    w = waves.PlaneWave2D(lam, mu, rho, waves=(kind,))
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (10, 2))
    h = 1e-5
    U = lambda x, t: w.U(x, t)
    Ut = (U(x, h) - U(x, -h)) / (2 * h)
    Ux = (U(x + [h, 0], 0) - U(x - [h, 0], 0)) / (2 * h)
    Uy = (U(x + [0, h], 0) - U(x - [0, h], 0)) / (2 * h)
    sxx_t, syy_t, sxy_t, u_t, v_t = Ut.T
    ux, vx = Ux[:, 3], Ux[:, 4]
    uy, vy = Uy[:, 3], Uy[:, 4]
    div = ux + vy
    assert np.allclose(sxx_t, lam * div + 2 * mu * ux, atol=1e-6)
    assert np.allclose(syy_t, lam * div + 2 * mu * vy, atol=1e-6)
    assert np.allclose(sxy_t, mu * (uy + vx), atol=1e-6)
    assert np.allclose(rho * u_t, Ux[:, 0] + Uy[:, 2], atol=1e-6)
    assert np.allclose(rho * v_t, Ux[:, 2] + Uy[:, 1], atol=1e-6)


def test_shear_wave_3d_solves_the_pde():
    w = waves.ShearWave3D()
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, (6, 3))
    h = 1e-5
    vt = (w.velocity(x, h) - w.velocity(x, -h)) / (2 * h)
    st = (w.stress_voigt(x, h) - w.stress_voigt(x, -h)) / (2 * h)
    vo = np.array([[0, 5, 4], [5, 1, 3], [4, 3, 2]])
    G = np.zeros((6, 3, 3))  # d_l v_c
    divs = np.zeros((6, 3))
    for l in range(3):
        e = np.zeros(3)
        e[l] = h
        G[:, :, l] = (w.velocity(x + e, 0) - w.velocity(x - e, 0)) / (2 * h)
        ds = (w.stress_voigt(x + e, 0) - w.stress_voigt(x - e, 0)) / (2 * h)
        for c in range(3):
            divs[:, c] += ds[:, vo[c, l]]
    for p in range(3):
        for q in range(p, 3):
            ref = 2.0 * np.trace(G, axis1=1, axis2=2) * (p == q) + 1.0 * (G[:, p, q] + G[:, q, p])
            assert np.allclose(st[:, vo[p, q]], ref, atol=1e-6)
    assert np.allclose(vt, divs, atol=1e-6)


# ------------------------------------------------------------------ sources

def test_point_source_location_and_partition_of_unity():
    mesh = synth.split_square(4, jitter=0.2, seed=1)
    B = _blocks(mesh, 2)
    S = Slab(B, 1, 0.01, "stdg")
    x = np.array([0.503, 0.497])
    e = locate(B.topo, x)
    # brute force: the point is inside element e (barycentric >= 0)
    V = B.topo.V[e]
    lam = np.linalg.solve((V[1:] - V[0]).T, x - V[0])
    assert lam.min() >= 0 and lam.sum() <= 1
    src = dict(pos=x[None, :], dir=np.array([[0.0, 1.0]]), amp=np.array([[2.0, 3.0]]))
    b = S.source_term(src).reshape(B.topo.n_elem, 2, 2, B.nphi)
    assert np.count_nonzero(np.abs(b).sum(axis=(1, 2, 3))) == 1
    # the nodal basis sums to one, so the DOFs of component y add up to dt w_a S_a
    assert np.allclose(b[e, :, 1].sum(axis=1), 0.01 * S.tb.w * [2.0, 3.0], atol=1e-15)
    assert np.all(b[e, :, 0] == 0)


@pytest.mark.parametrize("case", ["cn_2d", "stdg_2d", "cn_3d"])
def test_schur_krylov_step_equals_coupled_lu_step(case):
    """The oracle's Schur-complement Krylov step (eliminate the stress, CG or
    GMRES on the velocity system, back-substitute) reaches the coupled
    sparse-LU step: the solution of eqs. NM25/NM26 is unique (Section 4), so
    the two agree to the Krylov tolerance."""
    if case == "cn_2d":
        mesh, p, pg, sch = synth.split_square(4, periodic=True), 2, 0, "cn"
    elif case == "stdg_2d":
        mesh, p, pg, sch = synth.split_square(4, jitter=0.2, seed=5), 2, 1, "stdg"
    else:
        mesh, p, pg, sch = synth.kuhn_cube(2, periodic=False), 2, 0, "cn"
    B = _blocks(mesh, p, synth.lognormal_material(mesh.n_elem, seed=9))
    slab = Slab(B, pg, 0.02, sch)
    rng = np.random.default_rng(7)
    v0 = rng.standard_normal((B.topo.n_elem, B.dim, B.nphi))
    s0 = rng.standard_normal((B.topo.n_face, B.nsig, B.npsi))
    _, _, v1, s1 = slab.step(v0, s0)
    _, _, v2, s2, its = slab.step_schur(v0, s0, rtol=1e-13)
    assert its > 0
    assert np.linalg.norm(v2 - v1) <= 1e-10 * np.linalg.norm(v1)
    assert np.linalg.norm(s2 - s1) <= 1e-10 * np.linalg.norm(s1)


@pytest.mark.parametrize("case", ["stdg_2d_free", "cn_3d_periodic"])
def test_preconditioners_invert_single_element_columns(case):
    """Pre1 and Pre2 (Appendix A): for u supported on one element i, S u is
    supported on the stencil of i, whose restriction of S is exactly the
    diagonal block (Pre1) or the patch matrix A_i of eq. APPRE1 (Pre2); so
    (P S u)_i = u_i for both.  Pre2 is not block-diagonal, Pre1 is."""
    if case == "stdg_2d_free":
        mesh, p, pg, sch = synth.split_square(4, jitter=0.2, seed=5), 2, 1, "stdg"
    else:
        mesh, p, pg, sch = synth.kuhn_cube(3), 1, 0, "cn"
    B = _blocks(mesh, p, synth.lognormal_material(mesh.n_elem, seed=9))
    slab = Slab(B, pg, 0.02, sch)
    S = slab.schur()
    P1, P2 = slab.block_jacobi(), slab.patch_preconditioner()
    nb = slab.ng * B.dim * B.nphi
    rng = np.random.default_rng(3)
    for i in rng.choice(B.topo.n_elem, 5, replace=False):
        u = np.zeros(slab.nv)
        u[i * nb:(i + 1) * nb] = rng.standard_normal(nb)
        for P in (P1, P2):
            got = (P @ (S @ u))[i * nb:(i + 1) * nb]
            assert np.allclose(got, u[i * nb:(i + 1) * nb], rtol=0, atol=1e-10 * np.abs(u).max())
    # Pre2 couples an element to its neighbours' values, Pre1 does not
    i = 0
    off = P2[i * nb:(i + 1) * nb].toarray().copy()
    off[:, i * nb:(i + 1) * nb] = 0.0
    assert np.abs(off).max() > 1e-6 * np.abs(P2[i * nb:(i + 1) * nb].toarray()).max()
    off1 = P1[i * nb:(i + 1) * nb].toarray().copy()
    off1[:, i * nb:(i + 1) * nb] = 0.0
    assert not off1.any()


def test_patch_preconditioner_is_the_inverse_when_stencils_cover_the_mesh():
    """On two triangles (one square, free surface) each element's stencil is
    the whole mesh, so the patch matrix of eq. APPRE1 is the whole velocity
    operator and Pre2 is its exact inverse."""
    mesh = synth.split_square(1)
    B = _blocks(mesh, 2, synth.lognormal_material(mesh.n_elem, seed=4))
    slab = Slab(B, 1, 0.05, "stdg")
    S = slab.schur().toarray()
    P2 = slab.patch_preconditioner().toarray()
    assert np.abs(P2 @ S - np.eye(slab.nv)).max() <= 1e-10
