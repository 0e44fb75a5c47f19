"""Pins of the oracle's curved elements (Section 3: sub- and iso-parametric
maps of the reference triangle), 2D.

A curved element carries geometry nodes of degree q; its velocity basis is
the reference basis composed with the inverse map, and every integral over
it, its sub-simplices T_{i,j} and the dual elements they belong to is taken
in reference coordinates with |det J|.  These pins hold that path to:

- the straight path itself: geometry nodes placed by the affine map give
  the straight element's mass, dual Gram matrix, coupling blocks D and Q~
  and volume fractions (two independent integration routes: physical-
  coordinate rules against mapped reference rules);
- the geometry: the area of the disk meshed with quadratic boundary
  elements converges to pi at order >= 3 (straight edges: order 2);
- the discrete calculus on a curved free-surface mesh: a rigid rotation is
  in the kernel of K, and the discrete gradient of a linear velocity is
  exact (the mapped P_p space holds linear fields for q <= p);
- Section 5: CN conserves the energy and the space-time identity (eq.
  stsum4) holds on the curved mesh with heterogeneous material.
"""
import numpy as np
import pytest

import synth
from oracle.assemble import Blocks
from oracle.mesh import Topology
from oracle.slab import Slab


def _affine_nodes(mesh, q):
    V = mesh.unwrapped_vertices()
    ref = np.array([(i / q, j / q) for j in range(q + 1) for i in range(q + 1 - j)])
    return np.einsum("na,eac->enc", np.column_stack([1 - ref.sum(1), ref]), V)


def _velocity_nodes(B, e):
    """Physical positions of the velocity nodes of element e."""
    cm = B.curved.get(e)
    if cm is not None:
        return cm.x(B.lb.nodes)
    V = B.topo.V[e]
    return V[0] + B.lb.nodes @ (V[1:] - V[0])


@pytest.mark.parametrize("q", [2, 3])
def test_affine_placed_nodes_reproduce_the_straight_element(q):
    mesh = synth.split_square(3, jitter=0.2, seed=21)
    lam, mu, rho = synth.lognormal_material(mesh.n_elem, sigma=0.3, seed=22)
    topo = Topology(mesh.xyz, mesh.elem, None)
    Bs = Blocks(topo, 2, lam, mu, rho)
    ids = np.arange(mesh.n_elem)
    Bc = Blocks(topo, 2, lam, mu, rho, curved=(ids, _affine_nodes(mesh, q)))
    assert len(Bc.curved) == mesh.n_elem
    for e in range(mesh.n_elem):
        assert np.abs(Bc.Mbar[e] - Bs.Mbar[e]).max() <= 1e-13 * np.abs(Bs.Mbar[e]).max()
    for j in range(topo.n_face):
        assert np.abs(Bc.M[j] - Bs.M[j]).max() <= 1e-12 * np.abs(Bs.M[j]).max()
        for s in range(len(Bs.D[j])):
            scale = np.abs(Bs.D[j][s]).max()
            assert np.abs(Bc.D[j][s] - Bs.D[j][s]).max() <= 1e-12 * scale
            assert np.abs(Bc.Qt[j][s] - Bs.Qt[j][s]).max() <= 1e-12 * scale
    assert np.allclose(Bc.vol_sub, Bs.vol_sub, rtol=1e-13, atol=0)
    Ss, Sc = Slab(Bs, 1, 0.05, "stdg"), Slab(Bc, 1, 0.05, "stdg")
    assert abs(Ss.A - Sc.A).max() <= 1e-12 * abs(Ss.A).max()


def test_disk_area_converges_with_curved_boundary():
    """Sum of the element areas (int |det J|) of the unit disk: quadratic
    boundary edges converge at order >= 3, straight ones at order 2."""
    errs = {}
    for curved in (False, True):
        e = []
        for n in (4, 8):
            m = synth.disk_mesh(n, q=2)
            topo = Topology(m.xyz, m.elem, None)
            B = Blocks(topo, 1, *synth.homogeneous_material(m.n_elem), curved=m.meta["curved"] if curved else None)
            area = sum(B.elem_rule(k, 0)[1].sum() for k in range(m.n_elem))
            e.append(abs(area - np.pi))
        errs[curved] = e
    order_straight = np.log2(errs[False][0] / errs[False][1])
    order_curved = np.log2(errs[True][0] / errs[True][1])
    print("area errors", errs, "orders", order_straight, order_curved)
    assert 1.8 <= order_straight <= 2.2
    assert order_curved >= 3.0
    assert errs[True][1] < 1e-2 * errs[False][1]


@pytest.fixture(scope="module")
def disk():
    m = synth.disk_mesh(3, q=2, jitter=0.15, seed=31)
    lam, mu, rho = synth.lognormal_material(m.n_elem, sigma=0.3, seed=32)
    B = Blocks(Topology(m.xyz, m.elem, None), 2, lam, mu, rho, curved=m.meta["curved"])
    return m, B


def test_rigid_rotation_in_kernel_on_curved_disk(disk):
    m, B = disk
    S = Slab(B, 0, 0.1, "stdg")
    K = S.schur() - S.A[:S.nv, :S.nv]
    v = np.zeros((B.topo.n_elem, 1, 2, B.nphi))
    for e in range(B.topo.n_elem):
        x = _velocity_nodes(B, e)
        v[e, 0, 0] = -x[:, 1]
        v[e, 0, 1] = x[:, 0]
    assert np.abs(K @ v.ravel()).max() < 1e-12 * abs(K).max()
    # a non-rigid linear field is not in the kernel
    w = v.copy()
    for e in range(B.topo.n_elem):
        w[e, 0, 0] = _velocity_nodes(B, e)[:, 0]
    assert np.abs(K @ w.ravel()).max() > 1e-3 * abs(K).max()


def test_discrete_gradient_of_linear_field_exact_on_curved_disk(disk):
    """M_j^-1 sum_i Q~_{i,j} v_i = grad v for v linear (every face)."""
    m, B = disk
    G = np.array([[0.3, -1.2], [0.7, 0.4]])      # v = G x + c
    c = np.array([0.1, -0.2])
    v = np.stack([(_velocity_nodes(B, e) @ G.T + c).T for e in range(B.topo.n_elem)])
    for j, F in enumerate(B.topo.faces):
        sides = [F.left] if F.right < 0 else [F.left, F.right]
        g = sum(np.einsum("mlk,ck->mcl", B.Qt[j][s], v[e]) for s, e in enumerate(sides))
        gh = np.linalg.solve(B.M[j], g.reshape(B.npsi, -1)).reshape(B.npsi, 2, 2)
        for s in range(len(sides)):
            x, _, _ = B.sub_rule(j, s, 2)
            got = np.einsum("qm,mcl->qcl", B.duals[j].eval(x), gh)
            assert np.allclose(got, np.broadcast_to(G, got.shape), atol=1e-10), j


def test_energy_statements_on_curved_disk(disk):
    m, B = disk
    rng = np.random.default_rng(5)
    v0 = rng.standard_normal((B.topo.n_elem, 2, B.nphi))
    s0 = 0.1 * rng.standard_normal((B.topo.n_face, 3, B.npsi))
    S = Slab(B, 0, 0.03, "cn")
    v, s = v0, s0
    E0 = S.energy(v, s)
    for _ in range(4):
        _, _, v, s = S.step(v, s)
    assert abs(S.energy(v, s) - E0) <= 1e-12 * E0
    S2 = Slab(B, 1, 0.05, "stdg")
    v, s, E0 = v0, s0, S2.energy(v0, s0)
    for _ in range(2):
        vs, ss, v1, s1 = S2.step(v, s)
        E1 = S2.energy(v1, s1)
        assert abs(E1 - E0 + S2.jump_energy(vs, ss, v, s)) <= 1e-12 * E0
        assert E1 <= E0 * (1 + 1e-14)
        v, s, E0 = v1, s1, E1
