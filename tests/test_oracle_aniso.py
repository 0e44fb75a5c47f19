"""Pins of the oracle's general (anisotropic) material, Section 2.

The library takes a general medium as the Voigt matrix E~ of s~ = E~ e~,
with the strain's shear components e_xy = (d_y u + d_x v) / 2 (so the
isotropic matrix of eq. 5 has 2 mu on the shear diagonal).  The oracle turns
E~ into the tensor E[p,q,c,l] of eq. (1.1) and into the compliance form of
the energy.  These pins hold it to:

- the definition itself: sigma from E applied to a velocity gradient equals
  E~ times the Voigt strain rate of that gradient, and E equals the tensor
  entries the synthetic media are drawn from;
- eq. 5: the isotropic E~ reproduces the isotropic operator and energy of
  the Lame path exactly (a wrong shear factor changes mu there);
- the tensor contraction sigma : E^-1 sigma of the energy;
- Section 5: CN conserves and the space-time scheme dissipates energy with
  a general E = E^T > 0, and the CN velocity system stays SPD;
- an exact plane wave of a tilted anisotropic medium (Christoffel
  equation), built from the tensor entries directly, to which the scheme
  converges at order p + 1 or better.
"""
import numpy as np
import pytest

import synth
from oracle import waves
from oracle.assemble import (Blocks, compliance_from_voigt, stiffness,
                             stiffness_from_voigt, voigt_index)
from oracle.mesh import Topology
from oracle.slab import Slab


def _tensor_from_entries(H, dim):
    """E[p,q,c,l] = H[v(pq)][v(cl)]: the tensor entries laid out as a Voigt
    matrix, with both minor symmetries by construction."""
    vo = voigt_index(dim)
    E = np.zeros((dim,) * 4)
    for p in range(dim):
        for q in range(dim):
            for c in range(dim):
                for l in range(dim):
                    E[p, q, c, l] = H[vo[p, q], vo[c, l]]
    return E


def _eq5(dim, lam, mu):
    """The isotropic E~ of eq. 5 (its 2D restriction in 2D)."""
    ns = dim * (dim + 1) // 2
    Et = np.zeros((ns, ns))
    Et[:dim, :dim] = lam
    Et[np.arange(dim), np.arange(dim)] = lam + 2 * mu
    Et[np.arange(dim, ns), np.arange(dim, ns)] = 2 * mu
    return Et


@pytest.mark.parametrize("dim", [2, 3])
def test_voigt_matrix_acts_on_the_strain_rate(dim):
    Et, _ = synth.anisotropic_material(4, dim, seed=1)
    vo = voigt_index(dim)
    ns = dim * (dim + 1) // 2
    W = np.array([1.0] * dim + [2.0] * (ns - dim))
    rng = np.random.default_rng(2)
    for e in range(4):
        E = stiffness_from_voigt(dim, Et[e])
        # the tensor entries the medium was drawn from (H = E~ W^-1)
        assert np.abs(E - _tensor_from_entries(Et[e] / W[None, :], dim)).max() <= 1e-14 * np.abs(E).max()
        g = rng.standard_normal((dim, dim))           # g[c, l] = d_l v_c
        sig = np.einsum("pqcl,cl->pq", E, g)
        eps = np.zeros(ns)                             # Voigt strain rate, tensor shear
        for c in range(dim):
            for l in range(c, dim):
                eps[vo[c, l]] = g[c, c] if c == l else 0.5 * (g[c, l] + g[l, c])
        s = Et[e] @ eps
        for p in range(dim):
            for q in range(dim):
                assert abs(sig[p, q] - s[vo[p, q]]) <= 1e-13 * np.abs(s).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_compliance_is_the_tensor_contraction(dim):
    """s^T C s = sigma : eps with eps the strain E~^-1 s, summed over all
    tensor entries."""
    Et, _ = synth.anisotropic_material(3, dim, seed=5)
    vo = voigt_index(dim)
    rng = np.random.default_rng(6)
    for e in range(3):
        s = rng.standard_normal(dim * (dim + 1) // 2)
        eps = np.linalg.solve(Et[e], s)
        full = sum(s[vo[p, q]] * eps[vo[p, q]] for p in range(dim) for q in range(dim))
        C = compliance_from_voigt(dim, Et[e])
        assert abs(s @ C @ s - full) <= 1e-13 * abs(full)
        assert np.abs(C - C.T).max() <= 1e-13 * np.abs(C).max()


@pytest.mark.parametrize("dim,p,pg,scheme", [(2, 2, 1, "stdg"), (3, 1, 0, "cn")])
def test_isotropic_voigt_matrix_reproduces_the_lame_operator(dim, p, pg, scheme):
    mesh = synth.split_square(3, jitter=0.2, seed=7) if dim == 2 else synth.kuhn_cube(2, periodic=False)
    lam, mu, rho = synth.lognormal_material(mesh.n_elem, sigma=0.3, seed=9)
    topo = Topology(mesh.xyz, mesh.elem, mesh.period)
    Bi = Blocks(topo, p, lam, mu, rho)
    Ba = Blocks(topo, p, None, None, rho, stiffness=np.stack([_eq5(dim, a, b) for a, b in zip(lam, mu)]))
    for j in range(topo.n_face):
        assert np.abs(Ba.face_stiffness(j) - stiffness(dim, Bi.lam_j[j], Bi.mu_j[j])).max() <= 1e-13 * Bi.lam_j[j]
    Si, Sa = Slab(Bi, pg, 0.05, scheme), Slab(Ba, pg, 0.05, scheme)
    assert abs(Si.A - Sa.A).max() <= 1e-13 * abs(Si.A).max()
    rng = np.random.default_rng(0)
    v = rng.standard_normal((topo.n_elem, dim, Bi.nphi))
    s = rng.standard_normal((topo.n_face, Bi.nsig, Bi.npsi))
    assert abs(Si.energy(v, s) - Sa.energy(v, s)) <= 1e-13 * Si.energy(v, s)


def test_cn_anisotropic_energy_conservation_and_spd():
    """Section 5 with a homogeneous general E = E^T > 0: the CN velocity
    system is SPD and CN conserves the energy (drift <= 1e-12)."""
    mesh = synth.split_square(4, periodic=True, jitter=0.15, seed=12)
    Et, rho = synth.anisotropic_material(mesh.n_elem, 2, homogeneous=True, seed=13)
    B = Blocks(Topology(mesh.xyz, mesh.elem, mesh.period), 2, None, None, rho, stiffness=Et)
    S = Slab(B, 0, 0.03, "cn")
    K = S.schur().toarray()
    assert np.linalg.norm(K - K.T) <= 1e-14 * np.linalg.norm(K)
    assert np.linalg.eigvalsh(0.5 * (K + K.T)).min() > 0
    rng = np.random.default_rng(1)
    v = rng.standard_normal((B.topo.n_elem, 2, B.nphi))
    s = 0.1 * rng.standard_normal((B.topo.n_face, 3, B.npsi))
    E0 = S.energy(v, s)
    for _ in range(5):
        _, _, v, s = S.step(v, s)
    assert abs(S.energy(v, s) - E0) <= 1e-12 * E0


@pytest.mark.parametrize("dim", [2, 3])
def test_stdg_anisotropic_energy_dissipation_identity(dim):
    """Section 5.2, eq. (stsum4), heterogeneous general medium on a free-
    surface mesh: E^{n+1} - E^n + jump terms = 0."""
    mesh = synth.split_square(3, jitter=0.2, seed=14) if dim == 2 else synth.kuhn_cube(1, periodic=False)
    Et, rho = synth.anisotropic_material(mesh.n_elem, dim, sigma=0.3, seed=15)
    B = Blocks(Topology(mesh.xyz, mesh.elem, mesh.period), 1, None, None, rho, stiffness=Et)
    S = Slab(B, 1, 0.05, "stdg")
    rng = np.random.default_rng(0)
    v = rng.standard_normal((B.topo.n_elem, dim, B.nphi))
    s = 0.1 * rng.standard_normal((B.topo.n_face, B.nsig, B.npsi))
    E0 = S.energy(v, s)
    for _ in range(2):
        vs, ss, v1, s1 = S.step(v, s)
        E1 = S.energy(v1, s1)
        assert abs(E1 - E0 + S.jump_energy(vs, ss, v, s)) <= 1e-12 * E0
        assert E1 <= E0 * (1 + 1e-14)
        v, s, E0 = v1, s1, E1


def _tilted_wave(seed=11):
    Et, rho = synth.anisotropic_material(1, 2, homogeneous=True, seed=seed)
    E = _tensor_from_entries(Et[0] / np.array([1.0, 1.0, 2.0])[None, :], 2)
    return Et[0], rho[0], waves.AnisotropicPlaneWave(E, rho[0], (2 * np.pi, 2 * np.pi))


def test_anisotropic_plane_wave_solves_the_pde():
    """Eqs. (1.1), (1.2) by central differences, with the tensor entries."""
    Et, rho, w = _tilted_wave()
    E = _tensor_from_entries(Et / np.array([1.0, 1.0, 2.0])[None, :], 2)
    vo = voigt_index(2)
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, (8, 2))
    h = 1e-5
    vt = (w.velocity(x, h) - w.velocity(x, -h)) / (2 * h)
    st = (w.stress_voigt(x, h) - w.stress_voigt(x, -h)) / (2 * h)
    G = np.zeros((8, 2, 2))
    divs = np.zeros((8, 2))
    for l in range(2):
        e = np.zeros(2)
        e[l] = h
        G[:, :, l] = (w.velocity(x + e, 0) - w.velocity(x - e, 0)) / (2 * h)
        ds = (w.stress_voigt(x + e, 0) - w.stress_voigt(x - e, 0)) / (2 * h)
        for c in range(2):
            divs[:, c] += ds[:, vo[c, l]]
    sig_t = np.einsum("pqcl,ncl->npq", E, G)
    scale = np.abs(st).max()
    for p in range(2):
        for q in range(2):
            assert np.allclose(st[:, vo[p, q]], sig_t[:, p, q], atol=1e-6 * scale)
    assert np.allclose(rho * vt, divs, atol=1e-6 * scale)


def test_anisotropic_plane_wave_convergence_p2():
    """p = p_gamma = 2, one period of the tilted quasi-P wave on periodic
    jittered 4 x 4 and 8 x 8 meshes of the unit square: every variable
    converges at an observed order >= 3 (the Table 1 orders at p = 2 are
    3.5-4), with errors below 1% of the amplitude on the finer mesh.  A
    wrong shear factor or Voigt order gives an O(1) error that does not
    decrease."""
    Et, rho, wave = _tilted_wave()
    T = 2 * np.pi / wave.omega
    errs = []
    for n in (4, 8):
        m = synth.split_square(n, periodic=True, jitter=0.1, seed=3)
        B = Blocks(Topology(m.xyz, m.elem, m.period), 2, None, None, np.full(m.n_elem, rho),
                   stiffness=np.repeat(Et[None], m.n_elem, axis=0))
        nsteps = int(np.ceil(T / (0.2 / n)))
        S = Slab(B, 2, T / nsteps, "stdg")
        v, s = waves.project(B, wave, 0.0)
        for _ in range(nsteps):
            _, _, v, s = S.step(v, s)
        ev, es = waves.l2_errors(B, v, s, wave, T)
        errs.append(np.concatenate([ev, es]))
    amp = np.concatenate([np.abs(wave.alpha * wave.a), np.abs(wave.S[[0, 1, 0], [0, 1, 1]])])
    order = np.log2(errs[0] / errs[1])
    print("errors", errs[1], "orders", order)
    assert np.all(order >= 3.0), order
    assert np.all(errs[1] <= 0.01 * amp.max())
