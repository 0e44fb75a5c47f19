"""Pins of the oracle's discrete adjoint: gradients of a receiver misfit with
respect to per-element (lambda, mu, rho) against central finite differences
of the forward oracle (independent of the adjoint algebra)."""
import numpy as np
import pytest

import synth
from oracle.adjoint import MisfitProblem
from oracle.assemble import Blocks
from oracle.mesh import Topology
from oracle.slab import Slab


def _problem(lam, mu, rho, mesh, p, pg, scheme, dt, nsteps, data=None):
    B = Blocks(Topology(mesh.xyz, mesh.elem, mesh.period), p, lam, mu, rho)
    S = Slab(B, pg, dt, scheme)
    tau = np.array([0.5]) if scheme == "cn" else S.tb.tau
    amps = [synth.ricker((n + tau) * dt, 10.0, 0.02)[None, :] for n in range(nsteps)]
    src = dict(pos=np.array([[0.41, 0.37]]), dir=np.array([[0.3, 1.0]]))
    rec = np.array([[0.1, 0.9], [0.5, 0.95], [0.83, 0.71], [0.66, 0.2]])
    return MisfitProblem(S, rec, src, amps, data)


@pytest.mark.parametrize("scheme,pg", [("stdg", 1), ("cn", 0)])
def test_adjoint_gradient_matches_central_differences(scheme, pg):
    mesh = synth.split_square(4, jitter=0.15, seed=3)
    lam, mu, rho = synth.lognormal_material(mesh.n_elem, sigma=0.2, seed=5)
    dt, nsteps, p = 0.01, 6, 1
    true = synth.lognormal_material(mesh.n_elem, sigma=0.2, seed=6)
    v0 = np.zeros((mesh.n_elem, 2, 3))
    P_true = _problem(*true, mesh, p, pg, scheme, dt, nsteps)
    nf = P_true.S.nf
    s0 = np.zeros((nf, 3, P_true.S.npsi))
    _, data, _, _ = P_true.forward(v0, s0, keep=False)
    P = _problem(lam, mu, rho, mesh, p, pg, scheme, dt, nsteps, data)
    J, gl, gm, gr = P.gradient(v0, s0)
    assert J > 0
    g = np.concatenate([gl, gm, gr])
    theta = np.concatenate([lam, mu, rho])
    rng = np.random.default_rng(11)
    n = mesh.n_elem
    for _ in range(3):
        d = rng.standard_normal(3 * n) * theta
        eps = 1e-6
        Jp = _problem(*np.split(theta + eps * d, 3), mesh, p, pg, scheme, dt, nsteps, data).forward(v0, s0, keep=False)[0]
        Jm = _problem(*np.split(theta - eps * d, 3), mesh, p, pg, scheme, dt, nsteps, data).forward(v0, s0, keep=False)[0]
        fd = (Jp - Jm) / (2 * eps)
        assert abs(fd - g @ d) <= 1e-6 * abs(fd), (fd, g @ d)
