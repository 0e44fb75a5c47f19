"""Plane-wave exact solutions (Section 6.2) and L2 projections (oracle).

2D state U = (sigma_xx, sigma_yy, sigma_xy, u, v).  For a unit direction
n = (n_x, n_y) (the paper writes n = (1, 1); the vectors below are
eigenvectors only for a unit n, so n is normalised):
  r_p = (lambda + 2 mu n_x^2, lambda + 2 mu n_y^2, 2 mu n_x n_y, -n_x c_p, -n_y c_p)
  r_s = (-2 mu n_x n_y, 2 mu n_x n_y, mu (n_x^2 - n_y^2), n_y c_s, -n_x c_s)
  U(x, t) = alpha r sin(k.x - c |k| t), k = 2 pi (1, 1), c_p = sqrt((lambda + 2 mu)/rho),
  c_s = sqrt(mu/rho).
3D shear wave with polarisation a (a.n = 0):
  v = alpha c_s a sin(k.x - c_s |k| t),  sigma = -alpha mu (a n^T + n a^T) sin(k.x - c_s |k| t).
"""
from __future__ import annotations

import numpy as np

from . import quad
from .assemble import Blocks, voigt_index
from .basis import basis_at_ref, phys_basis


def eigvec_2d(kind, lam, mu, rho, n):
    n = np.asarray(n, float)
    n = n / np.linalg.norm(n)
    nx, ny = n
    cp = np.sqrt((lam + 2 * mu) / rho)
    cs = np.sqrt(mu / rho)
    if kind == "p":
        return np.array([lam + 2 * mu * nx * nx, lam + 2 * mu * ny * ny, 2 * mu * nx * ny,
                         -nx * cp, -ny * cp]), cp
    return np.array([-2 * mu * nx * ny, 2 * mu * nx * ny, mu * (nx * nx - ny * ny),
                     ny * cs, -nx * cs]), cs


class PlaneWave2D:
    """Superposition of P and S plane waves along direction n."""

    def __init__(self, lam=2.0, mu=1.0, rho=1.0, kvec=(2 * np.pi, 2 * np.pi), alpha=0.1,
                 waves=("p",)):
        self.k = np.asarray(kvec, float)
        self.alpha = alpha
        self.parts = [eigvec_2d(w, lam, mu, rho, self.k) for w in waves]
        self.knorm = np.linalg.norm(self.k)

    def U(self, x, t):
        """(npts, 5) state at points x (npts, 2) and time t."""
        x = np.atleast_2d(x)
        out = np.zeros((x.shape[0], 5))
        for r, c in self.parts:
            out += self.alpha * np.outer(np.sin(x @ self.k - c * self.knorm * t), r)
        return out

    def velocity(self, x, t):
        return self.U(x, t)[:, 3:5]

    def stress_voigt(self, x, t):
        return self.U(x, t)[:, 0:3]  # (xx, yy, xy)


class ShearWave3D:
    def __init__(self, lam=2.0, mu=1.0, rho=1.0, kvec=(2 * np.pi,) * 3,
                 pol=(1.0, -1.0, 0.0), alpha=0.1):
        self.k = np.asarray(kvec, float)
        self.n = self.k / np.linalg.norm(self.k)
        a = np.asarray(pol, float)
        self.a = a / np.linalg.norm(a)
        self.mu = mu
        self.cs = np.sqrt(mu / rho)
        self.alpha = alpha
        self.knorm = np.linalg.norm(self.k)

    def _phase(self, x, t):
        return np.sin(np.atleast_2d(x) @ self.k - self.cs * self.knorm * t)

    def velocity(self, x, t):
        return self.alpha * self.cs * np.outer(self._phase(x, t), self.a)

    def stress_voigt(self, x, t):
        S = -self.alpha * self.mu * (np.outer(self.a, self.n) + np.outer(self.n, self.a))
        vo = voigt_index(3)
        sv = np.zeros(6)
        for p in range(3):
            for q in range(p, 3):
                sv[vo[p, q]] = S[p, q]
        return np.outer(self._phase(x, t), sv)


class AnisotropicPlaneWave:
    """Plane wave in a homogeneous general medium with stiffness tensor
    E[p,q,c,l] (sigma_pq = sum E[p,q,c,l] d_l v_c, eq. 1.1) and density rho:
    v = alpha a sin(k.x - omega t),
    sigma_pq = -(alpha / omega) sum_cl E[p,q,c,l] a_c k_l sin(k.x - omega t),
    which solves eq. (1.1) identically and eq. (1.2) when
    rho omega^2 a = Gamma a, Gamma_pc = sum_ql E[p,q,c,l] k_q k_l (the
    Christoffel matrix).  ``branch`` picks the eigenpair (0 = fastest)."""

    def __init__(self, E, rho, kvec, alpha=0.1, branch=0):
        self.E = np.asarray(E, float)
        self.d = self.E.shape[0]
        self.k = np.asarray(kvec, float)
        self.rho = float(rho)
        self.alpha = alpha
        G = np.einsum("pqcl,q,l->pc", self.E, self.k, self.k)
        w, V = np.linalg.eigh(0.5 * (G + G.T))
        i = np.argsort(w)[::-1][branch]
        self.a = V[:, i]
        self.omega = np.sqrt(w[i] / self.rho)
        self.S = -(alpha / self.omega) * np.einsum("pqcl,c,l->pq", self.E, self.a, self.k)

    def _phase(self, x, t):
        return np.sin(np.atleast_2d(x) @ self.k - self.omega * t)

    def velocity(self, x, t):
        return self.alpha * np.outer(self._phase(x, t), self.a)

    def stress_voigt(self, x, t):
        vo = voigt_index(self.d)
        sv = np.zeros(self.d * (self.d + 1) // 2)
        for p in range(self.d):
            for q in range(p, self.d):
                sv[vo[p, q]] = self.S[p, q]
        return np.outer(self._phase(x, t), sv)


def project(B: Blocks, wave, t=0.0, extra_degree=6):
    """L2 projections of the wave's velocity onto P_p per element and of its
    stress onto the dual space per dual element (raw basis).

    Returns v[e][c][k] and s_raw[j][s][m].
    """
    d = B.dim
    ne, nf = B.topo.n_elem, B.topo.n_face
    v = np.zeros((ne, d, B.nphi))
    for e in range(ne):
        x, w, xi = B.elem_rule(e, 2 * B.p + extra_degree)
        phi, _ = basis_at_ref(B.lb, B.maps[e], xi)
        rhs = (phi * w[:, None]).T @ wave.velocity(x, t)  # (nphi, d)
        v[e] = np.linalg.solve(B.Mbar[e], rhs).T
    s = np.zeros((nf, B.nsig, B.npsi))
    psi_deg = 2 * B.p if d == 2 else B.p
    for j, F in enumerate(B.topo.faces):
        rhs = np.zeros((B.npsi, B.nsig))
        for side in ([0] if F.right < 0 else [0, 1]):
            x, w, _ = B.sub_rule(j, side, psi_deg + B.p + extra_degree)
            pv = B.duals[j].eval(x)
            rhs += (pv * w[:, None]).T @ wave.stress_voigt(x, t)
        s[j] = np.linalg.solve(B.M[j], rhs).T
    return v, s


def l2_errors(B: Blocks, v, s_raw, wave, t, extra_degree=6):
    """Per-variable L2 errors (velocity components, then Voigt stresses)."""
    d = B.dim
    ev = np.zeros(d)
    for e in range(B.topo.n_elem):
        x, w, xi = B.elem_rule(e, 2 * B.p + extra_degree)
        diff = basis_at_ref(B.lb, B.maps[e], xi)[0] @ v[e].T - wave.velocity(x, t)
        ev += (w[:, None] * diff ** 2).sum(axis=0)
    es = np.zeros(B.nsig)
    psi_deg = 2 * B.p if d == 2 else B.p
    for j, F in enumerate(B.topo.faces):
        for side in ([0] if F.right < 0 else [0, 1]):
            x, w, _ = B.sub_rule(j, side, 2 * psi_deg + extra_degree)
            diff = B.stress_at(s_raw[j], j, x) - wave.stress_voigt(x, t)
            es += (w[:, None] * diff ** 2).sum(axis=0)
    return np.sqrt(ev), np.sqrt(es)
