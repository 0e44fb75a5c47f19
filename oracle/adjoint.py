"""Discrete adjoint of the time-stepping scheme and material gradients of a
receiver misfit (oracle).

Forward map of one slab (eqs. NM25, NM26): the coupled system
    A(theta) X_n = Bm(theta) u_n + F_n,   u_{n+1} = Ex X_n,
with u_n = (v, sigma) the end-of-slab state at t^{n,-}, X_n the slab DOFs,
Bm the old-state coupling (e0 (x) rho Mbar and e0 (x) M_j), F_n the point
source and Ex the end-of-slab extraction (gamma(1) weights).

Misfit: J = sum_{n=1..N} sum_r |v_h(x_r, t^{n,-}) - d_r^n|^2 with v_h the
velocity of u_n.

Adjoint recursion (exact discrete adjoint, Lagrangian method):
    ubar_N = dJ_N/du_N;  for n = N-1..0:
      Lam_n = A^{-T} Ex^T ubar_{n+1},   ubar_n = dJ_n/du_n + Bm^T Lam_n
    dJ/dtheta = sum_n Lam_n^T (dBm/dtheta u_n - dA/dtheta X_n).

A depends on rho_e through the velocity mass blocks and on (lambda_j, mu_j)
linearly through the stress-velocity coupling; the per-element gradients
follow from the volume-weighted face material:
    d lambda_j / d lambda_e = |T_{e,j}| / |R_j|.
"""
from __future__ import annotations

import copy

import numpy as np
import scipy.sparse.linalg as spla

from .assemble import locate
from .basis import phys_basis
from .slab import Slab


class MisfitProblem:
    def __init__(self, slab: Slab, receivers, sources=None, amps=None, data=None):
        self.S = slab
        B = slab.B
        if B.Et_j is not None:
            raise ValueError("the material gradients are taken for the isotropic parameters")
        self.rec = np.asarray(receivers, float)
        self.rec_elem = [locate(B.topo, x) for x in self.rec]
        self.rec_phi = [phys_basis(B.lb, B.maps[e], x[None, :])[0][0]
                        for e, x in zip(self.rec_elem, self.rec)]
        self.sources = sources
        self.amps = amps  # list over steps of (n_src, N_gamma)
        self.data = data  # (N, n_rec, dim) or None
        self._build_derivative_blocks()

    # ------------------------------------------------------------- pieces
    def _with_material(self, lam_j, mu_j, rho):
        B = copy.copy(self.S.B)
        B.lam_j = np.asarray(lam_j, float)
        B.mu_j = np.asarray(mu_j, float)
        B.rho = np.asarray(rho, float)
        return Slab(B, self.S.tb.n - 1 if self.S.scheme == "stdg" else 0, self.S.dt, self.S.scheme)

    def _build_derivative_blocks(self):
        S = self.S
        nf, ne = S.nf, S.ne
        zf, ze = np.zeros(nf), np.zeros(ne)
        # A is affine in the material: the parts proportional to lambda_j, mu_j
        # and rho_i are obtained from unit-material assemblies.
        self.A_lam = self._with_material(np.ones(nf), zf, ze).A
        self.A_mu = self._with_material(zf, np.ones(nf), ze).A
        self.A_rho = self._with_material(zf, zf, np.ones(ne)).A
        nv = S.nv
        self.A_rho = self.A_rho[:nv, :nv]
        self.A_lam = self.A_lam[nv:, :nv]
        self.A_mu = self.A_mu[nv:, :nv]

    def _old_state_rhs(self, v_old, s_old):
        """Bm u_n (the right-hand side without sources), as a vector."""
        return self.S.rhs(v_old, s_old, None)

    def sample(self, v_state):
        d = self.S.d
        out = np.zeros((len(self.rec), d))
        for r, (e, phi) in enumerate(zip(self.rec_elem, self.rec_phi)):
            out[r] = v_state[e] @ phi
        return out

    # ------------------------------------------------------------- forward
    def forward(self, v0, s0, keep=True):
        S = self.S
        v, s = v0.copy(), s0.copy()
        states, slabs, J = [(v, s)], [], 0.0
        obs = []
        for n in range(len(self.amps)):
            src = None
            if self.sources is not None:
                src = dict(self.sources, amp=self.amps[n])
            x = S.solve(S.rhs(v, s, src))
            vsl = x[:S.nv].reshape(S.ne, S.ng, S.d, S.nphi)
            ssl = x[S.nv:].reshape(S.nf, S.ng, S.nsig, S.npsi)
            if S.scheme == "cn":
                v, s = vsl[:, 0].copy(), ssl[:, 0].copy()
            else:
                v = np.einsum("a,eack->eck", S.tb.e1, vsl)
                s = np.einsum("a,jasm->jsm", S.tb.e1, ssl)
            o = self.sample(v)
            obs.append(o)
            if self.data is not None:
                J += float(np.sum((o - self.data[n]) ** 2))
            if keep:
                slabs.append(x)
                states.append((v, s))
        return J, np.array(obs), states, slabs

    # ------------------------------------------------------------- adjoint
    def adjoint_step(self, v_old, s_old, X, vbar, sbar, lu_T=None):
        """One backward step of the recursion above: given the adjoint of the
        new state ubar_{n+1} = (vbar, sbar) (raw stress basis), the old state
        u_n and the slab DOFs X_n, return ubar_n = Bm^T Lam_n and the
        gradient increment Lam_n^T (dBm/dtheta u_n - dA/dtheta X_n) on the
        dual-element and element parameters: (vbar_n, sbar_n, g_lam_j,
        g_mu_j, g_rho)."""
        S = self.S
        nv, ns = S.nv, S.ns
        face_rows = np.arange(ns) // (S.ng * S.nsig * S.npsi)
        elem_rows = np.arange(nv) // (S.ng * S.d * S.nphi)
        # Xbar = Ex^T ubar
        if S.scheme == "cn":
            xv = vbar.reshape(S.ne, 1, S.d, S.nphi)
            xs = sbar.reshape(S.nf, 1, S.nsig, S.npsi)
        else:
            xv = np.einsum("a,eck->eack", S.tb.e1, vbar)
            xs = np.einsum("a,jsm->jasm", S.tb.e1, sbar)
        Xbar = np.concatenate([xv.ravel(), xs.ravel()])
        Lam = (lu_T or spla.splu(S.A.T.tocsc())).solve(Xbar)
        Lv, Ls = Lam[:nv], Lam[nv:]
        Xv = X[:nv]
        # dA/dtheta X terms
        g_lam_j = -np.bincount(face_rows, weights=Ls * (self.A_lam @ Xv), minlength=S.nf)
        g_mu_j = -np.bincount(face_rows, weights=Ls * (self.A_mu @ Xv), minlength=S.nf)
        g_rho = -np.bincount(elem_rows, weights=Lv * (self.A_rho @ Xv), minlength=S.ne)
        # dBm/drho u_n: the old-state momentum term is linear in rho
        b_unit = self._rho_unit_rhs(v_old, s_old)
        g_rho += np.bincount(elem_rows, weights=Lv * b_unit, minlength=S.ne)
        if S.scheme == "cn":
            # CN: the explicit coupling halves also depend on lambda, mu
            vo = v_old.reshape(-1)
            g_lam_j += np.bincount(face_rows, weights=Ls * (-(self.A_lam @ vo)), minlength=S.nf)
            g_mu_j += np.bincount(face_rows, weights=Ls * (-(self.A_mu @ vo)), minlength=S.nf)
        vb, sb = self._bm_transpose(Lam)
        return vb, sb, g_lam_j, g_mu_j, g_rho

    def faces_to_elements(self, g_lam_j, g_mu_j):
        """Face-parameter gradients passed to the elements with the volume
        weights d lambda_j / d lambda_e = |T_{e,j}| / |R_j|."""
        S = self.S
        B = S.B
        g_lam = np.zeros(S.ne)
        g_mu = np.zeros(S.ne)
        for j, F in enumerate(B.topo.faces):
            vl, vr = B.vol_sub[j]
            if F.right >= 0:
                tot = vl + vr
                g_lam[F.left] += g_lam_j[j] * vl / tot
                g_lam[F.right] += g_lam_j[j] * vr / tot
                g_mu[F.left] += g_mu_j[j] * vl / tot
                g_mu[F.right] += g_mu_j[j] * vr / tot
            else:
                g_lam[F.left] += g_lam_j[j]
                g_mu[F.left] += g_mu_j[j]
        return g_lam, g_mu

    def gradient(self, v0, s0, increments=None):
        """dJ/d(lambda_e, mu_e, rho_e) by the discrete adjoint.  With a list
        for ``increments``, each step's element increments (g_lam, g_mu,
        g_rho) are appended to it."""
        S = self.S
        J, obs, states, slabs = self.forward(v0, s0)
        N = len(slabs)
        lu_T = spla.splu(S.A.T.tocsc())
        g_lam_j = np.zeros(S.nf)
        g_mu_j = np.zeros(S.nf)
        g_rho = np.zeros(S.ne)
        # ubar as arrays shaped like the state
        vbar = np.zeros((S.ne, S.d, S.nphi))
        sbar = np.zeros((S.nf, S.nsig, S.npsi))
        for n in range(N - 1, -1, -1):
            # misfit at t^{n+1,-} acts on state n+1
            resid = obs[n] - self.data[n]
            for r, (e, phi) in enumerate(zip(self.rec_elem, self.rec_phi)):
                vbar[e] += 2.0 * np.outer(resid[r], phi)
            v_old, s_old = states[n]
            vbar, sbar, gl, gm, gr = self.adjoint_step(v_old, s_old, slabs[n], vbar, sbar, lu_T)
            if increments is not None:
                increments.append((*self.faces_to_elements(gl, gm), gr))
            g_lam_j += gl
            g_mu_j += gm
            g_rho += gr
        g_lam, g_mu = self.faces_to_elements(g_lam_j, g_mu_j)
        return J, g_lam, g_mu, g_rho

    def _rho_unit_rhs(self, v_old, s_old):
        """d(Bm u)/d(rho) summed per element row: the rho-proportional part of
        the velocity right-hand side with rho = 1."""
        S = self.S
        B = S.B
        out = np.zeros(S.nv)
        if S.scheme == "cn":
            for i in range(S.ne):
                mv = v_old[i] @ B.Mbar[i].T
                out[i * S.d * S.nphi:(i + 1) * S.d * S.nphi] = mv.ravel()
            return out
        e0 = S.tb.e0
        for i in range(S.ne):
            mv = v_old[i] @ B.Mbar[i].T
            for a in range(S.ng):
                base = ((i * S.ng + a) * S.d) * S.nphi
                out[base:base + S.d * S.nphi] = e0[a] * mv.ravel()
        return out

    def _bm_transpose(self, Lam):
        """Bm^T Lam as (vbar, sbar) state arrays."""
        S = self.S
        B = S.B
        nv = S.nv
        Lv = Lam[:nv].reshape(S.ne, S.ng, S.d, S.nphi)
        Ls = Lam[nv:].reshape(S.nf, S.ng, S.nsig, S.npsi)
        vbar = np.zeros((S.ne, S.d, S.nphi))
        sbar = np.zeros((S.nf, S.nsig, S.npsi))
        if S.scheme == "cn":
            # Bm u = [rho Mbar v + dt/2 D s ; M s + dt/2 E Qt v]
            for i in range(S.ne):
                vbar[i] = B.rho[i] * (Lv[i, 0] @ B.Mbar[i])
            for j in range(S.nf):
                sbar[j] = Ls[j, 0] @ B.M[j]
            off_vs = -S.A[:nv, nv:]
            off_sv = -S.A[nv:, :nv]
            vbar += (off_sv.T @ Lam[nv:]).reshape(vbar.shape)
            sbar += (off_vs.T @ Lam[:nv]).reshape(sbar.shape)
            return vbar, sbar
        e0 = S.tb.e0
        for i in range(S.ne):
            vbar[i] = B.rho[i] * (np.einsum("a,ack->ck", e0, Lv[i]) @ B.Mbar[i])
        for j in range(S.nf):
            sbar[j] = np.einsum("a,asm->sm", e0, Ls[j]) @ B.M[j]
        return vbar, sbar
