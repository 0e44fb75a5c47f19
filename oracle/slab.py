"""One space-time slab: the coupled system, its Schur complement, stepping
and energy (oracle).

Unknown ordering of the coupled system: velocity first, layout
[elem][a][c][k] (time node a, component c, basis k), then stress, layout
[face][a][s][m] (time node a, Voigt component s, raw dual basis m).

Space-time DG (eqs. NM25, NM26), with the nodal Gauss-Legendre time basis:
  momentum (i,a,c,k):
    sum_b T_ab rho_i (Mbar_i v_i[b])_ck - dt w_a sum_{j in S_i} sum_{l,m}
        D_ij[k,l,m] sigma_j[a, (c,l), m]
      = rho_i e0_a (Mbar_i v_i^-)_ck + (rho S)_i[a,c,k]
  stress (j,a,s=(p,q),m):
    sum_b T_ab (M_j sigma_j[b])_sm - dt w_a sum_{i' in {l,r}} sum_{c,l}
        E_j[p,q,c,l] sum_k Qt_{i'j}[m,l,k] v_{i'}[a,c,k]
      = e0_a (M_j sigma_j^-)_sm
The space-time blocks of eqs. (MD_2)-(MD_6) factor as T (x) Mbar, T (x) M,
dt W (x) D and dt W (x) Qt because the time basis is nodal at the
Gauss-Legendre points (int g_a g_b = w_a delta_ab).

Crank-Nicolson (eqs. NM25.cn, NM26.cn):
    rho Mbar v^{n+1} - dt/2 sum D sigma^{n+1} = rho Mbar v^n + dt/2 sum D sigma^n + rho S
    M sigma^{n+1} - dt/2 E Qt v^{n+1}       = M sigma^n + dt/2 E Qt v^n

The end-of-slab state is v(t^{n+1,-}) = sum_a g_a(1) v[a] (and likewise for
stress); for Crank-Nicolson it is the new value itself.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import quad
from .assemble import (Blocks, compliance_voigt, locate, stiffness,
                       voigt_index)
from .basis import TimeBasis, phys_basis


class Slab:
    def __init__(self, blocks: Blocks, p_gamma: int, dt: float, scheme: str = "stdg"):
        if scheme not in ("stdg", "cn"):
            raise ValueError(scheme)
        if scheme == "cn" and p_gamma != 0:
            raise ValueError("Crank-Nicolson uses p_gamma = 0")
        self.B = blocks
        self.scheme = scheme
        self.tb = TimeBasis(p_gamma)
        self.ng = self.tb.n
        self.dt = float(dt)
        B = blocks
        self.d, self.nphi, self.npsi, self.nsig = B.dim, B.nphi, B.npsi, B.nsig
        self.ne, self.nf = B.topo.n_elem, B.topo.n_face
        self.nv = self.ne * self.ng * self.d * self.nphi
        self.ns = self.nf * self.ng * self.nsig * self.npsi
        self._assemble()
        self._lu = None

    # ------------------------------------------------------------- indexing
    def vi(self, i, a, c, k):
        return ((i * self.ng + a) * self.d + c) * self.nphi + k

    def si(self, j, a, s, m):
        return self.nv + ((j * self.ng + a) * self.nsig + s) * self.npsi + m

    # ------------------------------------------------------------- assembly
    def _assemble(self):
        B, d, ng = self.B, self.d, self.ng
        vo = voigt_index(d)
        cn = self.scheme == "cn"
        T = np.array([[1.0]]) if cn else self.tb.T
        w = np.array([0.5]) if cn else self.tb.w  # coupling weight of the stress/velocity terms
        dt = self.dt
        rows, cols, vals = [], [], []

        def add(r, c, v):
            rows.append(r)
            cols.append(c)
            vals.append(v)

        # velocity mass: T (x) rho Mbar
        for i in range(self.ne):
            Mr = B.rho[i] * B.Mbar[i]
            for a in range(ng):
                for b in range(ng):
                    if T[a, b] == 0.0:
                        continue
                    for c in range(d):
                        for k in range(self.nphi):
                            for kk in range(self.nphi):
                                add(self.vi(i, a, c, k), self.vi(i, b, c, kk), T[a, b] * Mr[k, kk])
        # momentum-stress coupling: - dt w_a D
        for j, F in enumerate(B.topo.faces):
            sides = [F.left] if F.right < 0 else [F.left, F.right]
            for s_idx, i in enumerate(sides):
                Dm = B.D[j][s_idx]
                for a in range(ng):
                    for c in range(d):
                        for k in range(self.nphi):
                            for l in range(d):
                                for m in range(self.npsi):
                                    add(self.vi(i, a, c, k), self.si(j, a, vo[c, l], m),
                                        -dt * w[a] * Dm[k, l, m])
        # stress mass: T (x) M_j; stress-velocity coupling: - dt w_a E Qt
        pairs = [(p, q) for p in range(d) for q in range(p, d)]
        for j, F in enumerate(B.topo.faces):
            Mj = B.M[j]
            E = stiffness(d, B.lam_j[j], B.mu_j[j])
            for a in range(ng):
                for b in range(ng):
                    if T[a, b] == 0.0:
                        continue
                    for sv in range(self.nsig):
                        for m in range(self.npsi):
                            for mm in range(self.npsi):
                                add(self.si(j, a, sv, m), self.si(j, b, sv, mm), T[a, b] * Mj[m, mm])
            sides = [F.left] if F.right < 0 else [F.left, F.right]
            for s_idx, i in enumerate(sides):
                Qm = B.Qt[j][s_idx]
                for (p, q) in pairs:
                    sv = vo[p, q]
                    for c in range(d):
                        for l in range(d):
                            e = E[p, q, c, l]
                            if e == 0.0:
                                continue
                            for a in range(ng):
                                for m in range(self.npsi):
                                    for k in range(self.nphi):
                                        add(self.si(j, a, sv, m), self.vi(i, a, c, k),
                                            -dt * w[a] * e * Qm[m, l, k])
        n = self.nv + self.ns
        self.A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))

    # ------------------------------------------------------------- schur
    def schur(self):
        """Explicit velocity Schur complement S = A_vv - A_vs A_ss^{-1} A_sv,
        eq. (velocity.sys) / (velocity.sys.cn), as a CSR matrix."""
        nv = self.nv
        A = self.A
        Avv = A[:nv, :nv]
        Avs = A[:nv, nv:].tocsc()
        Asv = A[nv:, :nv].tocsr()
        Ass = A[nv:, nv:].tocsr()
        bs = self.ng * self.nsig * self.npsi
        inv_blocks = []
        for j in range(self.nf):
            blk = Ass[j * bs:(j + 1) * bs, j * bs:(j + 1) * bs].toarray()
            inv_blocks.append(np.linalg.inv(blk))
        Ainv = sp.block_diag(inv_blocks, format="csr")
        S = Avv - Avs @ (Ainv @ Asv)
        return S.tocsr()

    # ------------------------------------------------------------- rhs / solve
    def source_term(self, sources):
        """(rho S)_i for point sources, eq. (MD_5_2) with S_v = d delta(x - x_s) S(t)/rho.

        ``sources``: dict with ``pos`` (n, d), ``dir`` (n, d) and ``amp``
        (n, N_gamma) = S(t) at the slab's time nodes (the midpoint for
        Crank-Nicolson).  The time integral uses the Gauss-Legendre rule of
        the slab, which picks dt w_a S(t_a) for time node a.
        """
        out = np.zeros(self.nv)
        if sources is None:
            return out
        B = self.B
        w = np.array([1.0]) if self.scheme == "cn" else self.tb.w
        for s in range(len(sources["pos"])):
            x = np.asarray(sources["pos"][s], float)
            e = locate(B.topo, x)
            if e < 0:
                raise ValueError("source outside the mesh")
            phi, _ = phys_basis(B.lb, B.maps[e], x[None, :])
            for a in range(self.ng):
                for c in range(self.d):
                    for k in range(self.nphi):
                        out[self.vi(e, a, c, k)] += (self.dt * w[a] * sources["amp"][s][a]
                                                     * sources["dir"][s][c] * phi[0, k])
        return out

    def rhs(self, v_old, s_old_raw, sources=None):
        """Right-hand side for the old end-of-slab state (spatial arrays
        v_old[e][c][k] and raw stress s_old_raw[j][s][m])."""
        B, d = self.B, self.d
        b = np.zeros(self.nv + self.ns)
        if self.scheme == "cn":
            b[:self.nv] = 0.0
            for i in range(self.ne):
                mv = B.rho[i] * (v_old[i] @ B.Mbar[i].T)  # (d, nphi)
                for c in range(d):
                    for k in range(self.nphi):
                        b[self.vi(i, 0, c, k)] = mv[c, k]
            for j in range(self.nf):
                ms = s_old_raw[j] @ B.M[j].T
                for sv in range(self.nsig):
                    for m in range(self.npsi):
                        b[self.si(j, 0, sv, m)] = ms[sv, m]
            # explicit half of the coupling terms: minus the off-diagonal blocks times the old state
            nv = self.nv
            b[:nv] -= self.A[:nv, nv:] @ s_old_raw.reshape(-1)
            b[nv:] -= self.A[nv:, :nv] @ v_old.reshape(-1)
        else:
            e0 = self.tb.e0
            for i in range(self.ne):
                mv = B.rho[i] * (v_old[i] @ B.Mbar[i].T)
                for a in range(self.ng):
                    for c in range(d):
                        for k in range(self.nphi):
                            b[self.vi(i, a, c, k)] = e0[a] * mv[c, k]
            for j in range(self.nf):
                ms = s_old_raw[j] @ B.M[j].T
                for a in range(self.ng):
                    for sv in range(self.nsig):
                        for m in range(self.npsi):
                            b[self.si(j, a, sv, m)] = e0[a] * ms[sv, m]
        b[:self.nv] += self.source_term(sources)
        return b

    def solve(self, b):
        if self._lu is None:
            self._lu = spla.splu(self.A.tocsc())
        return self._lu.solve(b)

    def step(self, v_old, s_old_raw, sources=None):
        """One implicit step.  Returns (v_slab, s_slab_raw, v_end, s_end_raw):
        the slab DOFs [e][a][c][k], [j][a][s][m] and the end-of-slab spatial
        states."""
        x = self.solve(self.rhs(v_old, s_old_raw, sources))
        v = x[:self.nv].reshape(self.ne, self.ng, self.d, self.nphi)
        s = x[self.nv:].reshape(self.nf, self.ng, self.nsig, self.npsi)
        if self.scheme == "cn":
            return v, s, v[:, 0].copy(), s[:, 0].copy()
        e1 = self.tb.e1
        return v, s, np.einsum("a,eack->eck", e1, v), np.einsum("a,jasm->jsm", e1, s)

    # ------------------------------------------------------------- energy
    def energy(self, v, s_raw):
        """E = 1/2 sum_i int rho_i |v|^2 + 1/2 sum_j int_{R_j} sigma : E_j^{-1} sigma
        (the quantity of eqs. stsum5 and SP3F), by quadrature of the
        functions."""
        B, d = self.B, self.d
        ek = 0.0
        for i in range(self.ne):
            x, w = quad.simplex_rule(B.topo.V[i], 2 * B.p)
            val = B.velocity_at(v[i], i, x)
            ek += 0.5 * B.rho[i] * np.sum(w[:, None] * val * val)
        es = 0.0
        psi_deg = 2 * B.p if d == 2 else B.p
        for j, F in enumerate(B.topo.faces):
            C = compliance_voigt(d, B.lam_j[j], B.mu_j[j])
            for side in ([0] if F.right < 0 else [0, 1]):
                x, w = quad.simplex_rule(B.topo.sub_simplex(j, side), 2 * psi_deg)
                sv = B.stress_at(s_raw[j], j, x)  # (npts, nsig)
                es += 0.5 * np.sum(w * np.einsum("ps,st,pt->p", sv, C, sv))
        return ek + es

    def jump_energy(self, v_slab, s_slab_raw, v_old, s_old_raw):
        """1/2 ||[v]||_rho^2 + 1/2 ||[sigma]||_{E^-1}^2 at t^n (eq. stsum4), the
        jump between the new slab's start value and the old end value."""
        e0 = self.tb.e0
        vj = np.einsum("a,eack->eck", e0, v_slab) - v_old
        sj = np.einsum("a,jasm->jsm", e0, s_slab_raw) - s_old_raw
        return self.energy(vj, sj)
