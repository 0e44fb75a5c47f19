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
from .basis import TimeBasis, basis_at_ref, phys_basis


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
        """The coupled slab matrix, built from dense local blocks: per element
        T (x) I_d (x) rho_i Mbar_i, per face T (x) I_sigma (x) M_j, and per face
        side the couplings -dt w_a D_{i,j} (momentum rows) and
        -dt w_a E_j Qt_{i,j} (stress rows), scattered to their global rows and
        columns (duplicates are summed)."""
        B, d, ng = self.B, self.d, self.ng
        nphi, npsi, nsig = self.nphi, self.npsi, self.nsig
        ne, nf, nv = self.ne, self.nf, self.nv
        vo = voigt_index(d)
        cn = self.scheme == "cn"
        T = np.array([[1.0]]) if cn else self.tb.T
        w = np.array([0.5]) if cn else self.tb.w  # coupling weight of the stress/velocity terms
        dt = self.dt
        nvl, nsl = ng * d * nphi, ng * nsig * npsi  # unknowns per element / per face
        rows, cols, vals = [], [], []

        def emit(r0, c0, blocks):
            """Dense local blocks (n, R, C) whose rows start at global index
            r0[n] and columns at c0[n] (each block's rows and columns are
            contiguous in the global ordering)."""
            n, R, C = blocks.shape
            rr = np.broadcast_to((r0[:, None] + np.arange(R)[None, :])[:, :, None], (n, R, C))
            cc = np.broadcast_to((c0[:, None] + np.arange(C)[None, :])[:, None, :], (n, R, C))
            nz = blocks != 0.0
            rows.append(rr[nz])
            cols.append(cc[nz])
            vals.append(blocks[nz])

        # velocity mass: T (x) I_d (x) rho_i Mbar_i, rows/cols (a, c, k)
        Mr = B.rho[:, None, None] * np.asarray(B.Mbar)
        blk = np.einsum("ab,cC,ekK->eackbCK", T, np.eye(d), Mr).reshape(ne, nvl, nvl)
        e_idx = np.arange(ne)
        emit(e_idx * nvl, e_idx * nvl, blk)
        # stress mass: T (x) I_sigma (x) M_j, rows/cols (a, s, m)
        blk = np.einsum("ab,sS,jmn->jasmbSn", T, np.eye(nsig), np.asarray(B.M)).reshape(nf, nsl, nsl)
        f_idx = np.arange(nf)
        emit(nv + f_idx * nsl, nv + f_idx * nsl, blk)
        # Voigt selector P[c, l, s] = 1 where the tensor entry (c, l) is Voigt
        # component s, and the Hooke law per face on Voigt rows:
        # Ev[j, s=(p,q), c, l] = E_j[p, q, c, l] for p <= q
        P = np.zeros((d, d, nsig))
        for c in range(d):
            for l in range(d):
                P[c, l, vo[c, l]] = 1.0
        Ev = np.zeros((nf, nsig, d, d))
        for j in range(nf):
            E = B.face_stiffness(j)
            for pp in range(d):
                for qq in range(pp, d):
                    Ev[j, vo[pp, qq]] = E[pp, qq]
        Iw = -dt * np.diag(w)  # delta_{aA} (-dt w_a)
        faces = B.topo.faces
        for side in (0, 1):
            js = np.array([j for j in range(nf) if side == 0 or faces[j].right >= 0], dtype=np.int64)
            if js.size == 0:
                continue
            el = np.array([faces[j].left if side == 0 else faces[j].right for j in js], dtype=np.int64)
            D = np.stack([B.D[j][side] for j in js])    # (n, k, l, m)
            Qt = np.stack([B.Qt[j][side] for j in js])  # (n, m, l, k)
            # momentum rows (a, c, k), stress columns (A, s, m): -dt w_a D[k, l, m] for s = vo[c, l]
            blk = np.einsum("aA,cls,nklm->nackAsm", Iw, P, D).reshape(len(js), nvl, nsl)
            emit(el * nvl, nv + js * nsl, blk)
            # stress rows (a, s, m), velocity columns (A, c, k): -dt w_a sum_l Ev[s, c, l] Qt[m, l, k]
            blk = np.einsum("aA,nscl,nmlk->nasmAck", Iw, Ev[js], Qt).reshape(len(js), nsl, nvl)
            emit(nv + js * nsl, el * nvl, blk)
        n = nv + self.ns
        self.A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                               shape=(n, n))

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
        self._schur_parts = (S.tocsr(), Avs.tocsr(), Asv, Ainv)
        return self._schur_parts[0]

    def _element_neighbours(self):
        nb = [set() for _ in range(self.ne)]
        for F in self.B.topo.faces:
            if F.right >= 0 and F.right != F.left:
                nb[F.left].add(F.right)
                nb[F.right].add(F.left)
        return nb

    def block_jacobi(self):
        """Pre1 of Appendix A (eq. pre1): the inverses of the element diagonal
        blocks of the velocity operator, as a block-diagonal sparse matrix."""
        S = self._schur_parts[0] if getattr(self, "_schur_parts", None) is not None else self.schur()
        nb = self.ng * self.d * self.nphi
        blocks = [np.linalg.inv(S[i * nb:(i + 1) * nb, i * nb:(i + 1) * nb].toarray()) for i in range(self.ne)]
        return sp.block_diag(blocks, format="csr")

    def patch_preconditioner(self):
        """Pre2 of Appendix A (eqs. APPRE1, APPRE2): for each element i the
        velocity operator restricted to the stencil S_i of i and its face
        neighbours (diagonal blocks D and neighbour blocks N), inverted; the
        block row of element i of that inverse gives (P x)_i = sum_e
        A_i^-1(0, e) x_g(e).  Returned as a sparse matrix P."""
        S = self._schur_parts[0] if getattr(self, "_schur_parts", None) is not None else self.schur()
        S = S.tocsr()
        nb = self.ng * self.d * self.nphi
        nbrs = self._element_neighbours()
        rows, cols, vals = [], [], []
        for i in range(self.ne):
            st = [i] + sorted(nbrs[i])
            idx = np.concatenate([np.arange(e * nb, (e + 1) * nb) for e in st])
            Ainv = np.linalg.inv(S[idx][:, idx].toarray())
            rows.append(np.repeat(np.arange(i * nb, (i + 1) * nb), len(idx)))
            cols.append(np.tile(idx, nb))
            vals.append(Ainv[:nb].ravel())
        n = self.nv
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))

    def step_schur(self, v_old, s_old_raw, sources=None, rtol=1e-10, maxiter=100000):
        """The same step as step(), computed the way Section 4 describes:
        eliminate the stress (eq. velocity.sys, or velocity.sys.cn), solve the
        velocity system with a Krylov method (SciPy CG for Crank-Nicolson,
        whose system is SPD by Section 5; GMRES otherwise) to relative
        residual rtol from the old state copied to every time node, then
        back-substitute the stress (eq. NM26 / NM26.cn).

        Returns (v_slab, s_slab_raw, v_end, s_end_raw, iterations)."""
        if getattr(self, "_schur_parts", None) is None:
            self.schur()
        S, Avs, Asv, Ainv = self._schur_parts
        nv = self.nv
        b = self.rhs(v_old, s_old_raw, sources)
        bv = b[:nv] - Avs @ (Ainv @ b[nv:])
        x0 = np.repeat(v_old[:, None], self.ng, axis=1).reshape(-1)
        its = [0]

        def count(*_):
            its[0] += 1

        if self.scheme == "cn":
            v, info = spla.cg(S, bv, x0=x0, rtol=rtol, atol=0.0, maxiter=maxiter, callback=count)
        else:
            v, info = spla.gmres(S, bv, x0=x0, rtol=rtol, atol=0.0, restart=30, maxiter=maxiter,
                                 callback=count, callback_type="pr_norm")
        if info != 0:
            raise RuntimeError(f"Krylov solve did not converge (info {info})")
        sg = Ainv @ (b[nv:] - Asv @ v)
        v = v.reshape(self.ne, self.ng, self.d, self.nphi)
        sg = sg.reshape(self.nf, self.ng, self.nsig, self.npsi)
        if self.scheme == "cn":
            return v, sg, v[:, 0].copy(), sg[:, 0].copy(), its[0]
        e1 = self.tb.e1
        return v, sg, np.einsum("a,eack->eck", e1, v), np.einsum("a,jasm->jsm", e1, sg), its[0]

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
            e = B.locate(x)
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
        v_old[e][c][k] and raw stress s_old_raw[j][s][m]).

        Space-time: rho_i (e0 (x) Mbar_i) v_old_i and (e0 (x) M_j) sigma_old_j,
        the old-slab terms of eqs. (NM25), (NM26) with Mbar^-, M^- of eq.
        (MD_2_1).  Crank-Nicolson: rho_i Mbar_i v^n and M_j sigma^n plus the
        explicit halves of the coupling terms of eqs. (NM25.cn), (NM26.cn)."""
        B = self.B
        nv = self.nv
        b = np.zeros(nv + self.ns)
        # (rho_i Mbar_i v_old_i)[c][k] and (M_j sigma_old_j)[s][m]
        mv = np.einsum("e,ekl,ecl->eck", B.rho, np.asarray(B.Mbar), v_old)
        ms = np.einsum("jmn,jsn->jsm", np.asarray(B.M), s_old_raw)
        e0 = np.array([1.0]) if self.scheme == "cn" else self.tb.e0
        bv = b[:nv].reshape(self.ne, self.ng, self.d, self.nphi)
        bs = b[nv:].reshape(self.nf, self.ng, self.nsig, self.npsi)
        bv[:] = e0[None, :, None, None] * mv[:, None, :, :]
        bs[:] = e0[None, :, None, None] * ms[:, None, :, :]
        if self.scheme == "cn":
            # explicit half of the coupling terms: minus the off-diagonal blocks times the old state
            b[:nv] -= self.A[:nv, nv:] @ s_old_raw.reshape(-1)
            b[nv:] -= self.A[nv:, :nv] @ v_old.reshape(-1)
        b[:nv] += self.source_term(sources)
        return b

    def solve(self, b):
        # sparse direct LU of the coupled slab matrix, factored once.  The
        # column ordering only changes fill: minimum degree on A^T + A gives
        # about 5x less fill than COLAMD on the 2D meshes, COLAMD about 2.5x
        # less than minimum degree on the periodic tetrahedral ones.
        if self._lu is None:
            spec = "MMD_AT_PLUS_A" if self.d == 2 else "COLAMD"
            self._lu = spla.splu(self.A.tocsc(), permc_spec=spec)
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
            x, w, xi = B.elem_rule(i, 2 * B.p)
            val = basis_at_ref(B.lb, B.maps[i], xi)[0] @ v[i].T
            ek += 0.5 * B.rho[i] * np.sum(w[:, None] * val * val)
        es = 0.0
        psi_deg = 2 * B.p if d == 2 else B.p
        for j, F in enumerate(B.topo.faces):
            C = B.face_compliance(j)
            for side in ([0] if F.right < 0 else [0, 1]):
                x, w, _ = B.sub_rule(j, side, 2 * psi_deg)
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
