"""Element and face blocks of the scheme (oracle), eqs. (MD_2)-(MD_6).

All integrals use the exact rules of ``quad`` in physical coordinates, with
the stress basis in its *raw* form (``basis.DualRawBasis``), so the dual mass
matrices M_j are full.  The canonical orthonormal dual basis is only used to
translate stress DOFs at the boundary with the library.

Readings of the paper taken here:
  * Free-surface (boundary) faces: the dual element is T_{l,j} alone and the
    face integral over Gamma_j is dropped from D and Q (traction-free
    natural condition, sigma.n = 0).
  * Material: rho_i constant per element; E_j constant per dual element with
    the volume-weighted means lambda_j = (|T_l,j| lambda_l + |T_r,j| lambda_r)
    / |R_j| (and likewise mu_j), i.e. the L2 projection onto constants.
"""
from __future__ import annotations

import numpy as np

from . import quad
from .basis import (CurvedMap, DualRawBasis, ElementMap, LagrangeBasis,
                    basis_at_ref, n_phi, n_psi, phys_basis)
from .mesh import Topology


def voigt_index(dim: int):
    """vo[c][l]: Voigt component of the symmetric tensor entry (c, l).
    2D (xx, yy, xy); 3D (xx, yy, zz, yz, xz, xy), Section 2."""
    if dim == 2:
        return np.array([[0, 2], [2, 1]])
    return np.array([[0, 5, 4], [5, 1, 3], [4, 3, 2]])


def n_sigma(dim: int) -> int:
    return dim * (dim + 1) // 2


def stiffness(dim, lam, mu):
    """E[p,q,c,l] of the isotropic Hooke law, eq. (1.1b):
    sigma_pq = lambda div(v) delta_pq + mu (d_q v_p + d_p v_q),
    written as sigma_pq = sum_cl E[p,q,c,l] d_l v_c."""
    I = np.eye(dim)
    return (lam * np.einsum("pq,cl->pqcl", I, I)
            + mu * (np.einsum("pc,ql->pqcl", I, I) + np.einsum("pl,qc->pqcl", I, I)))


def voigt_weights(dim):
    """W: 1 on normal, 2 on shear Voigt components, so that the tensor
    contraction sigma : eps equals s^T W e for the Voigt vectors (Section 2
    lists each shear component once)."""
    return np.array([1.0] * dim + [2.0] * (n_sigma(dim) - dim))


def stiffness_from_voigt(dim, Et):
    """E[p,q,c,l] (sigma_pq = sum_cl E[p,q,c,l] d_l v_c) of a general
    material given by the matrix E~ of Section 2, s~ = E~ e~, where the strain
    rate's Voigt entry for (c, l) is (d_l v_c + d_c v_l) / 2.  Each Voigt
    column (c, l), c < l, contributes half to d_l v_c and half to d_c v_l;
    a normal column (c, c) contributes fully to d_c v_c."""
    vo = voigt_index(dim)
    Et = np.asarray(Et, float)
    E = np.zeros((dim, dim, dim, dim))
    for p in range(dim):
        for q in range(dim):
            for c in range(dim):
                for l in range(c, dim):
                    e = Et[vo[p, q], vo[c, l]]
                    if c == l:
                        E[p, q, c, c] += e
                    else:
                        E[p, q, c, l] += 0.5 * e
                        E[p, q, l, c] += 0.5 * e
    return E


def compliance_voigt(dim, lam, mu):
    """C with sigma : E^{-1} sigma = s^T C s for the Voigt vector s.

    3D: the inverse of the paper's 6x6 stiffness (eq. 5) with the factor 2
    on shear entries that turns the Voigt product into the tensor product.
    2D plane strain: the 3x3 restriction of the stiffness (normal block
    [[l+2m, l], [l, l+2m]], shear 2m), inverted the same way.
    """
    if dim == 3:
        Et = np.zeros((6, 6))
        Et[:3, :3] = lam
        Et[np.arange(3), np.arange(3)] = lam + 2 * mu
        Et[np.arange(3, 6), np.arange(3, 6)] = 2 * mu
        Wt = np.diag([1, 1, 1, 2, 2, 2.0])
    else:
        Et = np.array([[lam + 2 * mu, lam, 0], [lam, lam + 2 * mu, 0], [0, 0, 2 * mu]])
        Wt = np.diag([1, 1, 2.0])
    return Wt @ np.linalg.inv(Et)


def compliance_from_voigt(dim, Et):
    """C with sigma : E^{-1} sigma = s^T C s for a general E~ (Section 2):
    the strain is e~ = E~^{-1} s~ and the contraction sigma : eps is
    s~^T W e~, so C = W E~^{-1}."""
    return np.diag(voigt_weights(dim)) @ np.linalg.inv(np.asarray(Et, float))


class Blocks:
    """All blocks of one mesh / degree pair.

    Mbar[e]      (N_phi, N_phi)       int_{T_e} phi_k phi_m        (MD_2, spatial part)
    M[j]         (N_psi, N_psi)       int_{R_j} psi_k psi_m        (MD_2, spatial part)
    D[j][s]      (N_phi, d, N_psi)    int_G phi_k psi_m n_{i,j} - int_{T_ij} d_l phi_k psi_m   (MD_3)
    Qt[j][s]     (N_psi, d, N_phi)    int_{T_ij} psi d_l phi - int_G psi phi s_ij n_j          (qtilde)
    L[j]         Cholesky factor of M[j]: canonical coefficients = L^T raw coefficients
    lam_j, mu_j  dual-element material (isotropic)
    Et_j         dual-element Voigt stiffness E~_j (anisotropic), else None

    ``stiffness`` (n_elem, n_sigma, n_sigma), when given, is a general
    material per element in the Voigt form of Section 2; lam and mu are then
    ignored.  E~_j is the volume-weighted mean over R_j, like lambda_j.

    ``curved`` = (element ids, geometry nodes (n_c, N_q, d)) gives curved
    elements (Section 3: sub-/iso-parametric maps of degree q, 2D): their
    velocity basis is the reference basis composed with the inverse map,
    their barycentre and sub-simplices T_{i,j} are the images of the
    reference ones, and every integral over them is taken in reference
    coordinates with |det J|.  Their faces shared with other elements must
    be straight (geometry nodes at the affine positions); boundary faces may
    be curved.
    """

    def __init__(self, topo: Topology, p: int, lam, mu, rho, stiffness=None, curved=None):
        self.topo = topo
        d = self.dim = topo.dim
        self.p = p
        self.lb = LagrangeBasis(d, p)
        self.nphi = n_phi(d, p)
        self.npsi = n_psi(d, p)
        self.nsig = n_sigma(d)
        self.rho = np.asarray(rho, float)
        if stiffness is not None:   # isotropic parameters unused: NaN makes any use loud
            lam = mu = np.full(topo.n_elem, np.nan)
        lam = np.asarray(lam, float)
        mu = np.asarray(mu, float)
        psi_deg = 2 * p if d == 2 else p

        self.maps = [ElementMap(topo.V[e]) for e in range(topo.n_elem)]
        self.curved = {}
        if curved is not None:
            self._set_curved(*curved)
        self.bary = np.array([self.maps[e].x(np.full((1, d), 1.0 / (d + 1)))[0] if e in self.curved
                              else topo.V[e].mean(axis=0) for e in range(topo.n_elem)])
        self.Mbar = []
        for e in range(topo.n_elem):
            x, w, xi = self.elem_rule(e, 2 * p)
            phi, _ = basis_at_ref(self.lb, self.maps[e], xi)
            self.Mbar.append((phi * w[:, None]).T @ phi)

        self.duals, self.M, self.L, self.D, self.Qt = [], [], [], [], []
        self.lam_j = np.zeros(topo.n_face)
        self.mu_j = np.zeros(topo.n_face)
        self.vol_sub = np.zeros((topo.n_face, 2))
        for j, F in enumerate(topo.faces):
            sides = [0] if F.right < 0 else [0, 1]
            psi = self._dual_basis(F)
            self.duals.append(psi)
            G = np.zeros((self.npsi, self.npsi))
            Dj, Qj = [], []
            for s in sides:
                e = F.left if s == 0 else F.right
                emap = self.maps[e] if (s == 0 or e in self.curved) else ElementMap(F.Vr)
                x, w, _ = self.sub_rule(j, s, 2 * psi_deg)
                pv = psi.eval(x)
                G += (pv * w[:, None]).T @ pv
                self.vol_sub[j, s] = w.sum()
                # volume parts (a curved side integrates d_l phi through its
                # map: the rule is exact for J^-1 |det J| = adj J)
                x, w, xi = self.sub_rule(j, s, max(p - 1, 0) + psi_deg, extra=-1)
                pv = psi.eval(x)
                if e in self.curved:
                    _, gphi = basis_at_ref(self.lb, emap, xi)
                else:
                    _, gphi = phys_basis(self.lb, emap, x)
                Dv = -np.einsum("q,qlk,qm->klm", w, gphi, pv)
                Qv = np.einsum("q,qm,qlk->mlk", w, pv, gphi)
                if F.right >= 0:
                    x, w = quad.simplex_rule(F.X, p + psi_deg)
                    pv = psi.eval(x)
                    phi, _ = phys_basis(self.lb, emap, x)
                    sgn = 1.0 if s == 0 else -1.0
                    n_ij = sgn * F.normal
                    Df = np.einsum("q,qk,qm,l->klm", w, phi, pv, n_ij)
                    Qf = -sgn * np.einsum("q,qm,qk,l->mlk", w, pv, phi, F.normal)
                    Dv = Dv + Df
                    Qv = Qv + Qf
                Dj.append(Dv)
                Qj.append(Qv)
            self.M.append(G)
            self.L.append(np.linalg.cholesky(G))
            self.D.append(Dj)
            self.Qt.append(Qj)
            vl = self.vol_sub[j, 0]
            if F.right >= 0:
                vr = self.vol_sub[j, 1]
                self.lam_j[j] = (vl * lam[F.left] + vr * lam[F.right]) / (vl + vr)
                self.mu_j[j] = (vl * mu[F.left] + vr * mu[F.right]) / (vl + vr)
            else:
                self.lam_j[j] = lam[F.left]
                self.mu_j[j] = mu[F.left]
        self.Et_j = None
        if stiffness is not None:
            Et = np.asarray(stiffness, float)
            self.Et_j = np.zeros((topo.n_face, self.nsig, self.nsig))
            for j, F in enumerate(topo.faces):
                vl = self.vol_sub[j, 0]
                if F.right >= 0:
                    vr = self.vol_sub[j, 1]
                    self.Et_j[j] = (vl * Et[F.left] + vr * Et[F.right]) / (vl + vr)
                else:
                    self.Et_j[j] = Et[F.left]

    def face_stiffness(self, j):
        """E[p,q,c,l] of dual element j."""
        if self.Et_j is not None:
            return stiffness_from_voigt(self.dim, self.Et_j[j])
        return stiffness(self.dim, self.lam_j[j], self.mu_j[j])

    def face_compliance(self, j):
        """Voigt compliance form C of dual element j (sigma : E^-1 sigma = s^T C s)."""
        if self.Et_j is not None:
            return compliance_from_voigt(self.dim, self.Et_j[j])
        return compliance_voigt(self.dim, self.lam_j[j], self.mu_j[j])

    # ------------------------------------------------------------ geometry

    def _set_curved(self, ids, nodes):
        topo, d = self.topo, self.dim
        if d != 2:
            raise ValueError("curved elements are 2D here")
        nodes = np.asarray(nodes, float)
        nq = nodes.shape[1]
        q = next(k for k in range(1, 12) if (k + 1) * (k + 2) // 2 == nq)
        corner = [0, q, nq - 1]            # node indices of xi = (0,0), (1,0), (0,1)
        for e, X in zip(np.asarray(ids), nodes):
            e = int(e)
            V = topo.V[e]
            h = np.max(np.abs(V[1:] - V[0]))
            if np.max(np.abs(X[corner] - V)) > 1e-12 * max(1.0, np.max(np.abs(V))):
                raise ValueError(f"curved element {e}: corner nodes differ from its vertices")
            cm = CurvedMap(X, q)
            self.maps[e] = cm
            self.curved[e] = cm
            # faces shared with another element must be straight
            aff = ElementMap(V)
            ref = cm.gb.nodes
            for f in range(d + 1):
                j = topo.elem_faces[e, f]
                if topo.faces[j].right < 0:
                    continue
                lam = np.column_stack([1.0 - ref.sum(axis=1), ref])
                on = np.abs(lam[:, f]) < 1e-12
                straight = V[0][None, :] + ref[on] @ aff.J.T
                if np.max(np.abs(X[on] - straight)) > 1e-12 * max(1.0, h):
                    raise ValueError(f"curved element {e}: interior face {j} is not straight")

    def _ref_sub(self, e, f):
        """Reference vertices of T_{e,j} for local face f of e: the face's
        reference vertices, then the reference barycentre."""
        d = self.dim
        corners = np.vstack([np.zeros(d), np.eye(d)])
        return np.vstack([corners[[a for a in range(d + 1) if a != f]], np.full((1, d), 1.0 / (d + 1))])

    def elem_rule(self, e, degree):
        """(x, w, xi) of a rule over element e exact for integrands of degree
        ``degree`` in physical coordinates (their composition with a curved
        map of degree q, times |det J|, in reference coordinates)."""
        cm = self.curved.get(e)
        d = self.dim
        if cm is None:
            x, w = quad.simplex_rule(self.topo.V[e], degree)
            return x, w, self.maps[e].to_ref(x)
        corners = np.vstack([np.zeros(d), np.eye(d)])
        return quad.mapped_rule(cm, corners, degree * cm.q + d * (cm.q - 1))

    def sub_rule(self, j, side, degree, extra=0):
        """(x, w, xi) of a rule over T_{i,j} (i the element of ``side``), exact
        like elem_rule; ``extra`` adjusts the degree added for |det J| (-1:
        an integrand carrying J^-1, whose product with |det J| is adj J)."""
        F = self.topo.faces[j]
        e = F.left if side == 0 else F.right
        cm = self.curved.get(e)
        d = self.dim
        if cm is None:
            b = F.bl if side == 0 else F.br
            x, w = quad.simplex_rule(np.vstack([F.X, b[None, :]]), degree)
            emap = self.maps[e] if side == 0 else ElementMap(F.Vr)
            return x, w, emap.to_ref(x)
        f = F.lf if side == 0 else F.rf
        jdeg = d * (cm.q - 1) if extra == 0 else (d - 1) * (cm.q - 1)
        return quad.mapped_rule(cm, self._ref_sub(e, f), degree * cm.q + jdeg)

    def face_bary(self, F):
        """Barycentres of the face's elements in the left frame (images of the
        reference barycentre for curved elements)."""
        bl = self.bary[F.left] if F.left in self.curved else F.bl
        if F.right < 0:
            return bl, None
        return bl, (self.bary[F.right] if F.right in self.curved else F.br)

    def locate(self, x, tol=1e-12):
        """Lowest element index whose closed element contains x."""
        x = np.asarray(x, float)
        for e in range(self.topo.n_elem):
            xi = self.maps[e].to_ref(x[None, :])[0]
            bary = np.concatenate([[1 - xi.sum()], xi])
            if np.all(bary >= -tol):
                return e
        return -1

    def _dual_basis(self, F):
        if self.dim == 2:
            n1, n2 = F.X[0], F.X[1]
            bl, br = self.face_bary(F)
            br = br if br is not None else (n1 + n2 - bl)
            d1 = n2 - n1
            d2 = br - bl
            return DualRawBasis(2, self.p, n1, axes=[(d1 - d2) / 2, (d1 + d2) / 2])
        pts = [F.X, F.bl[None, :]]
        if F.br is not None:
            pts.append(F.br[None, :])
        c = np.vstack(pts).mean(axis=0)
        h = np.max(np.linalg.norm(F.X - c[None, :], axis=1))
        mono = DualRawBasis(3, self.p, c, scale=h)
        # Gram-Schmidt of the monomial sequence over the dual element, taken
        # as a Householder QR of its weighted values at an exact rule
        # (A = Q R, basis = monomials R^-1): the monomial Gram matrices of
        # the tetrahedral dual elements reach cond 1e8 at p = 4, where a
        # Cholesky factor would lose half the digits
        xs, ws = [], []
        for Ts in ([np.vstack([F.X, F.bl[None, :]])] +
                   ([np.vstack([F.X, F.br[None, :]])] if F.br is not None else [])):
            x, w = quad.simplex_rule(Ts, 2 * self.p)
            xs.append(x)
            ws.append(w)
        A = np.sqrt(np.concatenate(ws))[:, None] * mono.eval(np.vstack(xs))
        R = np.linalg.qr(A, mode="r")
        R = R * np.sign(np.diag(R))[:, None]
        return DualRawBasis(3, self.p, c, scale=h, mix=np.linalg.inv(R))

    # ------------------------------------------------------------ evaluation

    def velocity_at(self, v_elem, e, x):
        """v_elem (d, N_phi) of element e evaluated at physical points x."""
        phi, _ = phys_basis(self.lb, self.maps[e], x)
        return phi @ v_elem.T

    def stress_at(self, s_raw, j, x):
        """s_raw (n_sigma, N_psi) raw stress DOFs of face j at points x."""
        return self.duals[j].eval(x) @ s_raw.T

    def to_canonical(self, j, s_raw):
        return s_raw @ self.L[j]

    def from_canonical(self, j, s_can):
        return np.linalg.solve(self.L[j].T, s_can.T).T


def locate(topo: Topology, x, tol=1e-12):
    """Brute-force point location: lowest element index whose closed simplex
    contains x (ties between elements go to the lowest index)."""
    for e in range(topo.n_elem):
        V = topo.V[e]
        J = (V[1:] - V[0]).T
        lam = np.linalg.solve(J, np.asarray(x, float) - V[0])
        bary = np.concatenate([[1 - lam.sum()], lam])
        if np.all(bary >= -tol):
            return e
    return -1
