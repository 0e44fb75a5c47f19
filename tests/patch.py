"""Rows of the oracle's slab system for one element of a mesh too large to
assemble whole.

The stress mass T (x) M_j is block diagonal over the faces (Section 4, eq.
MD_2), so the velocity Schur complement of eq. (velocity.sys) couples an
element only to itself and to the elements across its faces, through the
faces' own blocks.  The rows of element i (and its columns) are therefore
those of the oracle built on the patch made of i and its face neighbours:
every block they involve (M_bar_i, D_ij, Qt_ij, M_j and the dual-element
material of each face j of i) depends only on the geometry and material of
i and of the element across j.  Patch elements keep their global order and
vertex ids, so left/right sides, local face indices and the raw dual bases
of the faces of i are the same as in the whole mesh.
tests/test_oracle_patch.py pins this against the whole-mesh oracle.
"""
from __future__ import annotations

import numpy as np

from oracle.assemble import Blocks
from oracle.mesh import Topology
from oracle.slab import Slab


class Patch:
    def __init__(self, mesh, i, p, p_gamma, dt, scheme, lam, mu, rho):
        elem = np.asarray(mesh.elem)
        d = elem.shape[1] - 1
        shared = np.isin(elem, elem[i]).sum(axis=1)
        self.elems = np.nonzero(shared >= d)[0]          # i and the elements across its faces
        self.li = int(np.searchsorted(self.elems, i))
        topo = Topology(mesh.xyz, elem[self.elems], mesh.period)
        self.B = Blocks(topo, p, np.asarray(lam)[self.elems], np.asarray(mu)[self.elems],
                        np.asarray(rho)[self.elems])
        self.slab = Slab(self.B, p_gamma, dt, scheme)
        s = self.slab
        self.blk = s.ng * s.d * s.nphi
        self.sblk = s.ng * s.nsig * s.npsi
        self.faces = [int(j) for j in topo.elem_faces[self.li]]
        self.d = d
        interior = sum(1 for j in self.faces if topo.faces[j].right >= 0)
        if interior != len(self.elems) - 1:
            raise ValueError("patch neighbours do not match the faces of the element")

    # ---------------------------------------------------------------- rows
    def vrows(self):
        return slice(self.li * self.blk, (self.li + 1) * self.blk)

    def gather_v(self, v_global):
        """Patch velocity vector from a global one in [elem][a][c][k] layout."""
        return np.asarray(v_global).reshape(-1, self.blk)[self.elems].ravel()

    def schur_row(self, v_global, S=None):
        S = self.slab.schur() if S is None else S
        return (S @ self.gather_v(v_global))[self.vrows()]

    def schur_col(self, w_global, S=None):
        S = self.slab.schur() if S is None else S
        return (S.T @ self.gather_v(w_global))[self.vrows()]

    # ---------------------------------------------------------------- faces
    def global_faces(self, face_code):
        """Global ids of the faces of i: faces are numbered in ascending
        (left element, local face) order, the left element being the lower
        index; face_code is that sorted list of left * (d + 1) + lf."""
        out = []
        for j in self.faces:
            F = self.B.topo.faces[j]
            code = int(self.elems[F.left]) * (self.d + 1) + F.lf
            g = int(np.searchsorted(face_code, code))
            if g >= len(face_code) or face_code[g] != code:
                raise ValueError("face not found in the global face list")
            out.append(g)
        return out

    def coupled_residual(self, v_slab, s_slab_can, v_old, s_old_can, face_code):
        """Residual b - A x of the coupled slab system (eqs. NM25, NM26 or
        their Crank-Nicolson forms) on the momentum rows of i and the stress
        rows of its faces, for global slab DOFs v_slab [e][a][c][k] and
        s_slab_can [face][a][s][m] in the canonical (orthonormal) dual basis,
        and the old end-of-slab state v_old [e][c][k], s_old_can [face][s][m].
        Stress of patch faces that are not faces of i stays zero: no row
        returned here reads it.  Returns (momentum residual, momentum rhs,
        [(stress residual, stress rhs) per face of i])."""
        s, B = self.slab, self.B
        gf = self.global_faces(face_code)
        ng, nsig, npsi = s.ng, s.nsig, s.npsi
        x = np.zeros(s.nv + s.ns)
        x[:s.nv] = self.gather_v(v_slab)
        s_old = np.zeros((s.nf, nsig, npsi))
        sv = np.asarray(s_slab_can).reshape(-1, ng * nsig, npsi)
        so = np.asarray(s_old_can).reshape(-1, nsig, npsi)
        for j, g in zip(self.faces, gf):
            x[s.si(j, 0, 0, 0):s.si(j, 0, 0, 0) + self.sblk] = B.from_canonical(j, sv[g]).ravel()
            s_old[j] = B.from_canonical(j, so[g])
        v_old_p = np.asarray(v_old).reshape(-1, s.d, s.nphi)[self.elems]
        b = s.rhs(v_old_p, s_old)
        r = b - s.A @ x
        vr = self.vrows()
        faces = []
        for j in self.faces:
            sl = slice(s.si(j, 0, 0, 0), s.si(j, 0, 0, 0) + self.sblk)
            faces.append((r[sl], b[sl]))
        return r[vr], b[vr], faces


def face_codes(elem):
    """Sorted left * (d + 1) + lf codes of all faces of a conforming
    (possibly periodic, vertex ids identified) simplex mesh."""
    elem = np.asarray(elem, dtype=np.int64)
    ne, nv = elem.shape
    keys = np.empty((ne * nv, nv - 1), dtype=np.int64)
    for f in range(nv):
        keys[f::nv] = np.sort(np.delete(elem, f, axis=1), axis=1)
    _, inv = np.unique(keys, axis=0, return_inverse=True)
    inv = inv.ravel()
    owner = np.full(inv.max() + 1, ne * nv, dtype=np.int64)
    codes = np.arange(ne * nv, dtype=np.int64)        # e * nv + f, ascending in (e, f)
    np.minimum.at(owner, inv, codes)
    return np.sort(owner)
