"""Primary/dual mesh topology and geometry (oracle), Section 3.

Faces: local face f of a simplex is the face opposite its local vertex f.
For a face shared by two elements, the left element l(j) is the one with the
smaller index and the right element r(j) the other ("assigned arbitrarily" in
the paper; this fixes the choice).  A face with a single element is a
boundary face (free surface, sigma.n = 0).  Face j numbering: ascending
(l(j), local face index in l(j)).

Periodic meshes identify vertices on opposite sides; each element is
unwrapped by the minimum-image rule relative to its first vertex, and the
right element of a face across a periodic seam is translated so that it
touches the face as seen from the left element.  The dual element R_j is
the union of the sub-simplices T_{l,j} and T_{r,j} spanned by the face and
the barycentre of each element.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def unwrap(xyz, elem, period):
    V = np.asarray(xyz, float)[np.asarray(elem)]
    if period is None:
        return V
    P = np.asarray(period, float)
    out = V.copy()
    for e in range(V.shape[0]):
        for a in range(1, V.shape[1]):
            out[e, a] = V[e, a] + P * np.round((V[e, 0] - V[e, a]) / P)
    return out


@dataclass
class Face:
    left: int
    lf: int               # local face index in the left element
    right: int            # -1 on the boundary
    rf: int
    gverts: tuple         # global vertex ids, ascending
    X: np.ndarray         # (d, d) face vertex coords in the left frame, rows ordered as gverts
    Vl: np.ndarray        # (d+1, d) left element vertices
    Vr: np.ndarray | None # (d+1, d) right element vertices, translated into the left frame
    bl: np.ndarray
    br: np.ndarray | None
    normal: np.ndarray    # unit normal from left to right


class Topology:
    def __init__(self, xyz, elem, period=None):
        elem = np.asarray(elem, dtype=np.int64)
        self.dim = elem.shape[1] - 1
        self.n_elem = elem.shape[0]
        self.elem = elem
        self.V = unwrap(xyz, elem, period)
        d = self.dim
        for e in range(self.n_elem):
            J = (self.V[e, 1:] - self.V[e, 0]).T
            if abs(np.linalg.det(J)) < 1e-14 * np.max(np.abs(J)) ** d:
                raise ValueError(f"degenerate element {e}")
        table = {}
        for e in range(self.n_elem):
            for f in range(d + 1):
                key = tuple(sorted(int(elem[e, a]) for a in range(d + 1) if a != f))
                table.setdefault(key, []).append((e, f))
        faces = []
        for key, lst in table.items():
            if len(lst) > 2:
                raise ValueError("non-manifold face")
            lst.sort()
            (l, lf) = lst[0]
            if len(lst) == 2:
                (r, rf) = lst[1]
                if r == l:
                    raise ValueError("element shares a face with itself")
            else:
                r, rf = -1, -1
            faces.append(self._make_face(key, l, lf, r, rf))
        faces.sort(key=lambda F: (F.left, F.lf))
        self.faces = faces
        self.n_face = len(faces)
        # element -> face ids, per local face
        self.elem_faces = -np.ones((self.n_elem, d + 1), dtype=np.int64)
        for j, F in enumerate(faces):
            self.elem_faces[F.left, F.lf] = j
            if F.right >= 0:
                self.elem_faces[F.right, F.rf] = j

    def _local_index(self, e, gv):
        return [int(np.where(self.elem[e] == g)[0][0]) for g in gv]

    def _make_face(self, key, l, lf, r, rf):
        Vl = self.V[l]
        il = self._local_index(l, key)
        X = Vl[il]
        bl = Vl.mean(axis=0)
        Vr = br = None
        if r >= 0:
            ir = self._local_index(r, key)
            shift = X[0] - self.V[r][ir[0]]
            Vr = self.V[r] + shift[None, :]
            if np.max(np.abs(Vr[ir] - X)) > 1e-9 * max(1.0, np.max(np.abs(X))):
                raise ValueError("unmatched periodic face")
            br = Vr.mean(axis=0)
        n = self._normal(X)
        c = X.mean(axis=0)
        if np.dot(c - bl, n) < 0:
            n = -n
        return Face(l, lf, r, rf, tuple(key), X, Vl, Vr, bl, br, n)

    def _normal(self, X):
        if self.dim == 2:
            t = X[1] - X[0]
            n = np.array([t[1], -t[0]])
        else:
            n = np.cross(X[1] - X[0], X[2] - X[0])
        return n / np.linalg.norm(n)

    def sub_simplex(self, j, side):
        """Vertices of T_{i,j} (the face plus the barycentre of side i)."""
        F = self.faces[j]
        b = F.bl if side == 0 else F.br
        return np.vstack([F.X, b[None, :]])

    def volume(self, e):
        J = (self.V[e, 1:] - self.V[e, 0]).T
        return abs(np.linalg.det(J)) / np.prod(np.arange(1, self.dim + 1))
