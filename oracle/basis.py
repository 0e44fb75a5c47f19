"""Basis functions (oracle).

Velocity (Section 3, "space-time basis functions"): the nodal basis of
conforming P_p finite elements on the reference simplex, i.e. Lagrange
polynomials through the equispaced nodes, built here by inverting the
monomial Vandermonde matrix.  Node order (the velocity DOF order at the
library boundary):
    2D: for j in 0..p, for i in 0..p-j: (i, j)/p
    3D: for k, for j, for i with i+j+k <= p: (i, j, k)/p

Time (same paragraph): Lagrange polynomials through the N_gamma = p_gamma+1
Gauss-Legendre points of [0, 1], which makes the time mass matrix diagonal.

Stress (dual mesh):
  2D: the paper uses the (p+1)^2 tensor-product functions of the unit square
      mapped to the quadrilateral dual element.  The oracle uses the span of
      xi^a eta^b (a, b <= p) in the affine frame x = n1 + xi e1 + eta e2 with
      e1 = (d1 - d2)/2, e2 = (d1 + d2)/2, d1 = n2 - n1 (the face, n1 the
      vertex with the smaller global index) and d2 = b_r - b_l (the segment
      joining the two barycentres; on a boundary face b_r is b_l mirrored
      through the face midpoint).  When the dual quadrilateral is a
      parallelogram this frame is exactly the paper's bilinear (then
      affine) map, with the corners n1, b_l, n2, b_r.  Raw order: lexicographic
      in (a, b), a major.
  3D: the rescaled Taylor monomials of the paper, i.e. P_p in physical
      coordinates.  Raw order: by total degree, then exponents
      (a, b, c) of x^a y^b z^c with a descending, then b descending.
The canonical (orthonormal) dual basis used for stress DOFs at the library
boundary is the Gram-Schmidt orthonormalisation of the raw sequence over the
dual element (Cholesky of the exact Gram matrix).  It depends only on the
nested spans of the raw sequence, so any raw basis with the same frame and
ordering gives the same canonical functions.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from .quad import gauss_legendre_01


def n_phi(dim: int, p: int) -> int:
    return math.comb(p + dim, dim)


def n_psi(dim: int, p: int) -> int:
    return (p + 1) ** 2 if dim == 2 else math.comb(p + 3, 3)


def _all_exponents(dim: int, p: int):
    return [e for e in itertools.product(range(p + 1), repeat=dim) if sum(e) <= p]


def lagrange_nodes(dim: int, p: int) -> np.ndarray:
    if p == 0:
        return np.full((1, dim), 1.0 / (dim + 1))
    out = []
    if dim == 2:
        for j in range(p + 1):
            for i in range(p + 1 - j):
                out.append((i / p, j / p))
    elif dim == 3:
        for k in range(p + 1):
            for j in range(p + 1 - k):
                for i in range(p + 1 - k - j):
                    out.append((i / p, j / p, k / p))
    else:
        raise ValueError(dim)
    return np.array(out)


class LagrangeBasis:
    """Nodal P_p basis on the reference simplex."""

    def __init__(self, dim: int, p: int):
        self.dim, self.p = dim, p
        self.exps = _all_exponents(dim, p)
        self.nodes = lagrange_nodes(dim, p)
        V = self._mono(self.nodes)
        # phi_k(x) = sum_e C[e, k] x^e, with V C = I
        self.C = np.linalg.inv(V)
        self.n = len(self.exps)

    def _mono(self, x):
        x = np.atleast_2d(x)
        return np.stack([np.prod(x ** np.array(e)[None, :], axis=1) for e in self.exps], axis=1)

    def _dmono(self, x):
        x = np.atleast_2d(x)
        out = np.zeros((x.shape[0], self.dim, len(self.exps)))
        for q, e in enumerate(self.exps):
            for a in range(self.dim):
                if e[a] == 0:
                    continue
                ee = list(e)
                ee[a] -= 1
                out[:, a, q] = e[a] * np.prod(x ** np.array(ee)[None, :], axis=1)
        return out

    def eval(self, xi):
        """(npts, N_phi) values at reference points."""
        return self._mono(xi) @ self.C

    def grad(self, xi):
        """(npts, dim, N_phi) reference gradients."""
        return np.einsum("pae,ek->pak", self._dmono(xi), self.C)


class ElementMap:
    """Affine map x = V0 + J xi of a simplex with vertex rows V (d+1, d)."""

    def __init__(self, V):
        self.V = np.asarray(V, float)
        self.J = (self.V[1:] - self.V[0]).T
        self.Jinv = np.linalg.inv(self.J)
        self.detJ = abs(np.linalg.det(self.J))

    def to_ref(self, x):
        return (np.atleast_2d(x) - self.V[0][None, :]) @ self.Jinv.T


class CurvedMap:
    """Map of degree q of a curved element (Section 3, sub- or iso-parametric
    maps): x(xi) = sum_a X_a N_a(xi) with N_a the Lagrange basis of degree q
    on the reference simplex (nodes in the velocity node order) and X_a the
    given geometry nodes.  q = 1 is the affine map."""

    curved = True

    def __init__(self, X, q):
        self.X = np.asarray(X, float)
        self.q = q
        self.dim = self.X.shape[1]
        self.gb = LagrangeBasis(self.dim, q)
        if self.gb.n != self.X.shape[0]:
            raise ValueError("geometry nodes do not match the degree")
        corners = np.vstack([np.zeros(self.dim), np.eye(self.dim)])
        self.V = self.x(corners)

    def x(self, xi):
        return self.gb.eval(np.atleast_2d(xi)) @ self.X

    def jac(self, xi):
        """(npts, d, d): J[p, c, a] = d x_c / d xi_a."""
        return np.einsum("pak,kc->pca", self.gb.grad(np.atleast_2d(xi)), self.X)

    def to_ref(self, x, tol=1e-14, maxit=50):
        """Reference points of physical points x (Newton from the affine guess)."""
        x = np.atleast_2d(np.asarray(x, float))
        A = (self.V[1:] - self.V[0]).T
        xi = np.linalg.solve(A, (x - self.V[0][None, :]).T).T
        for _ in range(maxit):
            r = self.x(xi) - x
            step = np.linalg.solve(self.jac(xi), r[..., None])[..., 0]
            xi = xi - step
            if np.max(np.abs(step)) <= tol:
                break
        return xi


def basis_at_ref(lb: LagrangeBasis, emap, xi):
    """Values (npts, N_phi) and physical gradients (npts, d, N_phi) of the
    velocity basis of element ``emap`` (affine or curved) at reference points."""
    xi = np.atleast_2d(xi)
    val = lb.eval(xi)
    g_ref = lb.grad(xi)
    if getattr(emap, "curved", False):
        Jinv = np.linalg.inv(emap.jac(xi))                     # (npts, a, c)
        g = np.einsum("pba,pbk->pak", Jinv, g_ref)
    else:
        g = np.einsum("ba,pbk->pak", emap.Jinv, g_ref)      # d/dx_a = sum_b Jinv[b,a] d/dxi_b
    return val, g


def phys_basis(lb: LagrangeBasis, emap, x):
    """Values (npts, N_phi) and physical gradients (npts, d, N_phi) of the
    velocity basis of the element ``emap`` at physical points ``x``."""
    return basis_at_ref(lb, emap, emap.to_ref(x))


# ---------------------------------------------------------------- time basis


class TimeBasis:
    """Lagrange basis through the Gauss-Legendre points of [0, 1].

    Attributes
      tau, w   nodes and weights (ascending)
      T        T[a,b] = g_a(1) g_b(1) - int_0^1 g_a'(t) g_b(t) dt, the time
               factor of M = M^+ - M^o of eqs. (MD_2)-(MD_2_3)
      e0, e1   g(0) and g(1)
    """

    def __init__(self, p_gamma: int):
        n = p_gamma + 1
        self.n = n
        self.tau, self.w = gauss_legendre_01(n)
        self.polys = []
        for a in range(n):
            others = np.delete(self.tau, a)
            c = np.poly1d([1.0])
            for t in others:
                c = c * np.poly1d([1.0, -t]) / (self.tau[a] - t)
            self.polys.append(c)
        self.e0 = np.array([P(0.0) for P in self.polys])
        self.e1 = np.array([P(1.0) for P in self.polys])
        tq, wq = gauss_legendre_01(n + 2)
        G = np.array([[P(t) for t in tq] for P in self.polys])
        dG = np.array([[P.deriv()(t) for t in tq] for P in self.polys])
        Mo = (dG * wq[None, :]) @ G.T
        self.T = np.outer(self.e1, self.e1) - Mo
        self.W = np.diag(self.w)

    def eval(self, t):
        return np.array([P(t) for P in self.polys])


# ---------------------------------------------------------------- dual basis


def dual_exponents(dim: int, p: int):
    if dim == 2:
        return [(a, b) for a in range(p + 1) for b in range(p + 1)]
    out = []
    for deg in range(p + 1):
        for a in range(deg, -1, -1):
            for b in range(deg - a, -1, -1):
                out.append((a, b, deg - a - b))
    return out


class DualRawBasis:
    """Raw (non-orthonormal) dual basis of one dual element.

    2D: monomials (2 xi - 1)^a (2 eta - 1)^b in the frame (origin n1, axes
        e1, e2); the affine shift keeps the nested spans of xi^a eta^b.
    3D: monomials ((x - c)/h)^alpha with c the dual element centroid and h
        a length scale (neither changes the canonical basis).
    ``mix`` (optional, n x n upper triangular): the basis is the monomials
        times mix, i.e. function i is a combination of monomials 0..i, which
        keeps the nested spans.
    """

    def __init__(self, dim: int, p: int, origin, axes=None, scale=1.0, mix=None):
        self.dim, self.p = dim, p
        self.mix = mix
        self.exps = dual_exponents(dim, p)
        self.origin = np.asarray(origin, float)
        if dim == 2:
            A = np.asarray(axes, float).T  # columns e1, e2
            self.Ainv = np.linalg.inv(A)
        else:
            self.Ainv = np.eye(3) / scale
        self.n = len(self.exps)

    def coords(self, x):
        y = (np.atleast_2d(x) - self.origin[None, :]) @ self.Ainv.T
        if self.dim == 2:
            # centre the frame coordinates on [-1, 1] (same nested spans,
            # better conditioned Gram matrices)
            y = 2.0 * y - 1.0
        return y

    def eval(self, x):
        y = self.coords(x)
        mono = np.stack([np.prod(y ** np.array(e)[None, :], axis=1) for e in self.exps], axis=1)
        return mono if self.mix is None else mono @ self.mix
