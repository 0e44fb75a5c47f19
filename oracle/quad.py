"""Exact quadrature on intervals and reference simplices (oracle).

Collapsed-coordinate rules: the reference simplex is the image of the unit
cube under the Duffy map, and the Jacobian factors (1-v) and (1-w)^2 are
absorbed into Gauss-Jacobi weights.  A rule built for degree q integrates
every polynomial of total degree <= q exactly, which is what the block
integrals of eqs. (MD_2)-(MD_6) need on the affine sub-simplices of
Section 3.
"""
from __future__ import annotations

import functools

import numpy as np
from scipy.special import roots_jacobi


def gauss_legendre_01(n: int):
    """n-point Gauss-Legendre rule on [0, 1] (exact to degree 2n-1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _gauss_jacobi_01(n: int, alpha: int):
    """Rule for int_0^1 g(v) (1-v)^alpha dv, exact for deg g <= 2n-1."""
    x, w = roots_jacobi(n, alpha, 0.0)
    return 0.5 * (x + 1.0), w / 2.0 ** (alpha + 1)


def n_points(degree: int) -> int:
    return max(1, (degree + 2) // 2)


@functools.lru_cache(maxsize=None)
def reference_rule(dim: int, degree: int):
    """Points (npts, dim) and weights on the reference simplex
    {x_i >= 0, sum x_i <= 1}; exact for total degree <= ``degree``.
    Built once per (dim, degree); the returned arrays are read-only."""
    pts, w = _reference_rule(dim, degree)
    pts.setflags(write=False)
    w.setflags(write=False)
    return pts, w


def _reference_rule(dim: int, degree: int):
    n = n_points(degree)
    if dim == 1:
        x, w = gauss_legendre_01(n)
        return x[:, None], w
    if dim == 2:
        u, wu = gauss_legendre_01(n)
        v, wv = _gauss_jacobi_01(n, 1)
        U, V = np.meshgrid(u, v, indexing="ij")
        W = np.outer(wu, wv)
        pts = np.stack([U * (1.0 - V), V], axis=-1).reshape(-1, 2)
        return pts, W.ravel()
    if dim == 3:
        u, wu = gauss_legendre_01(n)
        v, wv = _gauss_jacobi_01(n, 1)
        s, ws = _gauss_jacobi_01(n, 2)
        U, V, S = np.meshgrid(u, v, s, indexing="ij")
        W = wu[:, None, None] * wv[None, :, None] * ws[None, None, :]
        pts = np.stack([U * (1 - V) * (1 - S), V * (1 - S), S], axis=-1).reshape(-1, 3)
        return pts, W.ravel()
    raise ValueError(dim)


def simplex_rule(verts: np.ndarray, degree: int):
    """Rule on the affine simplex with vertex rows ``verts`` (k+1, d).

    k = number of rows - 1 is the simplex dimension (k <= d); the weight
    includes the k-dimensional volume factor, so faces embedded in
    d-space are handled too.
    """
    verts = np.asarray(verts, float)
    k = verts.shape[0] - 1
    ref, w = reference_rule(k, degree)
    J = (verts[1:] - verts[0]).T  # (d, k)
    pts = verts[0][None, :] + ref @ J.T
    if J.shape[0] == k:
        vol = abs(np.linalg.det(J))
    else:
        vol = np.sqrt(abs(np.linalg.det(J.T @ J)))
    return pts, w * vol


def mapped_rule(cmap, ref_verts: np.ndarray, degree: int):
    """Rule on the image under the element map ``cmap`` (x(xi), jac(xi)) of
    the reference sub-simplex with vertex rows ``ref_verts`` (d+1, d), exact
    for integrands of total degree <= ``degree`` in the reference
    coordinates (the weights include |det J(xi)|).  Returns (x, w, xi)."""
    ref_verts = np.asarray(ref_verts, float)
    d = ref_verts.shape[1]
    r, w = reference_rule(d, degree)
    A = (ref_verts[1:] - ref_verts[0]).T
    xi = ref_verts[0][None, :] + r @ A.T
    detJ = np.abs(np.linalg.det(cmap.jac(xi)))
    return cmap.x(xi), w * abs(np.linalg.det(A)) * detJ, xi
