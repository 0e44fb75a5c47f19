"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds *data only*: meshes (vertex coordinates and element
connectivity), per-element material parameters, source positions, source
time functions and receiver positions.  It contains none of the
discretisation's arithmetic (no bases, quadrature, blocks or solves), so
the CPU oracle and the HIP path can both consume its output without sharing
any code of the method.

All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).

Workload shapes follow the paper's tests: split-square triangulations of
the unit square (convergence test, Section 6.2), layered heterogeneous media
(the two-layer topography test, Section 6.4), Ricker point sources (tilted
Lamb problem, Section 6.3) and Kuhn-type tetrahedral cubes for the 3D runs
(Section 6.5).  The paper's own meshes are not available; these generators
stand in for them.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Mesh",
    "split_square",
    "kuhn_cube",
    "layered_material",
    "lognormal_material",
    "anisotropic_material",
    "homogeneous_material",
    "ricker",
    "random_points",
    "top_edge_receivers",
    "with_slivers",
    "inradius",
    "disk_mesh",
    "ragged_meshes",
    "workload",
]


@dataclass
class Mesh:
    """A simplex mesh given as plain arrays.

    ``xyz``      float64 (n_vert, dim) vertex coordinates.
    ``elem``     int64 (n_elem, dim+1) vertex indices of each simplex.
    ``period``   float64 (dim,) period lengths, or None for a non-periodic
                 mesh.  On a periodic mesh, vertices on opposite sides are
                 identified (stored once); element geometry is recovered by
                 the minimum-image convention relative to the element's
                 first vertex.
    """

    xyz: np.ndarray
    elem: np.ndarray
    period: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return int(self.xyz.shape[1])

    @property
    def n_elem(self) -> int:
        return int(self.elem.shape[0])

    @property
    def n_vert(self) -> int:
        return int(self.xyz.shape[0])

    def unwrapped_vertices(self) -> np.ndarray:
        """(n_elem, dim+1, dim) vertex coordinates with periodic unwrapping.

        This is input bookkeeping (which image of a vertex belongs to an
        element), not part of the discretisation.
        """
        v = self.xyz[self.elem]  # (E, d+1, d)
        if self.period is None:
            return v.copy()
        P = self.period[None, None, :]
        ref = v[:, :1, :]
        return v + P * np.round((ref - v) / P)

    def centroids(self) -> np.ndarray:
        return self.unwrapped_vertices().mean(axis=1)


def split_square(n: int, m: int | None = None, *, jitter: float = 0.0,
                 seed: int | None = None, periodic: bool = False,
                 lo=(0.0, 0.0), hi=(1.0, 1.0), diagonal: str = "/") -> Mesh:
    """n x m squares on [lo, hi], each split along the '/' diagonal (or the
    '\\' one with ``diagonal="\\"``).

    Vertices are numbered row-major with x fastest.  Square (i, j) with
    corners v00=(i,j), v10=(i+1,j), v11=(i+1,j+1), v01=(i,j+1) gives the two
    counter-clockwise triangles (v00, v10, v11) and (v00, v11, v01), in that
    order ('\\': (v00, v10, v01) and (v10, v11, v01)); squares are visited
    with i fastest.

    ``jitter`` moves every free vertex by i.i.d. U(-jitter, jitter) times the
    local spacing in each coordinate (boundary vertices stay fixed on a
    non-periodic mesh; on a periodic mesh every vertex moves).  Draws are
    taken for all vertices in vertex order, x then y, so the stream does not
    depend on which vertices are boundary ones.
    """
    m = n if m is None else m
    if diagonal not in ("/", "\\"):
        raise ValueError(f"diagonal must be '/' or '\\', not {diagonal!r}")
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    hx, hy = (hi[0] - lo[0]) / n, (hi[1] - lo[1]) / m
    nvx, nvy = (n, m) if periodic else (n + 1, m + 1)
    ii, jj = np.meshgrid(np.arange(nvx), np.arange(nvy), indexing="xy")
    xyz = np.stack([lo[0] + ii.ravel() * hx, lo[1] + jj.ravel() * hy], axis=1)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        d = rng.uniform(-jitter, jitter, size=(nvx * nvy, 2)) * np.array([hx, hy])
        if not periodic:
            ib = ii.ravel()
            jb = jj.ravel()
            free = (ib > 0) & (ib < n) & (jb > 0) & (jb < m)
            d[~free] = 0.0
        xyz = xyz + d

    def vid(i, j):
        if periodic:
            return (j % m) * nvx + (i % n)
        return j * nvx + i

    elem = np.empty((2 * n * m, 3), dtype=np.int64)
    e = 0
    for j in range(m):
        for i in range(n):
            v00, v10, v11, v01 = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            if diagonal == "/":
                elem[e] = (v00, v10, v11)
                elem[e + 1] = (v00, v11, v01)
            else:
                elem[e] = (v00, v10, v01)
                elem[e + 1] = (v10, v11, v01)
            e += 2
    period = (hi - lo) if periodic else None
    return Mesh(xyz=xyz, elem=elem, period=period,
                meta=dict(kind="split_square", n=n, m=m, jitter=jitter, seed=seed,
                          periodic=periodic, diagonal=diagonal))


def disk_mesh(n: int, *, radius: float = 1.0, q: int = 2, jitter: float = 0.0, seed: int | None = None) -> Mesh:
    """Triangulation of the disk of the given radius: the triangular lattice
    of a hexagon of n rings, ring k (k = 1..n) placed on the circle of radius
    k/n * radius with its 6k vertices at equal angles (vertex 0 at angle 0 of
    ring k is the lattice point on the first hexagon corner).  Counter-
    clockwise triangles.  ``jitter`` moves interior vertices radially and in
    angle by U(-jitter, jitter) times the ring spacing.

    Curved boundary (Section 3, iso-/sub-parametric maps): every triangle
    with an edge on the circle gets geometry nodes of degree q (the
    equispaced nodes of the reference triangle, in the velocity node order)
    placed by the affine map, except that the nodes inside its boundary edge
    move onto the circle at equally spaced angles between the edge's end
    vertices.  meta["curved"] = (elem ids (n_c,), nodes (n_c, N_q, 2)).
    """
    rng = np.random.default_rng(seed)
    # axial hexagon lattice points with their ring and position along the ring
    corners = [(1, 0), (0, 1), (-1, 1), (-1, 0), (0, -1), (1, -1)]
    index = {(0, 0): 0}
    pts = [(0.0, 0.0)]
    for k in range(1, n + 1):
        for side in range(6):
            c0, c1 = corners[side], corners[(side + 1) % 6]
            for t in range(k):
                a_ = (k * c0[0] + t * (c1[0] - c0[0]), k * c0[1] + t * (c1[1] - c0[1]))
                pos = side * k + t
                ang = 2.0 * np.pi * pos / (6 * k)
                r = k / n * radius
                if 0 < k < n and jitter > 0.0:
                    r += rng.uniform(-jitter, jitter) * radius / n
                    ang += rng.uniform(-jitter, jitter) * 2.0 * np.pi / (6 * k)
                index[a_] = len(pts)
                pts.append((r * np.cos(ang), r * np.sin(ang)))
    xyz = np.array(pts)

    def hexdist(a_):
        x, y = a_
        return max(abs(x), abs(y), abs(x + y))

    elem = []
    # the two lattice triangles with first corner (x, y): neighbours differ
    # by (1, 0), (0, 1) or (-1, 1)
    for (x, y) in sorted(index, key=lambda a_: index[a_]):
        for tri in (((x, y), (x + 1, y), (x, y + 1)), ((x, y), (x + 1, y - 1), (x + 1, y))):
            if all(v in index for v in tri) and max(hexdist(v) for v in tri) <= n:
                ids = [index[v] for v in tri]
                P = xyz[ids]
                area = (P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) - (P[2, 0] - P[0, 0]) * (P[1, 1] - P[0, 1])
                elem.append(ids if area > 0 else [ids[0], ids[2], ids[1]])
    elem = np.array(elem, dtype=np.int64)
    ring = np.zeros(len(pts), dtype=np.int64)
    for a_, i0 in index.items():
        ring[i0] = hexdist(a_)
    # geometry nodes of the boundary triangles
    ref = [(i / q, j / q) for j in range(q + 1) for i in range(q + 1 - j)]
    ids, nodes = [], []
    for e, (a0, a1, a2) in enumerate(elem):
        verts = [a0, a1, a2]
        on = [ring[v] == n for v in verts]
        edges = [(0, 1), (1, 2), (2, 0)]
        bnd = [(u, w) for (u, w) in edges if on[u] and on[w]]
        if not bnd:
            continue
        V = xyz[verts]
        X = np.array([V[0] + xi * (V[1] - V[0]) + eta * (V[2] - V[0]) for xi, eta in ref])
        for (u, w) in bnd:
            th0 = np.arctan2(V[u, 1], V[u, 0])
            th1 = np.arctan2(V[w, 1], V[w, 0])
            dth = (th1 - th0 + np.pi) % (2 * np.pi) - np.pi
            for qi, (xi, eta) in enumerate(ref):
                lam = np.array([1 - xi - eta, xi, eta])
                if abs(lam[u] + lam[w] - 1.0) < 1e-12 and lam[u] > 1e-12 and lam[w] > 1e-12:
                    th = th0 + lam[w] * dth
                    X[qi] = radius * np.array([np.cos(th), np.sin(th)])
        ids.append(e)
        nodes.append(X)
    meta = dict(kind="disk", n=n, radius=radius, q=q, jitter=jitter, seed=seed,
                curved=(np.array(ids, dtype=np.int64), np.array(nodes)))
    return Mesh(xyz=xyz, elem=elem, period=None, meta=meta)


def inradius(V: np.ndarray) -> np.ndarray:
    """Incircle radii of triangles with vertex coordinates V (n, 3, 2)."""
    V = np.asarray(V, float)
    a = np.linalg.norm(V[:, 1] - V[:, 2], axis=1)
    b = np.linalg.norm(V[:, 0] - V[:, 2], axis=1)
    c = np.linalg.norm(V[:, 0] - V[:, 1], axis=1)
    e1, e2 = V[:, 1] - V[:, 0], V[:, 2] - V[:, 0]
    area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
    return 2.0 * area / (a + b + c)


def with_slivers(mesh: Mesh, squares, ratio: float) -> Mesh:
    """The same split-square mesh ('/' diagonals) with one sliver per listed
    square (i, j): the corner (i+1, j) moves towards the midpoint of the
    square's diagonal until the incircle radius of the square's triangle
    (v00, v10, v11) is ``ratio`` times smaller than before (Section 6.6
    reduces it 70.53 times).  The square's other triangle is unchanged; the
    triangles of the neighbouring squares that share the moved corner are
    stretched but stay valid.  The squares must not share corners.  Returns
    a new mesh; the sliver triangles are meta["slivers"]."""
    n, m = mesh.meta["n"], mesh.meta["m"]
    if mesh.meta.get("diagonal", "/") != "/":
        raise ValueError("expects '/' diagonals")
    periodic = mesh.period is not None
    nvx = n if periodic else n + 1

    def vid(a, b):
        return (b % m) * nvx + (a % n) if periodic else b * nvx + a

    xyz = mesh.xyz.copy()
    U = mesh.unwrapped_vertices()
    slivers = []
    for i, j in squares:
        e0 = 2 * (j * n + i)                   # triangle (v00, v10, v11)
        v00, v10, v11 = U[e0]
        r0 = inradius(U[e0:e0 + 1])[0]
        mid = 0.5 * (v00 + v11)
        d = v11 - v00
        nrm = np.array([d[1], -d[0]]) / np.linalg.norm(d)   # towards v10 on a counter-clockwise square
        target = r0 / ratio
        lo, hi = 0.0, 0.5 * np.linalg.norm(d)
        for _ in range(200):
            mid_d = 0.5 * (lo + hi)
            if inradius(np.array([[v00, mid + mid_d * nrm, v11]]))[0] < target:
                lo = mid_d
            else:
                hi = mid_d
        new10 = mid + 0.5 * (lo + hi) * nrm
        xyz[vid(i + 1, j)] = xyz[vid(i + 1, j)] + (new10 - v10)   # in the stored vertex's frame
        slivers.append(e0)
    meta = dict(mesh.meta, slivers=tuple(slivers), sliver_ratio=ratio, sliver_squares=tuple(map(tuple, squares)))
    return Mesh(xyz=xyz, elem=mesh.elem.copy(), period=mesh.period, meta=meta)


def kuhn_cube(n: int, *, periodic: bool = True, lo=(0.0, 0.0, 0.0),
              hi=(1.0, 1.0, 1.0)) -> Mesh:
    """n^3 cubes, each cut into the 6 tetrahedra along its main diagonal.

    Each tetrahedron follows one monotone lattice path from corner (0,0,0)
    to corner (1,1,1) of its cube, one per permutation of the axes
    (itertools order).  All cubes use the same orientation, so the mesh is
    conforming and, when ``periodic``, matches across the periodic seams.
    """
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    h = (hi - lo) / n
    nv = n if periodic else n + 1
    kk, jj, ii = np.meshgrid(np.arange(nv), np.arange(nv), np.arange(nv), indexing="ij")
    xyz = np.stack([lo[0] + ii.ravel() * h[0], lo[1] + jj.ravel() * h[1],
                    lo[2] + kk.ravel() * h[2]], axis=1)

    def vid(i, j, k):
        if periodic:
            return ((k % n) * nv + (j % n)) * nv + (i % n)
        return (k * nv + j) * nv + i

    perms = list(itertools.permutations(range(3)))
    elem = np.empty((6 * n ** 3, 4), dtype=np.int64)
    e = 0
    for k in range(n):
        for j in range(n):
            for i in range(n):
                for perm in perms:
                    c = [0, 0, 0]
                    path = [vid(i, j, k)]
                    for ax in perm:
                        c[ax] += 1
                        path.append(vid(i + c[0], j + c[1], k + c[2]))
                    elem[e] = path
                    e += 1
    period = (hi - lo) if periodic else None
    return Mesh(xyz=xyz, elem=elem, period=period,
                meta=dict(kind="kuhn_cube", n=n, periodic=periodic))


def homogeneous_material(n_elem: int, lam=2.0, mu=1.0, rho=1.0):
    """Per-element (lambda, mu, rho) arrays of a homogeneous medium."""
    return (np.full(n_elem, float(lam)), np.full(n_elem, float(mu)),
            np.full(n_elem, float(rho)))


def lognormal_material(n_elem: int, *, base=(2.0, 1.0, 1.0), sigma: float = 0.2,
                       seed: int = 0):
    """(lambda, mu, rho) = base * exp(sigma Z), Z ~ N(0,1) i.i.d.

    Draws are element-major in (lambda, mu, rho) order.
    """
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n_elem, 3))
    f = np.exp(sigma * z)
    return base[0] * f[:, 0], base[1] * f[:, 1], base[2] * f[:, 2]


def anisotropic_material(n_elem: int, dim: int, *, lam: float = 2.0, mu: float = 1.0, rho: float = 1.0,
                         sigma: float = 0.2, strength: float = 0.5, homogeneous: bool = False,
                         seed: int = 0):
    """General (anisotropic) media in the Voigt form of Section 2: per
    element the matrix E~ with s~ = E~ e~ (tensor shear strains, so 2 mu on
    the isotropic shear diagonal), Voigt order (xx, yy, xy) or (xx, yy, zz,
    yz, xz, xy).  Returns (E~ (n_elem, n_sigma, n_sigma), rho (n_elem,)).

    The tensor entries E_ijkl of each element, laid out as the symmetric
    n_sigma x n_sigma matrix H[v(ij)][v(kl)], are exp(sigma Z) times those of
    the isotropic (lam, mu) medium plus strength * G G^T / n_sigma with
    G ~ N(0,1) n_sigma x n_sigma (positive definite, every normal-shear
    coupling present); E~ = H W with W = 1 on normal, 2 on shear columns.
    Draws are element-major: Z, then G row-major, then Z_rho with
    rho exp(sigma Z_rho).  ``homogeneous`` repeats element 0's draw."""
    ns = dim * (dim + 1) // 2
    rng = np.random.default_rng(seed)
    H0 = np.zeros((ns, ns))
    H0[:dim, :dim] = lam
    H0[np.arange(dim), np.arange(dim)] = lam + 2 * mu
    H0[np.arange(dim, ns), np.arange(dim, ns)] = mu
    W = np.array([1.0] * dim + [2.0] * (ns - dim))
    m = 1 if homogeneous else n_elem
    Et = np.empty((m, ns, ns))
    r = np.empty(m)
    for e in range(m):
        z = rng.standard_normal()
        G = rng.standard_normal((ns, ns))
        zr = rng.standard_normal()
        H = np.exp(sigma * z) * H0 + strength * (G @ G.T) / ns
        Et[e] = H * W[None, :]
        r[e] = rho * np.exp(sigma * zr)
    if homogeneous:
        Et = np.repeat(Et, n_elem, axis=0)
        r = np.repeat(r, n_elem)
    return Et, r


def layered_material(centroids: np.ndarray, *, sigma: float = 0.1, seed: int = 0,
                     axis: int = 1):
    """Three layers by centroid coordinate along ``axis``.

    Below 1/3: (rho, lambda, mu) = (2, 16, 8); below 2/3: (1.5, 6, 3); above:
    (1, 2, 1).  Each parameter of each element is then multiplied by
    exp(sigma Z), Z ~ N(0,1), element-major in (lambda, mu, rho) order.
    """
    y = centroids[:, axis]
    n = len(y)
    rho = np.where(y < 1 / 3, 2.0, np.where(y < 2 / 3, 1.5, 1.0))
    lam = np.where(y < 1 / 3, 16.0, np.where(y < 2 / 3, 6.0, 2.0))
    mu = np.where(y < 1 / 3, 8.0, np.where(y < 2 / 3, 3.0, 1.0))
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, 3))
    f = np.exp(sigma * z)
    return lam * f[:, 0], mu * f[:, 1], rho * f[:, 2]


def ricker(t, f0: float = 10.0, t_delay: float = 0.1, a1: float = 2.0):
    """Ricker-type source time function a1 (0.5 + a2 tau^2) exp(a2 tau^2).

    tau = t - t_delay, a2 = -(pi f0)^2.  The paper's formula (Section 6.3)
    has lost its exponential factor; this is the standard Ricker wavelet
    scaled by a1/2, so a1 = 2 gives unit peak amplitude.
    """
    t = np.asarray(t, float)
    a2 = -(math.pi * f0) ** 2
    tau2 = (t - t_delay) ** 2
    return a1 * (0.5 + a2 * tau2) * np.exp(a2 * tau2)


def random_points(n: int, dim: int, *, lo=0.05, hi=0.95, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n, dim))


def top_edge_receivers(n: int, y: float = 1.0) -> np.ndarray:
    """n receivers at ((r + 1/2)/n, y)."""
    x = (np.arange(n) + 0.5) / n
    return np.stack([x, np.full(n, y)], axis=1)


def ragged_meshes(n_mesh: int = 16, seed: int = 4002, lo: int = 512, hi: int = 16384):
    """Meshes of uneven size for a mesh batch: N_k = exp(U(ln lo, ln hi))
    triangles (seed), n_x = round(sqrt(N_k / 2)), n_y = round(N_k / (2 n_x))
    split squares of the unit square with 20% jitter (seed 4100 + k), and
    three lognormal layers (seed 4200 + k).  Returns [(mesh, (lam, mu, rho))]."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_mesh):
        Nk = math.exp(rng.uniform(math.log(lo), math.log(hi)))
        nx = max(1, round(math.sqrt(Nk / 2)))
        ny = max(1, round(Nk / (2 * nx)))
        m = split_square(nx, ny, jitter=0.2, seed=4100 + k)
        out.append((m, layered_material(m.centroids(), sigma=0.1, seed=4200 + k)))
    return out


def workload(name: str, scale: int | None = None) -> dict:
    """Named synthetic workloads.

    Returns a dict with the mesh, material, degrees, scheme, dt, number of
    steps and the source/receiver description.  ``scale`` overrides the
    mesh resolution (used for the small parity versions of a workload).

    c1: 8x8 periodic split square, p=1, Crank-Nicolson, homogeneous
        (rho, lambda, mu) = (1, 2, 1), plane P-wave, dt=0.01, 10 steps.
    c2: 64x64 split square with +-20% jitter (seed 2001), free surface,
        p=3, p_gamma=3, three lognormal layers (seed 2002), Ricker 10 Hz
        vertical force at (0.503, 0.497), dt=2.5e-3, 100 steps.
    c3: 32^3 periodic Kuhn cube, p=2, Crank-Nicolson, homogeneous, plane
        S-wave, dt=0.01, 50 steps.
    c5: 128x128 split square, free surface, p=2, p_gamma=2, lognormal
        sigma=0.2 (seed 5001), Ricker at (0.503, 0.303), 128 receivers on
        the top edge, dt=2e-3, 200 steps.
    """
    if name == "c1":
        n = scale or 8
        mesh = split_square(n, periodic=True)
        lam, mu, rho = homogeneous_material(mesh.n_elem)
        return dict(name=name, mesh=mesh, lam=lam, mu=mu, rho=rho, p=1, p_gamma=0,
                    scheme="cn", dt=0.01, steps=10, init="pwave2d", sources=None)
    if name == "c2":
        n = scale or 64
        mesh = split_square(n, jitter=0.2, seed=2001)
        lam, mu, rho = layered_material(mesh.centroids(), sigma=0.1, seed=2002)
        src = dict(pos=np.array([[0.503, 0.497]]), dir=np.array([[0.0, 1.0]]),
                   f0=10.0, t_delay=0.1)
        return dict(name=name, mesh=mesh, lam=lam, mu=mu, rho=rho, p=3, p_gamma=3,
                    scheme="stdg", dt=2.5e-3, steps=100, init="zero", sources=src)
    if name == "c3":
        n = scale or 32
        mesh = kuhn_cube(n, periodic=True)
        lam, mu, rho = homogeneous_material(mesh.n_elem)
        return dict(name=name, mesh=mesh, lam=lam, mu=mu, rho=rho, p=2, p_gamma=0,
                    scheme="cn", dt=0.01, steps=50, init="swave3d", sources=None)
    if name == "c5":
        n = scale or 128
        mesh = split_square(n)
        lam, mu, rho = lognormal_material(mesh.n_elem, base=(2.0, 1.0, 1.0), sigma=0.2,
                                          seed=5001)
        src = dict(pos=np.array([[0.503, 0.303]]), dir=np.array([[0.0, 1.0]]),
                   f0=10.0, t_delay=0.1)
        return dict(name=name, mesh=mesh, lam=lam, mu=mu, rho=rho, p=2, p_gamma=2,
                    scheme="stdg", dt=2e-3, steps=200, init="zero", sources=src,
                    receivers=top_edge_receivers(n if scale else 128))
    raise KeyError(name)
