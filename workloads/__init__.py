"""Seeded synthetic inputs: surface meshes and right-hand sides.

This module only *generates* data (vertex coordinates, triangle indices,
random vectors). It contains none of the method's arithmetic: no kernel,
no quadrature, no clustering, no approximation. Both the HIP path and the
CPU oracle receive exactly the arrays produced here.

Meshes are flat-triangle surface meshes: ``vertices`` is float64 [nv, 3],
``triangles`` is int32 [nt, 3] (0-based, outward orientation where the
surface is closed). All generators are deterministic.
"""
from __future__ import annotations

import hashlib
import math

import numpy as np

__all__ = [
    "icosahedron",
    "icosphere",
    "geodesic_sphere",
    "ellipsoid",
    "torus",
    "box_surface",
    "cube_surface",
    "random_x",
    "smooth_rhs",
    "mesh_hash",
    "workload_c0",
    "workload_c1",
]


def _orient_outward(vertices: np.ndarray, tris: np.ndarray, center: np.ndarray) -> np.ndarray:
    p0 = vertices[tris[:, 0]]
    p1 = vertices[tris[:, 1]]
    p2 = vertices[tris[:, 2]]
    n = np.cross(p1 - p0, p2 - p0)
    c = (p0 + p1 + p2) / 3.0 - center
    flip = np.einsum("ij,ij->i", n, c) < 0
    out = tris.copy()
    out[flip, 1], out[flip, 2] = tris[flip, 2], tris[flip, 1]
    return out


def icosahedron() -> tuple[np.ndarray, np.ndarray]:
    """Regular icosahedron inscribed in the unit sphere.

    Vertices are the cyclic permutations of (0, +-1, +-phi), normalised.
    Faces are the vertex triples that are pairwise at the edge length 2
    (before normalisation), oriented outward and sorted lexicographically.
    """
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    pts = []
    for s1 in (-1.0, 1.0):
        for s2 in (-phi, phi):
            pts.append((0.0, s1, s2))
            pts.append((s1, s2, 0.0))
            pts.append((s2, 0.0, s1))
    raw = np.array(pts, dtype=np.float64)
    faces = []
    n = len(raw)
    d = np.linalg.norm(raw[:, None, :] - raw[None, :, :], axis=2)
    adj = np.abs(d - 2.0) < 1e-9
    for a in range(n):
        for b in range(a + 1, n):
            if not adj[a, b]:
                continue
            for c in range(b + 1, n):
                if adj[a, c] and adj[b, c]:
                    faces.append((a, b, c))
    assert len(faces) == 20
    v = raw / np.linalg.norm(raw, axis=1, keepdims=True)
    t = _orient_outward(v, np.array(faces, dtype=np.int32), np.zeros(3))
    return v, t.astype(np.int32)


def icosphere(level: int) -> tuple[np.ndarray, np.ndarray]:
    """Icosahedron refined ``level`` times by edge midpoints projected to the unit sphere.

    Each triangle (a, b, c) becomes (a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca).
    New vertices are numbered in order of first appearance. Level L has
    20*4**L triangles and 10*4**L + 2 vertices.
    """
    v, t = icosahedron()
    verts = [tuple(p) for p in v]
    tris = [tuple(int(i) for i in f) for f in t]
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(i: int, j: int) -> int:
            key = (i, j) if i < j else (j, i)
            k = cache.get(key)
            if k is None:
                p = np.array(verts[i]) + np.array(verts[j])
                p = p / np.linalg.norm(p)
                verts.append(tuple(p))
                k = len(verts) - 1
                cache[key] = k
            return k

        new = []
        for a, b, c in tris:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        tris = new
    return np.array(verts, dtype=np.float64), np.array(tris, dtype=np.int32)


def geodesic_sphere(freq: int) -> tuple[np.ndarray, np.ndarray]:
    """Frequency-``freq`` geodesic sphere: each icosahedron face cut into freq**2 triangles.

    Grid points of each face are projected onto the unit sphere; points on shared
    edges and corners are merged. 20*freq**2 triangles.
    """
    v0, t0 = icosahedron()
    f = int(freq)
    assert f >= 1
    key_to_idx: dict[tuple[int, ...], int] = {}
    verts: list[np.ndarray] = []

    def vid(face: tuple[int, int, int], i: int, j: int) -> int:
        # barycentric integer coordinates (f-i-j, i, j) on face (a, b, c)
        a, b, c = face
        w = {a: f - i - j, b: i, c: j}
        key = tuple(sorted((k, wk) for k, wk in w.items() if wk > 0))
        idx = key_to_idx.get(key)
        if idx is None:
            p = (w[a] * v0[a] + w[b] * v0[b] + w[c] * v0[c]) / f
            p = p / np.linalg.norm(p)
            verts.append(p)
            idx = len(verts) - 1
            key_to_idx[key] = idx
        return idx

    tris = []
    for face in t0:
        fc = (int(face[0]), int(face[1]), int(face[2]))
        for i in range(f):
            for j in range(f - i):
                p = vid(fc, i, j)
                q = vid(fc, i + 1, j)
                r = vid(fc, i, j + 1)
                tris.append((p, q, r))
                if i + j < f - 1:
                    s = vid(fc, i + 1, j + 1)
                    tris.append((q, s, r))
    V = np.array(verts, dtype=np.float64)
    T = _orient_outward(V, np.array(tris, dtype=np.int32), np.zeros(3))
    return V, T.astype(np.int32)


def ellipsoid(freq: int, axes) -> tuple[np.ndarray, np.ndarray]:
    """Geodesic sphere of frequency ``freq`` scaled by semi-axes ``axes``."""
    V, T = geodesic_sphere(freq)
    return V * np.asarray(axes, dtype=np.float64)[None, :], T


def torus(R: float, r: float, nu: int, nv: int) -> tuple[np.ndarray, np.ndarray]:
    """Torus with major radius R and minor radius r on an nu x nv grid (2*nu*nv triangles)."""
    u = 2.0 * np.pi * np.arange(nu) / nu
    w = 2.0 * np.pi * np.arange(nv) / nv
    U, W = np.meshgrid(u, w, indexing="ij")
    X = (R + r * np.cos(W)) * np.cos(U)
    Y = (R + r * np.cos(W)) * np.sin(U)
    Z = r * np.sin(W)
    V = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    tris = []
    for i in range(nu):
        for j in range(nv):
            a = i * nv + j
            b = ((i + 1) % nu) * nv + j
            c = ((i + 1) % nu) * nv + (j + 1) % nv
            d = i * nv + (j + 1) % nv
            tris.append((a, b, c))
            tris.append((a, c, d))
    T = np.array(tris, dtype=np.int32)
    # outward w.r.t. the tube centre line
    p0, p1, p2 = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    n = np.cross(p1 - p0, p2 - p0)
    c = (p0 + p1 + p2) / 3.0
    ang = np.arctan2(c[:, 1], c[:, 0])
    core = np.stack([R * np.cos(ang), R * np.sin(ang), np.zeros_like(ang)], axis=1)
    flip = np.einsum("ij,ij->i", n, c - core) < 0
    T2 = T.copy()
    T2[flip, 1], T2[flip, 2] = T[flip, 2], T[flip, 1]
    return V.astype(np.float64), T2.astype(np.int32)


def box_surface(lx: float, ly: float, lz: float, nx: int, ny: int, nz: int):
    """Structured triangulated surface of the box [0,lx]x[0,ly]x[0,lz].

    Face grids have nx, ny, nz cells along x, y, z; each cell is cut into two
    triangles. Vertices on shared edges are merged. 4*(nx*ny + ny*nz + nx*nz) triangles.
    """
    index: dict[tuple[int, int, int], int] = {}
    verts = []

    def vid(i: int, j: int, k: int) -> int:
        key = (i, j, k)
        idx = index.get(key)
        if idx is None:
            verts.append((lx * i / nx, ly * j / ny, lz * k / nz))
            idx = len(verts) - 1
            index[key] = idx
        return idx

    tris = []

    def quad(a, b, c, d):
        tris.append((a, b, c))
        tris.append((a, c, d))

    for fixed, (n1, n2) in ((0, (ny, nz)), (1, (nx, nz)), (2, (nx, ny))):
        for side in (0, 1):
            for i in range(n1):
                for j in range(n2):
                    def P(ii, jj):
                        if fixed == 0:
                            return vid(side * nx, ii, jj)
                        if fixed == 1:
                            return vid(ii, side * ny, jj)
                        return vid(ii, jj, side * nz)
                    quad(P(i, j), P(i + 1, j), P(i + 1, j + 1), P(i, j + 1))
    V = np.array(verts, dtype=np.float64)
    T = _orient_outward(V, np.array(tris, dtype=np.int32), np.array([lx, ly, lz]) / 2.0)
    return V, T.astype(np.int32)


def cube_surface(n: int):
    """Surface of [-1,1]^3 with an n x n grid per face: 12 n^2 triangles, 6 n^2 + 2 nodes."""
    V, T = box_surface(2.0, 2.0, 2.0, n, n, n)
    return V - 1.0, T


def plate(n: int, size: float = 1.0):
    """Flat square [0,size]^2 in the plane z = 0, n x n grid, 2 n^2 triangles
    (every cluster coplanar: the Kelvin tensor decouples into in-plane and
    normal parts)."""
    g = np.linspace(0.0, size, n + 1)
    X, Y = np.meshgrid(g, g, indexing="ij")
    V = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    tris = []
    for i in range(n):
        for j in range(n):
            a = i * (n + 1) + j
            b = (i + 1) * (n + 1) + j
            tris.append((a, b, b + 1))
            tris.append((a, b + 1, a + 1))
    return V.astype(np.float64), np.array(tris, dtype=np.int32)


def random_x(n_dof: int, nrhs: int = 1, seed: int = 0) -> np.ndarray:
    """x ~ N(0,1), shape (nrhs, n_dof), from NumPy PCG64 ``default_rng(seed)``."""
    return np.random.default_rng(seed).standard_normal((nrhs, n_dof))


def smooth_rhs(vertices: np.ndarray, triangles: np.ndarray, seed: int = 1) -> np.ndarray:
    """Random smooth vector field sampled at the triangle centroids (length 3*nt, DOF 3i+a).

    g_a(x) = sum over m = 1..8 and monomials x^alpha with |alpha| <= 2 of
    c[m, a, alpha] x^alpha, monomials ordered 1, x, y, z, x^2, xy, xz, y^2, yz, z^2,
    coefficients N(0,1) from ``default_rng(seed)`` drawn with shape (8, 3, 10).
    """
    c = np.random.default_rng(seed).standard_normal((8, 3, 10))
    p = vertices[triangles]
    x = ((p[:, 0] + p[:, 1]) + p[:, 2]) / 3.0
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    mono = np.stack([np.ones_like(X), X, Y, Z, X * X, X * Y, X * Z, Y * Y, Y * Z, Z * Z], axis=1)
    g = np.einsum("mak,ik->ia", c, mono)
    return np.ascontiguousarray(g.reshape(-1))


def mesh_hash(vertices: np.ndarray, triangles: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(vertices, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(triangles, dtype=np.int32).tobytes())
    return h.hexdigest()[:16]


# Named workloads (material and approximation parameters used throughout).
def workload_c0():
    """Unit icosphere level 3 (1280 triangles, 3840 DOF), E=1, nu=0.3, eta=2, leaf 32, eps=1e-4."""
    V, T = icosphere(3)
    return dict(name="icosphere-L3", vertices=V, triangles=T, E=1.0, nu=0.3, eta=2.0,
                leaf=32, eps=1e-4, nrhs=1)


def workload_c1():
    """Unit icosphere level 5 (20480 triangles, 61440 DOF), eps=1e-6, 16 right-hand sides."""
    V, T = icosphere(5)
    return dict(name="icosphere-L5", vertices=V, triangles=T, E=1.0, nu=0.3, eta=2.0,
                leaf=32, eps=1e-6, nrhs=16)


def workload_c3():
    """Box [0,10]x[0,1]x[0,1], structured surface with h = 1/36: 108864 triangles,
    326592 DOF; nu = 0.3, E = 1; reference FP64 build at eps = 1e-7. Only the
    Dirichlet (single-layer) problem: the traction part needs the adjoint
    double-layer operator, which is not part of this library."""
    V, T = box_surface(10.0, 1.0, 1.0, 360, 36, 36)
    return dict(name="precision-box", vertices=V, triangles=T, E=1.0, nu=0.3, eta=2.0,
                leaf=32, eps=1e-7)


def batch_bodies(n_bodies: int = 96, n_lo: int = 2000, n_hi: int = 40000, seed: int = 2,
                 eps: float = 1e-5):
    """Independent bodies for one batched build: ellipsoids and tori.

    Per body, from NumPy PCG64 ``default_rng(seed)`` in this order: the kind
    (ellipsoid if a uniform draw is < 1/2, else torus), a target triangle count
    n log-uniform in [n_lo, n_hi], then the shape -- ellipsoid: semi-axes
    uniform in [0.5, 2] (three draws), a geodesic sphere of frequency
    round(sqrt(n/20)); torus: R = 1, r uniform in [0.2, 0.5], an n_u x n_v grid
    with n_v = round(sqrt(n r / 2)), n_u = round(n / (2 n_v)) -- and Poisson's
    ratio uniform in [0.2, 0.45]. E = 1 and the given eps for every body.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_bodies):
        is_ell = rng.random() < 0.5
        n = float(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        if is_ell:
            axes = rng.uniform(0.5, 2.0, 3)
            f = max(1, int(round(np.sqrt(n / 20.0))))
            V, T = ellipsoid(f, axes)
            kind = "ellipsoid"
        else:
            r = float(rng.uniform(0.2, 0.5))
            nv = max(3, int(round(np.sqrt(n * r / 2.0))))
            nu_ = max(3, int(round(n / (2.0 * nv))))
            V, T = torus(1.0, r, nu_, nv)
            kind = "torus"
        pr = float(rng.uniform(0.2, 0.45))
        out.append(dict(kind=kind, vertices=V, triangles=T, E=1.0, nu=pr, eps=eps))
    return out


def workload_c2():
    """96 bodies (ellipsoids and tori, 2k-40k triangles, log-uniform), eps 1e-5,
    8 right-hand sides per body; eta 2, leaf 32."""
    return dict(name="batch96", bodies=batch_bodies(96, 2000, 40000, seed=2, eps=1e-5), eta=2.0,
                leaf=32, nrhs=8)


def serving_requests(n_requests: int = 2000, seed: int = 4, dof_lo: int = 1000,
                     dof_hi: int = 80000):
    """Requests of the serving workload, from NumPy PCG64 ``default_rng(seed)``.

    Per request, in this order: the mesh type, uniform over sphere, ellipsoid,
    torus; the DOF count log-uniform in [dof_lo, dof_hi] (triangles = DOF/3);
    for an ellipsoid three semi-axes uniform in [0.5, 2], for a torus r uniform
    in [0.2, 0.5] (R = 1); Poisson's ratio uniform in [0.2, 0.45]; eps uniform
    over {1e-3, 1e-5, 1e-7}; a solve (probability 1/2) or m products with m
    uniform in 1..32; then the seed of the request's vectors. Spheres and
    ellipsoids are geodesic spheres of frequency round(sqrt(n/20)); tori use the
    grid rule of ``batch_bodies``. Meshes are generated lazily by ``mesh_of``.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_requests):
        kind = ("sphere", "ellipsoid", "torus")[int(rng.integers(0, 3))]
        dof = float(np.exp(rng.uniform(np.log(dof_lo), np.log(dof_hi))))
        n = dof / 3.0
        shape = {}
        if kind == "ellipsoid":
            shape["axes"] = tuple(float(a) for a in rng.uniform(0.5, 2.0, 3))
        elif kind == "torus":
            shape["r"] = float(rng.uniform(0.2, 0.5))
        nu = float(rng.uniform(0.2, 0.45))
        eps = (1e-3, 1e-5, 1e-7)[int(rng.integers(0, 3))]
        solve = bool(rng.random() < 0.5)
        m = 1 if solve else int(rng.integers(1, 33))
        vseed = int(rng.integers(0, 2**31 - 1))
        out.append(dict(kind=kind, n=n, shape=shape, nu=nu, E=1.0, eps=eps, solve=solve, m=m,
                        vseed=vseed))
    return out


def mesh_of(req: dict):
    """Mesh of a serving request (see ``serving_requests``)."""
    n = req["n"]
    if req["kind"] == "torus":
        r = req["shape"]["r"]
        nv = max(3, int(round(np.sqrt(n * r / 2.0))))
        nu_ = max(3, int(round(n / (2.0 * nv))))
        return torus(1.0, r, nu_, nv)
    f = max(1, int(round(np.sqrt(n / 20.0))))
    V, T = geodesic_sphere(f)
    if req["kind"] == "ellipsoid":
        V = V * np.asarray(req["shape"]["axes"])[None, :]
    return V, T
