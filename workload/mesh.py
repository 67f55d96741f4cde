"""Cube-split tetrahedral meshes with periodic face connectivity.

Recipe (the workloads of the elastic ADER-DG benchmarks):
  * unit cube [0,1]^3, n x n x n cubes of edge h = 1/n;
  * each cube split into the 6 Kuhn tetrahedra: for every permutation pi of the
    axes (lexicographic order), vertices c, c+h e_pi0, c+h(e_pi0+e_pi1),
    c+h(1,1,1); this split is conforming and translation invariant, so faces
    also match across the periodic boundary;
  * if a tetrahedron is negatively oriented its local vertices 1 and 2 are
    swapped;
  * lattice points strictly inside the cube are moved by h*U(-0.1,0.1) per
    coordinate (boundary points stay, so periodic faces stay congruent);
  * element order: cube (x-major), then permutation.

Face convention (shared by every consumer of these tables): local face s of
an element is the local-vertex triple FACE_VERTS[s]; its outward normal is
(x_b - x_a) x (x_c - x_a).  For face s of element e the tables give the
neighbour element nu = neigh[e,s], the neighbour's local face j = nface[e,s]
and the orientation h = orient[e,s], the position of e's first face vertex
inside nu's face triple.  face_rot packs j | h << 2.
"""
from __future__ import annotations

from dataclasses import dataclass
from itertools import permutations

import numpy as np

FACE_VERTS = ((0, 2, 1), (0, 1, 3), (0, 3, 2), (1, 2, 3))
BASE_SEED = 190311521


def seed_for(index: int) -> int:
    return BASE_SEED + int(index)


@dataclass
class CubeMesh:
    n: int
    h: float
    X: np.ndarray        # (E, 4, 3) float64 vertex coordinates (unwrapped)
    V: np.ndarray        # (E, 4) int64 periodic vertex ids
    neigh: np.ndarray    # (E, 4) int32
    nface: np.ndarray    # (E, 4) int8
    orient: np.ndarray   # (E, 4) int8

    @property
    def E(self) -> int:
        return self.X.shape[0]

    @property
    def face_rot(self) -> np.ndarray:
        return (self.nface.astype(np.uint8) | (self.orient.astype(np.uint8) << 2)).astype(np.uint8)


EVEN_PERMS = tuple(p for p in permutations(range(4))
                   if sum(1 for i in range(4) for j in range(i + 1, 4) if p[i] > p[j]) % 2 == 0)


def cube_mesh(n: int, seed: int, jitter: float = 0.1, relabel: bool = False) -> CubeMesh:
    """relabel=True applies a random even permutation to the local vertex order
    of every element (orientation preserved), so that all 12 combinations of
    neighbour face j and orientation h occur."""
    if n < 3:
        raise ValueError("need n >= 3 for unique periodic face pairing")
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / n
    disp = rng.uniform(-jitter, jitter, size=(n, n, n, 3)) * h
    lat = np.arange(n)
    interior = (lat > 0)
    mask = interior[:, None, None] & interior[None, :, None] & interior[None, None, :]
    disp[~mask] = 0.0

    perms = list(permutations(range(3)))
    E = 6 * n ** 3
    ci, cj, ck = np.meshgrid(lat, lat, lat, indexing="ij")
    corner = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)   # (n^3, 3)
    L = np.zeros((n ** 3, 6, 4, 3), dtype=np.int64)
    for pidx, p in enumerate(perms):
        e0 = np.eye(3, dtype=np.int64)[p[0]]
        e1 = np.eye(3, dtype=np.int64)[p[1]]
        verts = [np.zeros(3, np.int64), e0, e0 + e1, np.ones(3, np.int64)]
        sign = np.linalg.det(np.array([e0, e0 + e1, np.ones(3)], dtype=float))
        if sign < 0:
            verts[1], verts[2] = verts[2], verts[1]
        for v in range(4):
            L[:, pidx, v, :] = corner + verts[v]
    L = L.reshape(E, 4, 3)
    if relabel:
        prng = np.random.Generator(np.random.PCG64(seed + 31))
        choice = prng.integers(0, len(EVEN_PERMS), size=E)
        perm = np.array(EVEN_PERMS)[choice]                  # (E, 4)
        L = np.take_along_axis(L, perm[:, :, None], axis=1)
    Lm = L % n
    V = (Lm[..., 0] * n + Lm[..., 1]) * n + Lm[..., 2]
    X = L.astype(np.float64) * h + disp[Lm[..., 0], Lm[..., 1], Lm[..., 2]]

    # periodic face pairing by sorted vertex-id triple
    fv = np.array(FACE_VERTS)
    tri = V[:, fv]                                   # (E, 4, 3)
    st = np.sort(tri, axis=2)
    nv = n ** 3
    key = (st[..., 0] * nv + st[..., 1]) * nv + st[..., 2]
    key = key.ravel()
    order = np.argsort(key, kind="stable")
    ks = key[order]
    if not (np.all(ks[0::2] == ks[1::2]) and (len(ks) < 3 or np.all(ks[1:-1:2] != ks[2::2]))):
        raise RuntimeError("face pairing is not one-to-one")
    a, b = order[0::2], order[1::2]
    partner = np.empty_like(order)
    partner[a] = b
    partner[b] = a
    neigh = (partner // 4).reshape(E, 4).astype(np.int32)
    nface = (partner % 4).reshape(E, 4).astype(np.int8)
    first = tri[:, :, 0].ravel()                     # first vertex id of each face
    ntri = tri.reshape(-1, 3)[partner]               # neighbour's face triple
    hpos = np.argmax(ntri == first[:, None], axis=1)
    if not np.all(ntri[np.arange(len(first)), hpos] == first):
        raise RuntimeError("orientation lookup failed")
    orient = hpos.reshape(E, 4).astype(np.int8)
    return CubeMesh(n=n, h=h, X=X, V=V, neigh=neigh, nface=nface, orient=orient)


def random_materials(E: int, seed: int):
    """rho ~ U[2000,3000], cp ~ U[4000,6000], cs = cp / U[1.6,2.0] per element.
    Returns (E, 3) float64 columns (rho, cp, cs)."""
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    rho = rng.uniform(2000.0, 3000.0, E)
    cp = rng.uniform(4000.0, 6000.0, E)
    cs = cp / rng.uniform(1.6, 2.0, E)
    return np.stack([rho, cp, cs], axis=1)


def random_dofs(E: int, P: int, B: int, seed: int, dtype=np.float64):
    """DOFs N(0,1), element-major layout (E, P, B)."""
    rng = np.random.Generator(np.random.PCG64(seed + 104729))
    return rng.standard_normal((E, P, B)).astype(dtype)


def dt_from_mesh(mesh: CubeMesh, materials: np.ndarray, factor: float = 0.1) -> float:
    """dt = factor * h_min / cp_max with h_min the smallest insphere diameter
    6 V / (sum of face areas) over the mesh."""
    X = mesh.X
    e1 = X[:, 1] - X[:, 0]
    e2 = X[:, 2] - X[:, 0]
    e3 = X[:, 3] - X[:, 0]
    vol = np.abs(np.einsum("ei,ei->e", e1, np.cross(e2, e3))) / 6.0
    area = np.zeros(X.shape[0])
    for (a, b, c) in FACE_VERTS:
        area += 0.5 * np.linalg.norm(np.cross(X[:, b] - X[:, a], X[:, c] - X[:, a]), axis=1)
    hmin = np.min(6.0 * vol / area)
    return float(factor * hmin / np.max(materials[:, 1]))


def graded_cube_mesh(n: int, seed: int, ratio: float, jitter: float = 0.1, relabel: bool = False) -> CubeMesh:
    """cube_mesh with the x coordinate mapped by g(x) = (r^x - 1) / (r - 1),
    so cell widths along x grow geometrically by the factor r = ratio from
    x = 0 to x = 1.  g fixes 0 and 1 and leaves y, z alone, so the periodic
    faces stay congruent."""
    m = cube_mesh(n, seed, jitter=jitter, relabel=relabel)
    if ratio != 1.0:
        X = m.X.copy()
        X[..., 0] = (ratio ** X[..., 0] - 1.0) / (ratio - 1.0)
        m = CubeMesh(n=m.n, h=m.h, X=X, V=m.V, neigh=m.neigh, nface=m.nface, orient=m.orient)
    return m


def element_time_steps(mesh: CubeMesh, materials: np.ndarray, factor: float = 0.1) -> np.ndarray:
    """Per-element CFL time step factor * h_e / cp_e, h_e the insphere
    diameter 6 V / (sum of face areas) of element e."""
    X = mesh.X
    e1, e2, e3 = X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]
    vol = np.abs(np.einsum("ei,ei->e", e1, np.cross(e2, e3))) / 6.0
    area = np.zeros(X.shape[0])
    for (a, b, c) in FACE_VERTS:
        area += 0.5 * np.linalg.norm(np.cross(X[:, b] - X[:, a], X[:, c] - X[:, a]), axis=1)
    return factor * (6.0 * vol / area) / materials[:, 1]


def rate2_clusters(dt_elem: np.ndarray, neigh: np.ndarray, max_clusters: int = 8):
    """Time-step clusters of rate 2: element e goes to the largest c with
    2^c dt0 <= dt_e (dt0 = min dt_e, c < max_clusters), then clusters are
    lowered until face neighbours differ by at most one level.  Returns
    (cluster int32 [E], dt0)."""
    dt0 = float(np.min(dt_elem))
    c = np.floor(np.log2(dt_elem / dt0) + 1e-12).astype(np.int64)
    c = np.clip(c, 0, max_clusters - 1)
    nb = np.where(neigh >= 0, neigh, np.arange(len(c))[:, None])
    while True:
        lim = np.min(c[nb], axis=1) + 1
        new = np.minimum(c, lim)
        if np.array_equal(new, c):
            break
        c = new
    return c.astype(np.int32), dt0


def permute_elements(mesh: CubeMesh, order: np.ndarray) -> CubeMesh:
    """The same mesh with its elements renumbered: new element i is old
    element order[i] (neighbour ids remapped, faces unchanged)."""
    order = np.asarray(order, dtype=np.int64)
    inv = np.empty_like(order)
    inv[order] = np.arange(len(order))
    nb = mesh.neigh[order]
    neigh = np.where(nb >= 0, inv[np.maximum(nb, 0)], -1).astype(np.int32)
    return CubeMesh(n=mesh.n, h=mesh.h, X=mesh.X[order], V=mesh.V[order], neigh=neigh,
                    nface=mesh.nface[order], orient=mesh.orient[order])


def layered_materials(mesh: CubeMesh, seed: int, layer: float = 1.0 / 3.0, slowdown: float = 1.5):
    """A slower layer over a halfspace: elements whose centroid has
    z > 1 - layer take the layer material, the others the halfspace
    material.  The halfspace material is one draw of random_materials; the
    layer has the same density and both wave speeds divided by `slowdown`.
    Returns (E, 3) float64 columns (rho, cp, cs)."""
    half = random_materials(1, seed)[0]
    lay = np.array([half[0], half[1] / slowdown, half[2] / slowdown])
    top = mesh.X.mean(axis=1)[:, 2] > 1.0 - layer
    return np.where(top[:, None], lay[None, :], half[None, :])
