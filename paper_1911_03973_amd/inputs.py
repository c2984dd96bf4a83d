"""Seeded synthetic inputs for the element-based solvers.

This module only *generates data*: meshes of the unit square / unit cube, node
jitter, Dirichlet node sets, right-hand-side functions sampled at the nodes and
the parameter draws of the batched workload.  It contains none of the finite
element arithmetic (no local matrices, no residual, no solver), so the CPU
oracle's tests and the GPU path can both consume exactly the same inputs.

Mesh conventions (Section 1, Fig. 1 of the paper: the unit square split into
triangles; the uniform refinement levels of Section 3):

* 2-D, ``n`` squares per side, ``(n+1)**2`` nodes numbered row-major with the
  first coordinate fastest: node (i, j) -> j*(n+1) + i at (i/n, j/n).
  Square (i, j) with corners a=(i,j), b=(i+1,j), c=(i+1,j+1), d=(i,j+1) is cut
  along its (0,0)-(1,1) diagonal into the triangles [a,b,c] and [a,c,d].
  For n=1 this gives nodes 0:(0,0) 1:(1,0) 2:(0,1) 3:(1,1) and triangles
  [0,1,3], [0,3,2]; n=2 gives the 8-element / 9-node mesh.
* 3-D, ``n`` cubes per side, ``(n+1)**3`` nodes numbered (i, j, k) ->
  (k*(n+1) + j)*(n+1) + i.  Every cube is split into the 6 Kuhn
  (Freudenthal) tetrahedra [v000, v000+e_a, v000+e_a+e_b, v111], one per
  permutation (a, b, c) of the axes.
* Element order: cells (squares / cubes) are visited either row-major or along
  a Morton (Z-order) curve of the cell index; the 2 or 6 simplices of one cell
  are consecutive.  The Morton order gives every run of consecutive elements a
  compact footprint, which is what the GPU path's element chunks rely on for
  locality; the mathematics does not depend on the order.
"""
from __future__ import annotations

import dataclasses
import itertools

import numpy as np

__all__ = [
    "Mesh",
    "square_mesh",
    "square_mesh_p2",
    "cube_mesh",
    "cube_hierarchy",
    "boundary_nodes",
    "dirichlet_nodes",
    "random_sine",
    "random_sine_params",
    "batched_params",
]


@dataclasses.dataclass
class Mesh:
    """A simplicial mesh: node coordinates and element -> node table.

    coords : float64 array (n_nodes, dim)
    elems  : int32 array (n_elems, dim+1), 0-based node ids
    n      : cells per side of the generating grid (0 if not structured)
    """

    coords: np.ndarray
    elems: np.ndarray
    n: int = 0

    @property
    def dim(self) -> int:
        return int(self.coords.shape[1])

    @property
    def nb(self) -> int:
        return int(self.elems.shape[1])

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.elems.shape[0])


def _part1by1(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.uint64) & np.uint64(0xFFFFFFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x0000FFFF0000FFFF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x00FF00FF00FF00FF)
    v = (v | (v << np.uint64(4))) & np.uint64(0x0F0F0F0F0F0F0F0F)
    v = (v | (v << np.uint64(2))) & np.uint64(0x3333333333333333)
    v = (v | (v << np.uint64(1))) & np.uint64(0x5555555555555555)
    return v


def _part1by2(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
    return v


def _cell_order(codes: np.ndarray, order: str) -> np.ndarray:
    if order == "rowmajor":
        return np.arange(codes.shape[0], dtype=np.int64)
    if order == "morton":
        return np.argsort(codes, kind="stable")
    raise ValueError(f"unknown element order {order!r}")


def _jitter(coords: np.ndarray, interior: np.ndarray, h: float, amount: float, seed: int) -> None:
    if amount == 0.0:
        return
    rng = np.random.default_rng(seed)
    d = rng.uniform(-amount * h, amount * h, size=(int(interior.sum()), coords.shape[1]))
    coords[interior] += d


def square_mesh(n: int, order: str = "morton", jitter: float = 0.0, seed: int = 0) -> Mesh:
    """Uniform diagonal-cut triangulation of (0,1)^2 with n x n squares.

    jitter: interior nodes move by U(-jitter*h, jitter*h) per coordinate
    (h = 1/n), drawn from numpy's default_rng(seed).
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    h = 1.0 / n
    m = n + 1
    jj, ii = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    coords = np.stack([ii.ravel() * h, jj.ravel() * h], axis=1).astype(np.float64)
    interior = ((ii > 0) & (ii < n) & (jj > 0) & (jj < n)).ravel()
    _jitter(coords, interior, h, jitter, seed)

    cj, ci = np.meshgrid(np.arange(n, dtype=np.int64), np.arange(n, dtype=np.int64), indexing="ij")
    ci = ci.ravel()
    cj = cj.ravel()
    perm = _cell_order(_part1by1(ci) | (_part1by1(cj) << np.uint64(1)), order)
    ci = ci[perm]
    cj = cj[perm]
    a = cj * m + ci
    b = a + 1
    c = a + m + 1
    d = a + m
    t1 = np.stack([a, b, c], axis=1)
    t2 = np.stack([a, c, d], axis=1)
    elems = np.stack([t1, t2], axis=1).reshape(-1, 3).astype(np.int32)
    return Mesh(coords=coords, elems=elems, n=n)


def square_mesh_p2(n: int, order: str = "morton", jitter: float = 0.0, seed: int = 0) -> Mesh:
    """Quadratic (P2) triangles on the diagonal-cut mesh of n x n squares.

    The nodes are the points of the (2n+1) x (2n+1) lattice of half-steps:
    lattice point (I, J) -> J*(2n+1) + I; even-even points are the triangle
    vertices, the others the midpoints of the horizontal, vertical and
    diagonal edges (the diagonal midpoint is the square's centre).  Each
    element lists its vertices [a, b, c] as in :func:`square_mesh`, then the
    midpoints of its edges (a, b), (b, c), (c, a).  Jitter moves the interior
    vertices as in :func:`square_mesh` (same seed, same draws); midpoints stay
    at the middle of their (straight) edges.  ``Mesh.n`` is 2n, the lattice
    size, so :func:`boundary_nodes` finds the boundary by lattice index.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    base = square_mesh(n, order=order, jitter=jitter, seed=seed)
    m, M = n + 1, 2 * n + 1
    vi, vj = np.arange(base.n_nodes) % m, np.arange(base.n_nodes) // m
    lat = (2 * vj) * M + 2 * vi  # lattice id of every vertex
    coords = np.zeros((M * M, 2))
    coords[lat] = base.coords
    e = base.elems.astype(np.int64)
    la, lb, lc = lat[e[:, 0]], lat[e[:, 1]], lat[e[:, 2]]

    def mid(p, q):  # lattice midpoint of two lattice points (both even-even)
        return ((p // M + q // M) // 2) * M + (p % M + q % M) // 2

    mab, mbc, mca = mid(la, lb), mid(lb, lc), mid(lc, la)
    for mm, p, q in ((mab, la, lb), (mbc, lb, lc), (mca, lc, la)):
        coords[mm] = 0.5 * (coords[p] + coords[q])
    elems = np.stack([la, lb, lc, mab, mbc, mca], axis=1).astype(np.int32)
    return Mesh(coords=coords, elems=elems, n=2 * n)


def cube_mesh_p2(n: int, order: str = "morton", jitter: float = 0.0, seed: int = 0) -> Mesh:
    """Quadratic (P2) tetrahedra on the Kuhn mesh of n^3 cubes.

    The nodes are the points of the (2n+1)^3 lattice of half-steps: lattice
    point (I, J, K) -> (K*(2n+1) + J)*(2n+1) + I; even points are the
    tetrahedron vertices, the others the midpoints of the lattice edges and of
    the face and cube diagonals of the split.  Each element lists its vertices
    [v0, v1, v2, v3] as in :func:`cube_mesh`, then the midpoints of its edges
    (0,1), (0,2), (0,3), (1,2), (1,3), (2,3).  Jitter moves the interior
    vertices as in :func:`cube_mesh` (same seed, same draws); midpoints stay at
    the middle of their (straight) edges.  ``Mesh.n`` is 2n, the lattice size.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    base = cube_mesh(n, order=order, jitter=jitter, seed=seed)
    m, M = n + 1, 2 * n + 1
    ids = np.arange(base.n_nodes)
    vi, vj, vk = ids % m, (ids // m) % m, ids // (m * m)
    lat = ((2 * vk) * M + 2 * vj) * M + 2 * vi  # lattice id of every vertex
    coords = np.zeros((M ** 3, 3))
    coords[lat] = base.coords
    e = base.elems.astype(np.int64)
    lv = [lat[e[:, a]] for a in range(4)]

    def mid(p, q):  # lattice midpoint of two even lattice points
        pi, pj, pk = p % M, (p // M) % M, p // (M * M)
        qi, qj, qk = q % M, (q // M) % M, q // (M * M)
        return (((pk + qk) // 2) * M + (pj + qj) // 2) * M + (pi + qi) // 2

    mids = []
    for a, b in ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)):
        mm = mid(lv[a], lv[b])
        coords[mm] = 0.5 * (coords[lv[a]] + coords[lv[b]])
        mids.append(mm)
    elems = np.stack(lv + mids, axis=1).astype(np.int32)
    return Mesh(coords=coords, elems=elems, n=2 * n)


def square_hierarchy(mesh: Mesh, coarsest: int = 16, order: str = "morton") -> list:
    """The meshes of n, n/2, ..., coarsest squares per side nested in `mesh`
    (a square_mesh of n squares, n / coarsest a power of two): coarse node
    (I, J) of level l takes the coordinates of fine node (2^l I, 2^l J), so a
    jittered mesh keeps its jitter on every level.  Finest first."""
    n = mesh.n
    if n <= 0 or coarsest < 1 or n % coarsest or (n // coarsest) & (n // coarsest - 1):
        raise ValueError("n / coarsest must be a power of two")
    out = [mesh]
    m = n + 1
    level = 1
    while n >> level >= coarsest:
        nl = n >> level
        c = square_mesh(nl, order=order)
        ml = nl + 1
        jj, ii = np.meshgrid(np.arange(ml), np.arange(ml), indexing="ij")
        fine = (jj.ravel() << level) * m + (ii.ravel() << level)
        out.append(Mesh(coords=np.ascontiguousarray(mesh.coords[fine]), elems=c.elems, n=nl))
        level += 1
    return out


def cube_hierarchy(mesh: Mesh, coarsest: int = 5, order: str = "morton") -> list:
    """The meshes of n, n/2, ..., coarsest cubes per side nested in `mesh` (a
    cube_mesh of n cubes, n / coarsest a power of two): coarse node (I, J, K)
    of level l takes the coordinates of fine node (2^l I, 2^l J, 2^l K).  The
    Kuhn split of every level uses the same (0,0,0)-(1,1,1) diagonal, so each
    coarse tetrahedron is a union of fine ones.  Finest first."""
    n = mesh.n
    if n <= 0 or coarsest < 1 or n % coarsest or (n // coarsest) & (n // coarsest - 1):
        raise ValueError("n / coarsest must be a power of two")
    out = [mesh]
    m = n + 1
    level = 1
    while n >> level >= coarsest:
        nl = n >> level
        c = cube_mesh(nl, order=order)
        ml = nl + 1
        kk, jj, ii = np.meshgrid(np.arange(ml), np.arange(ml), np.arange(ml), indexing="ij")
        fine = ((kk.ravel() << level) * m + (jj.ravel() << level)) * m + (ii.ravel() << level)
        out.append(Mesh(coords=np.ascontiguousarray(mesh.coords[fine]), elems=c.elems, n=nl))
        level += 1
    return out


def cube_mesh(n: int, order: str = "morton", jitter: float = 0.0, seed: int = 0) -> Mesh:
    """Kuhn triangulation of (0,1)^3: n^3 cubes, 6 tetrahedra each."""
    if n < 1:
        raise ValueError("n must be >= 1")
    h = 1.0 / n
    m = n + 1
    kk, jj, ii = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    coords = np.stack([ii.ravel() * h, jj.ravel() * h, kk.ravel() * h], axis=1).astype(np.float64)
    interior = ((ii > 0) & (ii < n) & (jj > 0) & (jj < n) & (kk > 0) & (kk < n)).ravel()
    _jitter(coords, interior, h, jitter, seed)

    ck, cj, ci = np.meshgrid(
        np.arange(n, dtype=np.int64), np.arange(n, dtype=np.int64), np.arange(n, dtype=np.int64),
        indexing="ij",
    )
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    code = _part1by2(ci) | (_part1by2(cj) << np.uint64(1)) | (_part1by2(ck) << np.uint64(2))
    perm = _cell_order(code, order)
    ci, cj, ck = ci[perm], cj[perm], ck[perm]
    v000 = (ck * m + cj) * m + ci
    step = np.array([1, m, m * m], dtype=np.int64)  # node-id offset of a unit move along x, y, z
    v111 = v000 + step.sum()
    tets = []
    for p in itertools.permutations(range(3)):
        v1 = v000 + step[p[0]]
        v2 = v1 + step[p[1]]
        tets.append(np.stack([v000, v1, v2, v111], axis=1))
    elems = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    return Mesh(coords=coords, elems=elems, n=n)


def boundary_nodes(mesh: Mesh, which: str = "all") -> np.ndarray:
    """Node ids on the boundary of the unit square/cube (sorted, int32).

    which = "all"  : every node of the boundary
    which = "x2=0" : only the nodes with second coordinate 0 (the bottom edge)
    Detection uses the generating grid index, so jittered meshes (interior-only
    jitter) are handled exactly.
    """
    n = mesh.n
    if n <= 0:
        raise ValueError("boundary_nodes needs a structured mesh")
    m = n + 1
    ids = np.arange(mesh.n_nodes, dtype=np.int64)
    i = ids % m
    j = (ids // m) % m
    if which == "x2=0":
        sel = j == 0
    elif which == "all":
        sel = (i == 0) | (i == n) | (j == 0) | (j == n)
        if mesh.dim == 3:
            k = ids // (m * m)
            sel |= (k == 0) | (k == n)
    else:
        raise ValueError(f"unknown boundary part {which!r}")
    return ids[sel].astype(np.int32)


def dirichlet_nodes(mesh: Mesh, which: str = "all") -> np.ndarray:
    """Alias of :func:`boundary_nodes` for the Dirichlet part of the boundary."""
    return boundary_nodes(mesh, which)


def random_sine_params(seed: int, terms: int = 8, max_freq: int = 8):
    """Amplitudes a_k ~ N(0,1), then frequencies p_k, q_k ~ U{1..max_freq}.

    Drawn in that order (a, then p, then q) from numpy default_rng(seed).
    """
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(terms)
    p = rng.integers(1, max_freq + 1, size=terms)
    q = rng.integers(1, max_freq + 1, size=terms)
    return a, p, q


def random_sine(coords: np.ndarray, seed: int, terms: int = 8, max_freq: int = 8) -> np.ndarray:
    """f(x) = sum_k a_k sin(pi p_k x1) sin(pi q_k x2), sampled at the nodes (float64)."""
    a, p, q = random_sine_params(seed, terms, max_freq)
    x1 = coords[:, 0]
    x2 = coords[:, 1]
    f = np.zeros(coords.shape[0], dtype=np.float64)
    for ak, pk, qk in zip(a, p, q):
        f += ak * np.sin(np.pi * pk * x1) * np.sin(np.pi * qk * x2)
    return f


def batched_params(count: int = 256, base_seed: int = 1000, n_min: int = 32, n_max: int = 512):
    """Per-problem (n, nu, seed) for the batched workload.

    n ~ U{n_min..n_max}, nu = 10**U(-3, 3), drawn from default_rng(base_seed);
    problem i uses seed base_seed + 1 + i for its right-hand side.
    """
    rng = np.random.default_rng(base_seed)
    ns = rng.integers(n_min, n_max + 1, size=count)
    nus = 10.0 ** rng.uniform(-3.0, 3.0, size=count)
    return [(int(ns[i]), float(nus[i]), base_seed + 1 + i) for i in range(count)]
