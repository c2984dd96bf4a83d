"""FP64 reference of the quadratic (P2) triangle matrices (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of the
benchmark may import this module.  It shares no code with the GPU library.

The paper's outlook names higher-order elements as the next step; it gives no
formulas for them.  This module takes the textbook definition: on a straight
triangle with barycentric coordinates lambda_0..2 (vertex k <-> lambda_k), the
six Lagrange basis functions
    phi_k = lambda_k (2 lambda_k - 1)        k = 0, 1, 2  (vertices)
    phi_3 = 4 lambda_0 lambda_1, phi_4 = 4 lambda_1 lambda_2,
    phi_5 = 4 lambda_2 lambda_0                           (edge midpoints)
and the local matrices K_ij = int grad phi_i . grad phi_j, M_ij = int phi_i
phi_j, as in eq. (2) for P1.  The integrals are evaluated by a collapsed
(Duffy) tensor Gauss-Legendre rule on the reference triangle, exact for the
degree-4 integrands of M, with the affine map of the element; the GPU library
integrates barycentric monomials in closed form instead.

For tetrahedra (`local_matrices_p2_tet`) the ten functions are
    phi_k = lambda_k (2 lambda_k - 1)        k = 0..3     (vertices)
    phi_{4+e} = 4 lambda_u lambda_v          e = (0,1), (0,2), (0,3), (1,2), (1,3), (2,3)
integrated by the collapsed (Stroud conical product) Gauss rule on the
reference tetrahedron, exact for the degree-4 mass integrands.

Pins (tests/test_oracle_p2.py): K annihilates constants, the vertex rows of M
integrate to zero and the midpoint rows to area/3, the discrete solution of a
problem whose exact solution is quadratic is that quadratic at every node, and
the nodal error of a smooth solution falls faster than the P1 rate.
"""
from __future__ import annotations

import numpy as np

NB = 6


def _rule(k=4):
    """Points (xi, eta) and weights of the collapsed Gauss rule on the reference
    triangle {xi, eta >= 0, xi + eta <= 1} (weights sum to 1/2)."""
    g, w = np.polynomial.legendre.leggauss(k)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    xi, eta, wt = [], [], []
    for a in range(k):
        for b in range(k):
            u, v = g[a], g[b]
            xi.append(u)
            eta.append(v * (1.0 - u))
            wt.append(w[a] * w[b] * (1.0 - u))
    return np.array(xi), np.array(eta), np.array(wt)


def _basis(l0, l1, l2):
    """Values of the six basis functions at barycentric points (arrays)."""
    return np.stack([l0 * (2 * l0 - 1), l1 * (2 * l1 - 1), l2 * (2 * l2 - 1),
                     4 * l0 * l1, 4 * l1 * l2, 4 * l2 * l0])


def _basis_grad_bary(l0, l1, l2):
    """d phi_k / d lambda_a, shape (6, 3, n_points)."""
    z = np.zeros_like(l0)
    return np.stack([
        np.stack([4 * l0 - 1, z, z]),
        np.stack([z, 4 * l1 - 1, z]),
        np.stack([z, z, 4 * l2 - 1]),
        np.stack([4 * l1, 4 * l0, z]),
        np.stack([z, 4 * l2, 4 * l1]),
        np.stack([4 * l2, z, 4 * l0]),
    ])


def local_matrices_p2(coords, elems):
    """K_e, M_e (n_elems, 6, 6) and area (n_elems,) of straight P2 triangles.

    coords (n_nodes, 2); elems (n_elems, 6): vertices, then the midpoints of
    edges (0,1), (1,2), (2,0).  Only the vertices enter the (affine) map."""
    coords = np.asarray(coords, dtype=np.float64)
    elems = np.asarray(elems, dtype=np.int64)
    xi, eta, wt = _rule(4)
    l0, l1, l2 = 1.0 - xi - eta, xi, eta
    phi = _basis(l0, l1, l2)                 # (6, q)
    dphi = _basis_grad_bary(l0, l1, l2)      # (6, 3, q)
    ne = elems.shape[0]
    K = np.empty((ne, NB, NB))
    M = np.empty((ne, NB, NB))
    area = np.empty(ne)
    Mref = np.einsum("iq,jq,q->ij", phi, phi, wt)  # int over the reference triangle
    step = 32768
    for e0 in range(0, ne, step):  # blocks of elements, each by the same formulas
        p = coords[elems[e0:e0 + step, :3]]                       # (b, 3, 2)
        B = np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]], axis=2)  # columns: edge vectors
        det = np.linalg.det(B)
        Binv = np.linalg.inv(B)                                   # rows: grad lambda_1, grad lambda_2
        gl = np.concatenate([-(Binv[:, 0:1] + Binv[:, 1:2]), Binv], axis=1)  # (b, 3, 2)
        G = np.einsum("kaq,ead->ekqd", dphi, gl)                   # grad phi_k at the points
        jac = np.abs(det)
        K[e0:e0 + step] = np.einsum("eiqd,ejqd,q->eij", G, G, wt) * jac[:, None, None]
        M[e0:e0 + step] = Mref[None] * jac[:, None, None]
        area[e0:e0 + step] = 0.5 * jac
    return K, M, area


TET_EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def _rule_tet(k=4):
    """Points (x, y, z) and weights of the collapsed Gauss rule on the reference
    tetrahedron {x, y, z >= 0, x + y + z <= 1} (weights sum to 1/6): the cube
    point (u, v, w) maps to (u, v (1 - u), w (1 - u)(1 - v)) with Jacobian
    (1 - u)^2 (1 - v)."""
    g, w = np.polynomial.legendre.leggauss(k)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    pts, wt = [], []
    for a in range(k):
        for b in range(k):
            for c in range(k):
                u, v, t = g[a], g[b], g[c]
                pts.append((u, v * (1.0 - u), t * (1.0 - u) * (1.0 - v)))
                wt.append(w[a] * w[b] * w[c] * (1.0 - u) ** 2 * (1.0 - v))
    p = np.array(pts)
    return p[:, 0], p[:, 1], p[:, 2], np.array(wt)


def local_matrices_p2_tet(coords, elems):
    """K_e, M_e (n_elems, 10, 10) and volume (n_elems,) of straight P2
    tetrahedra.  coords (n_nodes, 3); elems (n_elems, 10): vertices, then the
    midpoints of the edges in TET_EDGES order.  Only the vertices enter the
    (affine) map."""
    coords = np.asarray(coords, dtype=np.float64)
    elems = np.asarray(elems, dtype=np.int64)
    x, y, z, wt = _rule_tet(4)
    lam = np.stack([1.0 - x - y - z, x, y, z])  # (4, q)
    nq = wt.size
    phi = np.empty((10, nq))
    dphi = np.zeros((10, 4, nq))  # d phi_k / d lambda_a
    for k in range(4):
        phi[k] = lam[k] * (2.0 * lam[k] - 1.0)
        dphi[k, k] = 4.0 * lam[k] - 1.0
    for e, (u, v) in enumerate(TET_EDGES):
        phi[4 + e] = 4.0 * lam[u] * lam[v]
        dphi[4 + e, u] = 4.0 * lam[v]
        dphi[4 + e, v] = 4.0 * lam[u]
    ne = elems.shape[0]
    K = np.empty((ne, 10, 10))
    M = np.empty((ne, 10, 10))
    vol = np.empty(ne)
    Mref = np.einsum("iq,jq,q->ij", phi, phi, wt)  # int over the reference tetrahedron
    step = 16384
    for e0 in range(0, ne, step):
        p = coords[elems[e0:e0 + step, :4]]                                   # (b, 4, 3)
        B = np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]], axis=2)  # columns: edges
        det = np.linalg.det(B)
        Binv = np.linalg.inv(B)                                               # rows: grad lambda_1..3
        gl = np.concatenate([-Binv.sum(axis=1, keepdims=True), Binv], axis=1)  # (b, 4, 3)
        G = np.einsum("kaq,ead->ekqd", dphi, gl)
        jac = np.abs(det)
        K[e0:e0 + step] = np.einsum("eiqd,ejqd,q->eij", G, G, wt) * jac[:, None, None]
        M[e0:e0 + step] = Mref[None] * jac[:, None, None]
        vol[e0:e0 + step] = jac / 6.0
    return K, M, vol
