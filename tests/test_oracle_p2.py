"""Pins of the P2 triangle oracle (oracle/p2.py) against facts of the
quadratic Lagrange space, none of which re-derive its quadrature."""
import numpy as np
import pytest

import oracle
import oracle.p2 as op2
from paper_1911_03973_amd import inputs


def test_stiffness_annihilates_constants_and_is_symmetric_psd():
    mesh = inputs.square_mesh_p2(3, jitter=0.25, seed=2)
    K, M, area = op2.local_matrices_p2(mesh.coords, mesh.elems)
    assert np.abs(K.sum(axis=2)).max() <= 1e-12 * np.abs(K).max()
    assert np.abs(K - K.transpose(0, 2, 1)).max() <= 1e-13 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert ev[:, 0].min() >= -1e-12 * ev.max()
    assert np.all(ev[:, 1] > 1e-6 * ev[:, -1])  # only the constants in the kernel


def test_mass_rows_integrate_the_basis():
    """sum_j M_ij = int phi_i: 0 for the vertex functions, area/3 for the
    midpoint functions; M is symmetric positive definite."""
    mesh = inputs.square_mesh_p2(3, jitter=0.25, seed=3)
    K, M, area = op2.local_matrices_p2(mesh.coords, mesh.elems)
    rows = M.sum(axis=2)
    assert np.abs(rows[:, :3]).max() <= 1e-14
    assert np.abs(rows[:, 3:] - area[:, None] / 3).max() <= 1e-14
    assert np.abs(M.sum(axis=(1, 2)) - area).max() <= 1e-14
    assert np.linalg.eigvalsh(M)[:, 0].min() > 0


def test_reference_triangle_area_and_mass_diagonal_ratio():
    """On any triangle the mass matrix is area/180 times a fixed integer matrix
    with 6 on the vertex and 32 on the midpoint diagonal entries."""
    mesh = inputs.Mesh(coords=np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [0.5, 0.0], [0.5, 0.5], [0.0, 0.5]]),
                       elems=np.array([[0, 1, 2, 3, 4, 5]], dtype=np.int32))
    K, M, area = op2.local_matrices_p2(mesh.coords, mesh.elems)
    assert area[0] == pytest.approx(0.5)
    S = M[0] * 180 / area[0]
    assert np.abs(S - np.round(S)).max() <= 1e-12
    assert np.allclose(np.diag(S), [6, 6, 6, 32, 32, 32])


def _quadratic(x, y):
    return 1.0 + x - 2.0 * y + 3.0 * x * x - x * y + 2.0 * y * y


@pytest.mark.parametrize("nu,jitter", [(0.0, 0.0), (2.0, 0.25), (37.5, 0.2)])
def test_quadratic_solution_is_reproduced_exactly(nu, jitter):
    """With u quadratic, f = -Lap u + nu u is quadratic and its nodal
    interpolant is exact, so b = M f is the exact Galerkin load and the P2
    solution equals u at every node (a dropped or wrong entry of K or M, or a
    wrong basis, breaks this)."""
    mesh = inputs.square_mesh_p2(6, jitter=jitter, seed=5)
    K, M, _ = op2.local_matrices_p2(mesh.coords, mesh.elems)
    x, y = mesh.coords[:, 0], mesh.coords[:, 1]
    u = _quadratic(x, y)
    lap = 2 * 3.0 + 2 * 2.0
    f = -lap + nu * u
    b = oracle.rhs(mesh.n_nodes, mesh.elems, M, f)
    nd = inputs.boundary_nodes(mesh, "all")
    mask = oracle.mask_from_nodes(mesh.n_nodes, nd)
    x0 = np.zeros(mesh.n_nodes)
    x0[nd] = u[nd]
    xs, info = oracle.pcg(mesh.n_nodes, mesh.elems, K, M, nu, b, mask, x0, rtol=1e-14, max_iter=5000,
                          raise_on_noconv=False)
    assert np.abs(xs - u).max() <= 1e-10 * np.abs(u).max(), info


def test_nodal_error_falls_faster_than_p1():
    """For a smooth solution the P2 nodal error falls by about 2^3 or more per
    halving of h (P1: about 2^2)."""
    errs = []
    for n in (4, 8, 16):
        mesh = inputs.square_mesh_p2(n)
        K, M, _ = op2.local_matrices_p2(mesh.coords, mesh.elems)
        x, y = mesh.coords[:, 0], mesh.coords[:, 1]
        u = np.sin(np.pi * x) * np.sin(np.pi * y)
        f = (2 * np.pi ** 2 + 1.0) * u
        b = oracle.rhs(mesh.n_nodes, mesh.elems, M, f)
        nd = inputs.boundary_nodes(mesh, "all")
        mask = oracle.mask_from_nodes(mesh.n_nodes, nd)
        xs, _ = oracle.pcg(mesh.n_nodes, mesh.elems, K, M, 1.0, b, mask, np.zeros(mesh.n_nodes), rtol=1e-13,
                           max_iter=5000)
        errs.append(np.abs(xs - u).max())
    rates = [errs[i] / errs[i + 1] for i in range(2)]
    assert min(rates) > 6.0, (errs, rates)


# ---- P2 tetrahedra ----

def test_tet_stiffness_annihilates_constants_and_is_symmetric_psd():
    mesh = inputs.cube_mesh_p2(2, jitter=0.2, seed=2)
    K, M, vol = op2.local_matrices_p2_tet(mesh.coords, mesh.elems)
    assert np.abs(K.sum(axis=2)).max() <= 1e-12 * np.abs(K).max()
    assert np.abs(K - K.transpose(0, 2, 1)).max() <= 1e-13 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert ev[:, 0].min() >= -1e-12 * ev.max()
    assert np.all(ev[:, 1] > 1e-6 * ev[:, -1])
    assert abs(vol.sum() - 1.0) <= 1e-13  # the tetrahedra tile the unit cube


def test_tet_mass_is_the_textbook_matrix():
    """sum_j M_ij = int phi_i: -vol/20 for vertices, vol/5 for midpoints; and
    M = vol/420 times the integer matrix with 6 / 1 between vertices, -4 / -6
    between a vertex and an edge through / not through it, 32 / 16 / 8
    between an edge and itself / an edge sharing a vertex / the opposite edge."""
    mesh = inputs.cube_mesh_p2(2, jitter=0.2, seed=3)
    K, M, vol = op2.local_matrices_p2_tet(mesh.coords, mesh.elems)
    rows = M.sum(axis=2)
    assert np.abs(rows[:, :4] + vol[:, None] / 20).max() <= 1e-15
    assert np.abs(rows[:, 4:] - vol[:, None] / 5).max() <= 1e-15
    E = op2.TET_EDGES
    S = np.empty((10, 10))
    for i in range(4):
        for j in range(4):
            S[i, j] = 6 if i == j else 1
        for e, (u, v) in enumerate(E):
            S[i, 4 + e] = S[4 + e, i] = -4 if i in (u, v) else -6
    for a, ea in enumerate(E):
        for b, eb in enumerate(E):
            shared = len(set(ea) & set(eb))
            S[4 + a, 4 + b] = 32 if shared == 2 else (16 if shared == 1 else 8)
    assert np.abs(M - vol[:, None, None] / 420 * S[None]).max() <= 1e-15


def _quadratic3(x, y, z):
    return 1.0 + x - 2.0 * y + 0.5 * z + 3.0 * x * x - x * y + 2.0 * y * y + y * z - z * z + 0.5 * x * z


@pytest.mark.parametrize("nu,jitter", [(0.0, 0.0), (2.0, 0.2), (37.5, 0.15)])
def test_tet_quadratic_solution_is_reproduced_exactly(nu, jitter):
    mesh = inputs.cube_mesh_p2(3, jitter=jitter, seed=5)
    K, M, _ = op2.local_matrices_p2_tet(mesh.coords, mesh.elems)
    x, y, z = mesh.coords[:, 0], mesh.coords[:, 1], mesh.coords[:, 2]
    u = _quadratic3(x, y, z)
    lap = 2 * 3.0 + 2 * 2.0 - 2 * 1.0
    f = -lap + nu * u
    b = oracle.rhs(mesh.n_nodes, mesh.elems, M, f)
    nd = inputs.boundary_nodes(mesh, "all")
    mask = oracle.mask_from_nodes(mesh.n_nodes, nd)
    x0 = np.zeros(mesh.n_nodes)
    x0[nd] = u[nd]
    xs, info = oracle.pcg(mesh.n_nodes, mesh.elems, K, M, nu, b, mask, x0, rtol=1e-14, max_iter=5000,
                          raise_on_noconv=False)
    assert np.abs(xs - u).max() <= 1e-10 * np.abs(u).max(), info


def test_tet_nodal_error_falls_faster_than_p1():
    errs = []
    for n in (2, 4, 8):
        mesh = inputs.cube_mesh_p2(n)
        K, M, _ = op2.local_matrices_p2_tet(mesh.coords, mesh.elems)
        x, y, z = mesh.coords[:, 0], mesh.coords[:, 1], mesh.coords[:, 2]
        u = np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)
        f = (3 * np.pi ** 2 + 1.0) * u
        b = oracle.rhs(mesh.n_nodes, mesh.elems, M, f)
        nd = inputs.boundary_nodes(mesh, "all")
        mask = oracle.mask_from_nodes(mesh.n_nodes, nd)
        xs, _ = oracle.pcg(mesh.n_nodes, mesh.elems, K, M, 1.0, b, mask, np.zeros(mesh.n_nodes), rtol=1e-13,
                           max_iter=5000)
        errs.append(np.abs(xs - u).max())
    rates = [errs[i] / errs[i + 1] for i in range(2)]
    assert min(rates) > 6.0, (errs, rates)
