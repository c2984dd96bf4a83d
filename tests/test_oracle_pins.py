"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these tests compares the oracle with itself: each checks it against a
closed form, a hand-derived value, a different formula, an invariant, a
library routine (DST-I Poisson solve, dense linear algebra) or an error bound
printed in the paper.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.fft

import oracle
from paper_1911_03973_amd import inputs


def _load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as fh:
        return json.load(fh)


def dense_from_oracle(mesh, K, M, nu, free=None):
    """Columns A e_j obtained from the oracle residual with b = 0."""
    n = mesh.n_nodes
    cols = free if free is not None else np.arange(n)
    A = np.zeros((n, len(cols)))
    for k, j in enumerate(cols):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, k] = -oracle.residual(n, mesh.elems, K, M, nu, None, e)
    return A


# --------------------------------------------------------------------------
# Fig. 1 meshes (Section 1)
# --------------------------------------------------------------------------

def test_fig1_mesh_sizes():
    m1 = inputs.square_mesh(1, order="rowmajor")
    m2 = inputs.square_mesh(2, order="rowmajor")
    assert (m1.n_nodes, m1.n_elems) == (4, 2)
    assert (m2.n_nodes, m2.n_elems) == (9, 8)


def test_two_element_mesh_values(golden_dir):
    g = _load(golden_dir, "fig1_two_element.json")
    m = inputs.square_mesh(1, order="rowmajor")
    np.testing.assert_array_equal(m.coords, np.array(g["coords"], float))
    np.testing.assert_array_equal(m.elems, np.array(g["elems"]))
    K, M, vol = oracle.local_matrices(m.coords, m.elems)
    np.testing.assert_allclose(2 * K, np.array(g["K_e_times_2"], float), atol=1e-15)
    np.testing.assert_allclose(24 * M, np.array(g["M_e_times_24"], float), atol=1e-14)
    Kd = dense_from_oracle(m, K, M, 0.0)
    np.testing.assert_allclose(2 * Kd, np.array(g["K_times_2"], float), atol=1e-15)
    Md = dense_from_oracle(m, np.zeros_like(K), M, 1.0)
    np.testing.assert_allclose(24 * Md, np.array(g["M_times_24"], float), atol=1e-14)
    b = oracle.rhs(4, m.elems, M, np.ones(4))
    np.testing.assert_allclose(6 * b, np.array(g["b_times_6_for_f_equal_1"], float), atol=1e-15)


def test_eight_element_mesh_values(golden_dir):
    g = _load(golden_dir, "fig1_eight_element.json")
    m = inputs.square_mesh(g["n_squares_per_side"], order="rowmajor")
    assert (m.n_nodes, m.n_elems) == (g["n_nodes"], g["n_elems"])
    c = g["centre_node"]
    K, M, _ = oracle.local_matrices(m.coords, m.elems)
    Kd = dense_from_oracle(m, K, M, 0.0)
    np.testing.assert_allclose(Kd[c], np.array(g["K_centre_row"], float), atol=1e-14)
    b = oracle.rhs(m.n_nodes, m.elems, M, np.ones(m.n_nodes))
    assert b[c] == pytest.approx(g["b_centre_f1"], abs=1e-15)
    nd = inputs.boundary_nodes(m)
    mask = oracle.mask_from_nodes(m.n_nodes, nd)
    x0 = np.zeros(m.n_nodes)
    x, info = oracle.pcg(m.n_nodes, m.elems, K, M, 0.0, b, mask, x0, rtol=1e-14)
    assert x[c] == pytest.approx(g["u_centre_homogeneous_dirichlet"], abs=1e-14)
    x0[nd] = 1.0  # Section 3 boundary data u = 1
    x, info = oracle.pcg(m.n_nodes, m.elems, K, M, 0.0, b, mask, x0, rtol=1e-14)
    assert x[c] == pytest.approx(g["u_centre_dirichlet_one"], abs=1e-14)
    np.testing.assert_array_equal(x[nd], 1.0)


def test_reference_elements(golden_dir):
    g = _load(golden_dir, "reference_elements.json")
    t = g["triangle"]
    K, M, vol = oracle.local_matrices(np.array(t["coords"], float), np.array([[0, 1, 2]], np.int32))
    np.testing.assert_allclose(2 * K[0], t["K_e_times_2"], atol=1e-15)
    np.testing.assert_allclose(24 * M[0], t["M_e_times_24"], atol=1e-14)
    assert vol[0] == pytest.approx(t["vol"], abs=1e-16)
    t = g["tetrahedron"]
    K, M, vol = oracle.local_matrices(np.array(t["coords"], float), np.array([[0, 1, 2, 3]], np.int32))
    np.testing.assert_allclose(6 * K[0], t["K_e_times_6"], atol=1e-14)
    np.testing.assert_allclose(120 * M[0], t["M_e_times_120"], atol=1e-13)
    assert vol[0] == pytest.approx(t["vol"], abs=1e-16)


# --------------------------------------------------------------------------
# Local matrices against an independent construction
# --------------------------------------------------------------------------

def _independent_local(coords, elems):
    """Gradients from the Vandermonde system [1 p_j^T] c = e_i, mass by quadrature.

    The quadrature rules are exact for quadratics: edge midpoints (weights vol/3)
    in 2-D, the symmetric 4-point rule (a=0.5854101966249685, b=0.1381966011250105,
    weights vol/4) in 3-D.
    """
    ne, nb = elems.shape
    d = nb - 1
    K = np.zeros((ne, nb, nb))
    M = np.zeros((ne, nb, nb))
    for e in range(ne):
        P = coords[elems[e]]
        V = np.hstack([np.ones((nb, 1)), P])
        C = np.linalg.solve(V, np.eye(nb))  # column i: coefficients of lambda_i
        grads = C[1:, :].T  # (nb, d)
        vol = abs(np.linalg.det(V)) / math.factorial(d)
        K[e] = vol * grads @ grads.T
        if d == 2:
            pts = np.array([[0.5, 0.5, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5]])
            w = np.full(3, vol / 3)
        else:
            a, b = 0.5854101966249685, 0.1381966011250105
            pts = np.full((4, 4), b) + np.eye(4) * (a - b)
            w = np.full(4, vol / 4)
        for q in range(len(w)):
            lam = pts[q]
            M[e] += w[q] * np.outer(lam, lam)
    return K, M


@pytest.mark.parametrize("dim", [2, 3])
def test_local_matrices_independent_formula(dim):
    mesh = inputs.square_mesh(5, jitter=0.2, seed=3) if dim == 2 else inputs.cube_mesh(3, jitter=0.2, seed=4)
    K, M, vol = oracle.local_matrices(mesh.coords, mesh.elems)
    Ki, Mi = _independent_local(mesh.coords, mesh.elems)
    np.testing.assert_allclose(K, Ki, rtol=0, atol=1e-12 * np.abs(Ki).max())
    np.testing.assert_allclose(M, Mi, rtol=0, atol=1e-13 * np.abs(Mi).max())


# --------------------------------------------------------------------------
# Invariants (P4)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
def test_invariants(dim):
    mesh = inputs.square_mesh(7, jitter=0.2, seed=1) if dim == 2 else inputs.cube_mesh(4, jitter=0.2, seed=2)
    n = mesh.n_nodes
    K, M, vol = oracle.local_matrices(mesh.coords, mesh.elems)
    # rows of K sum to zero: K 1 = 0
    r = oracle.residual(n, mesh.elems, K, M, 0.0, None, np.ones(n))
    assert np.abs(r).max() < 1e-13
    # total mass 1^T M 1 = |Omega| = 1 and sum(b) = int f for f = 1
    Mx = -oracle.residual(n, mesh.elems, np.zeros_like(K), M, 1.0, None, np.ones(n))
    assert Mx.sum() == pytest.approx(1.0, abs=1e-13)
    b = oracle.rhs(n, mesh.elems, M, np.ones(n))
    assert b.sum() == pytest.approx(1.0, abs=1e-13)
    assert vol.sum() == pytest.approx(1.0, abs=1e-13)
    # symmetry, K_e PSD with exactly one zero eigenvalue (constants), M_e SPD
    np.testing.assert_allclose(K, np.transpose(K, (0, 2, 1)), atol=1e-14)
    ev = np.linalg.eigvalsh(K)
    assert (ev[:, 0] > -1e-12).all() and (np.abs(ev[:, 0]) < 1e-12).all() and (ev[:, 1] > 1e-6).all()
    assert (np.linalg.eigvalsh(M)[:, 0] > 0).all()


def test_dilation_scaling():
    rng = np.random.default_rng(7)
    for dim, power in ((2, 0), (3, 1)):
        P = rng.standard_normal((dim + 1, dim))
        el = np.arange(dim + 1, dtype=np.int32)[None, :]
        K1, M1, v1 = oracle.local_matrices(P, el)
        K2, M2, v2 = oracle.local_matrices(2.5 * P, el)
        np.testing.assert_allclose(K2, 2.5 ** power * K1, rtol=1e-12)
        np.testing.assert_allclose(M2, 2.5 ** dim * M1, rtol=1e-12)


# --------------------------------------------------------------------------
# Exact reproduction of linear functions (P5)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim,nu", [(2, 0.0), (2, 3.0), (3, 0.0), (3, 10.0)])
def test_linear_reproduction(dim, nu):
    mesh = inputs.square_mesh(9, jitter=0.2, seed=11) if dim == 2 else inputs.cube_mesh(5, jitter=0.2, seed=12)
    n = mesh.n_nodes
    coef = np.array([0.3, -1.2, 0.7, 2.1])[: dim + 1]
    u = coef[0] + mesh.coords @ coef[1:]
    K, M, _ = oracle.local_matrices(mesh.coords, mesh.elems)
    b = oracle.rhs(n, mesh.elems, M, nu * u)  # f = nu u since -lap(u) = 0
    nd = inputs.boundary_nodes(mesh)
    mask = oracle.mask_from_nodes(n, nd)
    interior = mask == 0
    # the element residual of the exact solution vanishes at interior nodes
    r = oracle.residual(n, mesh.elems, K, M, nu, b, u, mask)
    assert np.abs(r).max() < 1e-13
    if nu == 0.0:
        r0 = oracle.residual(n, mesh.elems, K, M, 0.0, None, u)
        assert np.abs(r0[interior]).max() < 1e-13
    x0 = np.zeros(n)
    x0[nd] = u[nd]
    x, info = oracle.pcg(n, mesh.elems, K, M, nu, b, mask, x0, rtol=1e-13)
    assert np.abs(x - u).max() < 1e-11


# --------------------------------------------------------------------------
# Spectrum formula of Section 3 (P3)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [9, 17, 33])
def test_spectrum_formula(n):
    mesh = inputs.square_mesh(n - 1)
    K, M, _ = oracle.local_matrices(mesh.coords, mesh.elems)
    nd = inputs.boundary_nodes(mesh)
    free = np.setdiff1d(np.arange(mesh.n_nodes), nd)
    A = dense_from_oracle(mesh, K, M, 0.0, free)[free]
    ev = np.sort(np.linalg.eigvalsh(A))
    i = np.arange(1, n - 1)
    lam = 4 * (np.sin(i[:, None] * np.pi / (2 * (n - 1))) ** 2 + np.sin(i[None, :] * np.pi / (2 * (n - 1))) ** 2)
    np.testing.assert_allclose(ev, np.sort(lam.ravel()), atol=1e-12)
    if n == 33:
        assert ev[0] == pytest.approx(0.0192611, abs=1e-7)
        assert ev[-1] == pytest.approx(7.9807389, abs=1e-7)


# --------------------------------------------------------------------------
# Config-1 problem reduces to a DST-I Poisson solve (P6, P10)
# --------------------------------------------------------------------------

def _dst_poisson(N, rhs_interior):
    m = N - 1
    k = np.arange(1, m + 1)
    lam1d = 2 - 2 * np.cos(k * np.pi / (m + 1))
    lam = lam1d[:, None] + lam1d[None, :]
    hat = scipy.fft.dstn(rhs_interior, type=1)
    return scipy.fft.idstn(hat / lam, type=1)


def test_config1_matches_dst_poisson():
    N = 64
    mesh = inputs.square_mesh(N)
    n = mesh.n_nodes
    K, M, _ = oracle.local_matrices(mesh.coords, mesh.elems)
    b = oracle.rhs(n, mesh.elems, M, np.ones(n))
    nd = inputs.boundary_nodes(mesh)
    mask = oracle.mask_from_nodes(n, nd)
    d = oracle.jacobi_diag(n, mesh.elems, K, M, 0.0)
    np.testing.assert_allclose(d[mask == 0], 4.0, atol=1e-13)  # constant diagonal (P10)
    x, info = oracle.pcg(n, mesh.elems, K, M, 0.0, b, mask, np.zeros(n), rtol=1e-12, max_iter=2000)
    h = 1.0 / N
    u = _dst_poisson(N, np.full((N - 1, N - 1), h * h))  # rows: j (x2), cols: i (x1)
    grid = x.reshape(N + 1, N + 1)[1:-1, 1:-1]
    np.testing.assert_allclose(grid, u, atol=1e-12)
    _, info8 = oracle.pcg(n, mesh.elems, K, M, 0.0, b, mask, np.zeros(n), rtol=1e-8)
    assert info8["relres"] <= 1e-8
    assert 100 <= info8["iters"] <= 140


# --------------------------------------------------------------------------
# 3-D Kuhn mesh: interior rows of K are h times the 7-point stencil (P7)
# --------------------------------------------------------------------------

def test_kuhn_mesh_seven_point_stencil():
    N = 6
    h = 1.0 / N
    mesh = inputs.cube_mesh(N)
    n = mesh.n_nodes
    K, M, _ = oracle.local_matrices(mesh.coords, mesh.elems)
    x = np.random.default_rng(5).standard_normal(n)
    Kx = -oracle.residual(n, mesh.elems, K, M, 0.0, None, x)
    g = x.reshape(N + 1, N + 1, N + 1)
    st = 6 * g[1:-1, 1:-1, 1:-1] - (g[2:, 1:-1, 1:-1] + g[:-2, 1:-1, 1:-1] + g[1:-1, 2:, 1:-1]
                                     + g[1:-1, :-2, 1:-1] + g[1:-1, 1:-1, 2:] + g[1:-1, 1:-1, :-2])
    np.testing.assert_allclose(Kx.reshape(N + 1, N + 1, N + 1)[1:-1, 1:-1, 1:-1], h * st, atol=1e-13)


# --------------------------------------------------------------------------
# Brute force: explicit Boolean C_e, dense assembly as in eq. (3) (P8)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
def test_brute_force_dense_assembly(dim):
    mesh = inputs.square_mesh(4, jitter=0.2, seed=21) if dim == 2 else inputs.cube_mesh(2, jitter=0.2, seed=22)
    n, nb = mesh.n_nodes, mesh.nb
    nu = 0.7
    K, M, _ = oracle.local_matrices(mesh.coords, mesh.elems)
    A = np.zeros((n, n))
    for e in range(mesh.n_elems):
        C = np.zeros((nb, n))
        C[np.arange(nb), mesh.elems[e]] = 1.0
        A += C.T @ (K[e] + nu * M[e]) @ C
    rng = np.random.default_rng(3)
    x = rng.standard_normal(n)
    f = rng.standard_normal(n)
    be = oracle.rhs_local(n, mesh.elems, M, f)
    b = sum(np.eye(n)[:, mesh.elems[e]] @ be[e] for e in range(mesh.n_elems))
    np.testing.assert_allclose(oracle.rhs(n, mesh.elems, M, f), b, atol=1e-14)
    np.testing.assert_allclose(oracle.residual(n, mesh.elems, K, M, nu, b, x), b - A @ x, atol=1e-13)
    np.testing.assert_allclose(oracle.residual_alg1(n, mesh.elems, K, M, nu, be, x), b - A @ x, atol=1e-13)
    np.testing.assert_allclose(oracle.jacobi_diag(n, mesh.elems, K, M, nu), np.diag(A), atol=1e-14)
    nd = inputs.boundary_nodes(mesh)
    mask = oracle.mask_from_nodes(n, nd)
    free = mask == 0
    x0 = np.zeros(n)
    x0[nd] = rng.standard_normal(len(nd))
    u = x0.copy()
    u[free] = np.linalg.solve(A[np.ix_(free, free)], b[free] - A[np.ix_(free, ~free)] @ x0[~free])
    xs, info = oracle.pcg(n, mesh.elems, K, M, nu, b, mask, x0, rtol=1e-14)
    np.testing.assert_allclose(xs, u, atol=1e-12)
    # unpreconditioned CG reaches the same solution
    xc, _ = oracle.pcg(n, mesh.elems, K, M, nu, b, mask, x0, rtol=1e-14, jacobi=False)
    np.testing.assert_allclose(xc, u, atol=1e-12)


def test_invalid_inputs_rejected():
    mesh = inputs.square_mesh(2)
    bad = mesh.elems.copy()
    bad[3, 1] = mesh.n_nodes
    with pytest.raises(oracle.OracleError):
        oracle.local_matrices(mesh.coords, bad)
    degenerate = mesh.coords.copy()
    degenerate[4] = degenerate[0]  # collapse the centre onto a corner
    with pytest.raises(oracle.OracleError):
        oracle.local_matrices(degenerate, mesh.elems)


# --------------------------------------------------------------------------
# Richardson and Chebyshev iterations of Section 2 (P9)
# --------------------------------------------------------------------------

def _section3_problem(n_nodes_side=33):
    N = n_nodes_side - 1
    mesh = inputs.square_mesh(N)
    n = mesh.n_nodes
    K, M, _ = oracle.local_matrices(mesh.coords, mesh.elems)
    b = oracle.rhs(n, mesh.elems, M, np.ones(n))
    nd = inputs.boundary_nodes(mesh)
    mask = oracle.mask_from_nodes(n, nd)
    x0 = np.zeros(n)
    x0[nd] = 1.0
    u, _ = oracle.pcg(n, mesh.elems, K, M, 0.0, b, mask, x0, rtol=1e-12, max_iter=5000)
    lam1 = 8 * math.sin(math.pi / (2 * N)) ** 2
    lam2 = 8 * math.sin((N - 1) * math.pi / (2 * N)) ** 2
    return mesh, K, M, b, mask, x0, u, lam1, lam2


def test_chebyshev_and_richardson_bounds():
    mesh, K, M, b, mask, x0, u, l1, l2 = _section3_problem()
    n = mesh.n_nodes
    e0 = np.linalg.norm(x0 - u)
    it = 124
    xr = oracle.richardson(n, mesh.elems, K, M, 0.0, b, mask, x0, l1, l2, it)
    x2 = oracle.cheb2(n, mesh.elems, K, M, 0.0, b, mask, x0, l1, l2, 32, it)
    x3 = oracle.cheb3(n, mesh.elems, K, M, 0.0, b, mask, x0, l1, l2, it)
    q = (math.sqrt(l2) - math.sqrt(l1)) / (math.sqrt(l2) + math.sqrt(l1))
    er, e2, e3 = (np.linalg.norm(v - u) for v in (xr, x2, x3))
    assert er <= ((l2 - l1) / (l2 + l1)) ** it * e0 * (1 + 1e-9)
    assert e3 <= 2 * q ** it * e0 * (1 + 1e-6)
    # "only the 3-level method converged" after 124 iterations on the 33^2 mesh
    assert e3 < 1e-2 * er and e3 < e2
    # The 2-level error after l whole cycles is P_N(A)^l e0, bounded by
    # (2 q^N)^l.  It holds for N = 16 over three cycles and for N = 32 over one;
    # with N = 32 the later cycles exceed it by far: the instability of the
    # root ordering that Section 3 reports.
    for N, cycles in ((16, 3), (32, 1)):
        xc = oracle.cheb2(n, mesh.elems, K, M, 0.0, b, mask, x0, l1, l2, N, N * cycles)
        assert np.linalg.norm(xc - u) <= (2 * q ** N) ** cycles * e0
    x96 = oracle.cheb2(n, mesh.elems, K, M, 0.0, b, mask, x0, l1, l2, 32, 96)
    assert np.linalg.norm(x96 - u) > 5 * (2 * q ** 32) ** 3 * e0


def test_two_and_three_level_agree_after_N_steps():
    mesh, K, M, b, mask, x0, u, l1, l2 = _section3_problem(17)
    n = mesh.n_nodes
    N = 8
    x2 = oracle.cheb2(n, mesh.elems, K, M, 0.0, b, mask, x0, l1, l2, N, N)
    x3 = oracle.cheb3(n, mesh.elems, K, M, 0.0, b, mask, x0, l1, l2, N)
    np.testing.assert_allclose(x2, x3, atol=1e-12 * np.abs(x3).max())
    # The printed alpha/beta program takes a different first beta and so does
    # not reproduce x^N (kept only as a variant).
    x3l = oracle.cheb3_listing(n, mesh.elems, K, M, 0.0, b, mask, x0, l1, l2, N)
    assert np.abs(x3l - x3).max() > 1e-6


def _error_components(mesh, K, M, mask, x, u):
    """Eigenvalues of K_II and the components of the free-node error x - u along its eigenvectors."""
    free = mask == 0
    A = dense_from_oracle(mesh, K, M, 0.0)[np.ix_(free, free)]
    lam, V = np.linalg.eigh(A)
    return lam, V.T @ (x - u)[free]


@pytest.mark.parametrize("kind", ["equations", "program"])
def test_chebyshev_error_is_the_scaled_chebyshev_polynomial(kind):
    """After k steps of the three-level method the error along every eigenvector
    of K_II is P_k(lambda) times its initial component, with
    P_k = T_k((d - x)/c) / T_k(d/c) for eq. (9) and U_k((d - x)/c) / U_k(d/c)
    for the alpha/beta program (second kind), d = (l1+l2)/2, c = (l2-l1)/2; the
    polynomials come from scipy.special, independently of the recurrences."""
    from scipy import special

    mesh, K, M, b, mask, x0, u, l1, l2 = _section3_problem(17)
    n = mesh.n_nodes
    d, c = 0.5 * (l1 + l2), 0.5 * (l2 - l1)
    lam, c0 = _error_components(mesh, K, M, mask, x0, u)
    poly = special.eval_chebyt if kind == "equations" else special.eval_chebyu
    run = oracle.cheb3 if kind == "equations" else oracle.cheb3_listing
    for k in (1, 2, 3, 5, 8, 20, 40):
        xk = run(n, mesh.elems, K, M, 0.0, b, mask, x0, l1, l2, k)
        _, ck = _error_components(mesh, K, M, mask, xk, u)
        want = poly(k, (d - lam) / c) / poly(k, d / c) * c0
        assert np.abs(ck - want).max() <= 1e-10 * np.abs(c0).max(), (kind, k)
    # and the two kinds differ from the second step on
    x2 = oracle.cheb3_listing(n, mesh.elems, K, M, 0.0, b, mask, x0, l1, l2, 2)
    _, c2 = _error_components(mesh, K, M, mask, x2, u)
    first_kind = special.eval_chebyt(2, (d - lam) / c) / special.eval_chebyt(2, d / c) * c0
    assert np.abs(c2 - first_kind).max() > 1e-3 * np.abs(c0).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_residual_scale_bounds_the_residual(dim):
    """s = |b| + sum_e C_e^T |A_e| |x_e| bounds the residual componentwise,
    dominates |b| + |A||x| of the assembled matrix (element absolute values are
    never smaller than those of the sums), and is attained when no term
    cancels (mass matrix only, x >= 0, b <= 0)."""
    mesh = inputs.square_mesh(6, jitter=0.2, seed=3) if dim == 2 else inputs.cube_mesh(3, jitter=0.15, seed=3)
    n = mesh.n_nodes
    K, M, _ = oracle.local_matrices(mesh.coords, mesh.elems)
    rng = np.random.default_rng(7)
    nu = 0.7
    b = rng.standard_normal(n)
    x = rng.standard_normal(n)
    s = oracle.residual_scale(n, mesh.elems, K, M, nu, b, x)
    r = oracle.residual(n, mesh.elems, K, M, nu, b, x)
    A = dense_from_oracle(mesh, K, M, nu)
    assert np.all(s >= np.abs(r) * (1 - 1e-14))
    assert np.all(s >= (np.abs(b) + np.abs(A) @ np.abs(x)) * (1 - 1e-14))
    # strictly larger somewhere: the stiffness entries of shared edges cancel in the sum
    assert np.any(s > (np.abs(b) + np.abs(A) @ np.abs(x)) * (1 + 1e-6))
    # no cancellation: the mass part alone with x >= 0 and b <= 0 gives r = b - M x = -s
    Z = np.zeros_like(K)
    xp, bn = np.abs(x), -np.abs(b)
    s_m = oracle.residual_scale(n, mesh.elems, Z, M, nu, bn, xp)
    r_m = oracle.residual(n, mesh.elems, Z, M, nu, bn, xp)
    np.testing.assert_allclose(s_m, -r_m, rtol=1e-14)
    np.testing.assert_allclose(s_m, np.abs(bn) + nu * dense_from_oracle(mesh, Z, M, 1.0) @ xp, rtol=1e-13)
    # b = NULL counts as b = 0
    np.testing.assert_allclose(oracle.residual_scale(n, mesh.elems, K, M, nu, None, x),
                               s - np.abs(b), rtol=1e-12, atol=1e-14)


def test_richardson_is_chebyshev_with_one_root():
    mesh, K, M, b, mask, x0, u, l1, l2 = _section3_problem(17)
    n = mesh.n_nodes
    xr = oracle.richardson(n, mesh.elems, K, M, 0.0, b, mask, x0, l1, l2, 20)
    x1 = oracle.cheb2(n, mesh.elems, K, M, 0.0, b, mask, x0, l1, l2, 1, 20)
    np.testing.assert_allclose(xr, x1, rtol=0, atol=1e-15)
