"""Pins of the multigrid oracle (oracle/mg.py) against facts of nested P1
spaces and of symmetric V-cycles, none of which re-derive its formulas."""
import numpy as np
import pytest

import oracle
import oracle.mg as omg
from paper_1911_03973_amd import inputs


def _hierarchy(n, coarsest, jitter, which, nu, seed=0):
    fine = inputs.square_mesh(n, jitter=jitter, seed=seed)
    meshes = inputs.square_hierarchy(fine, coarsest=coarsest)
    nds = [inputs.boundary_nodes(m, which) for m in meshes]
    levels, Ps = omg.hierarchy(meshes, nds, nu)
    return meshes, nds, levels, Ps


@pytest.mark.parametrize("nc", [1, 2, 5, 8])
def test_prolongation_reproduces_linear_functions(nc):
    """P1 interpolation is exact for linear functions."""
    P = omg.prolongation(nc)
    mc, mf = nc + 1, 2 * nc + 1
    J, I = np.divmod(np.arange(mc * mc), mc)
    j, i = np.divmod(np.arange(mf * mf), mf)
    for a, b, c in [(1.0, 0.0, 0.0), (0.3, -1.25, 2.5), (-2.0, 0.75, 0.125)]:
        got = P @ (a + b * I + c * J)
        want = a + b * i / 2.0 + c * j / 2.0
        assert np.abs(got - want).max() <= 1e-14


def test_prolongation_is_the_identity_on_coarse_nodes_and_a_partition_of_unity():
    nc = 4
    P = omg.prolongation(nc).toarray()
    mc, mf = nc + 1, 2 * nc + 1
    assert np.allclose(P.sum(axis=1), 1.0, rtol=0, atol=1e-15)
    for J in range(mc):
        for I in range(mc):
            row = P[(2 * J) * mf + 2 * I]
            assert row[J * mc + I] == 1.0 and np.count_nonzero(row) == 1


def _galerkin_gap(P, fine, coarse, nu):
    Kf, Mf, _ = oracle.local_matrices(fine.coords, fine.elems)
    Kc, Mc, _ = oracle.local_matrices(coarse.coords, coarse.elems)
    Af = omg.assemble_dense(fine.n_nodes, fine.elems, Kf, Mf, nu)
    Ac = omg.assemble_dense(coarse.n_nodes, coarse.elems, Kc, Mc, nu)
    P = P.toarray() if hasattr(P, "toarray") else P
    return np.abs(P.T @ Af @ P - Ac).max() / np.abs(Ac).max()


@pytest.mark.parametrize("n,nu", [(2, 0.0), (8, 0.0), (8, 0.7), (16, 3.0)])
def test_galerkin_identity_of_nested_p1_spaces(n, nu):
    """The coarse P1 space is a subspace of the fine one, so the coarse
    stiffness and mass matrices are P^T A_h P exactly (up to rounding)."""
    fine = inputs.square_mesh(n)
    coarse = inputs.square_hierarchy(fine, coarsest=n // 2)[1]
    assert _galerkin_gap(omg.prolongation(n // 2), fine, coarse, nu) <= 1e-13


def test_galerkin_identity_detects_interpolation_along_the_wrong_diagonal():
    """Planted mistake: odd-odd fine nodes averaged over the other diagonal of
    the coarse square.  Still a partition of unity and exact for linears, but
    no longer the P1 space of the coarse mesh, so the identity fails -- in the
    mass part: the right-angled triangles give the diagonal edges no
    stiffness coupling, so with nu = 0 both diagonals yield the same
    matrices, and only nu > 0 tells them apart."""
    n = 8
    fine = inputs.square_mesh(n)
    coarse = inputs.square_hierarchy(fine, coarsest=n // 2)[1]
    nc = n // 2
    mc, mf = nc + 1, 2 * nc + 1
    P = omg.prolongation(nc).toarray()
    for J in range(nc):
        for I in range(nc):
            row = (2 * J + 1) * mf + 2 * I + 1
            P[row] = 0.0
            P[row, J * mc + I + 1] = 0.5
            P[row, (J + 1) * mc + I] = 0.5
    assert _galerkin_gap(P, fine, coarse, 0.0) <= 1e-13
    assert _galerkin_gap(P, fine, coarse, 1.0) > 1e-4


@pytest.mark.parametrize("smooth", [1, 2, 3])
def test_vcycle_is_symmetric_positive_definite(smooth):
    """Equal pre- and post-smoothing with a symmetric smoother, restriction =
    P^T and an exact coarsest solve make B symmetric and positive definite."""
    _, _, levels, Ps = _hierarchy(32, 8, 0.2, "x2=0", 0.5, seed=3)
    n = levels[0].n_nodes
    rng = np.random.default_rng(7)
    r1, r2 = rng.standard_normal(n), rng.standard_normal(n)
    r1[levels[0].mask == 1] = 0.0
    r2[levels[0].mask == 1] = 0.0
    z1 = omg.vcycle(levels, Ps, r1, smooth, 2.0 / 3.0)
    z2 = omg.vcycle(levels, Ps, r2, smooth, 2.0 / 3.0)
    scale = np.linalg.norm(r1) * np.linalg.norm(z2)
    assert abs(r1 @ z2 - r2 @ z1) <= 1e-13 * scale
    assert r1 @ z1 > 0 and r2 @ z2 > 0
    assert np.all(z1[levels[0].mask == 1] == 0.0)


def test_one_level_cycle_solves_the_free_node_system():
    _, nds, levels, Ps = _hierarchy(16, 16, 0.2, "x2=0", 1.5, seed=4)
    L = levels[0]
    rng = np.random.default_rng(2)
    r = rng.standard_normal(L.n_nodes)
    z = omg.vcycle(levels, Ps, r, 2, 2.0 / 3.0)
    rr = np.where(L.free, r, 0.0)
    assert np.linalg.norm(L.residual(rr, z)) <= 1e-12 * np.linalg.norm(rr)
    assert np.all(z[nds[0]] == 0.0)


@pytest.mark.parametrize("smooth,bound", [(1, 0.55), (2, 0.4)])
def test_vcycle_contraction_is_mesh_independent(smooth, bound):
    """The A-norm contraction of e <- (I - B A) e, estimated by power
    iteration, stays bounded well below one as h halves (the defining
    property of multigrid; a wrong transfer weight or a missing smoothing
    step makes it grow with n)."""
    rates = []
    for n in (16, 32, 64):
        _, _, levels, Ps = _hierarchy(n, 4, 0.0, "all", 0.0)
        L = levels[0]
        zero = np.zeros(L.n_nodes)

        def apply_a(v):
            return -L.residual(zero, v)

        e = np.random.default_rng(n).standard_normal(L.n_nodes) * L.free
        e /= np.sqrt(e @ apply_a(e))
        rate = 0.0
        for _ in range(20):
            e = e - omg.vcycle(levels, Ps, apply_a(e), smooth, 2.0 / 3.0)
            rate = np.sqrt(e @ apply_a(e))
            e /= rate
        rates.append(rate)
    assert max(rates) < bound, rates
    assert rates[-1] - rates[-2] < 0.03, rates


# ---- Kuhn cube meshes (3D) ----

def test_prolongation3_reproduces_linear_functions_and_partitions_unity():
    for nc in (1, 2, 3):
        P = omg.prolongation3(nc)
        mc, mf = nc + 1, 2 * nc + 1
        K, rem = np.divmod(np.arange(mc ** 3), mc * mc)
        J, I = np.divmod(rem, mc)
        k, rem = np.divmod(np.arange(mf ** 3), mf * mf)
        j, i = np.divmod(rem, mf)
        for a, b, c, d in [(1.0, 0.0, 0.0, 0.0), (0.3, -1.25, 2.5, 0.75)]:
            got = P @ (a + b * I + c * J + d * K)
            want = a + b * i / 2.0 + c * j / 2.0 + d * k / 2.0
            assert np.abs(got - want).max() <= 1e-14
        assert np.allclose(P.sum(axis=1), 1.0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("n,nu", [(2, 0.0), (4, 0.0), (4, 1.3)])
def test_galerkin_identity_of_nested_kuhn_meshes(n, nu):
    """Uniform refinement of the Kuhn split of the cube lattice is again a
    Kuhn split with the same diagonal, so the coarse P1 space is a subspace of
    the fine one and P^T A_h P = A_2h."""
    fine = inputs.cube_mesh(n)
    coarse = inputs.cube_hierarchy(fine, coarsest=n // 2)[1]
    assert _galerkin_gap(omg.prolongation3(n // 2), fine, coarse, nu) <= 1e-13


def test_galerkin_identity_3d_detects_the_wrong_cube_diagonal():
    """Planted mistake: cube centres averaged over the (1,0,0)-(0,1,1)
    diagonal, which is not an edge of the Kuhn split."""
    n = 4
    fine = inputs.cube_mesh(n)
    coarse = inputs.cube_hierarchy(fine, coarsest=n // 2)[1]
    nc = n // 2
    mc, mf = nc + 1, 2 * nc + 1
    P = omg.prolongation3(nc).toarray()
    for K in range(nc):
        for J in range(nc):
            for I in range(nc):
                row = ((2 * K + 1) * mf + 2 * J + 1) * mf + 2 * I + 1
                P[row] = 0.0
                P[row, (K * mc + J) * mc + I + 1] = 0.5
                P[row, ((K + 1) * mc + J + 1) * mc + I] = 0.5
    assert _galerkin_gap(P, fine, coarse, 0.0) > 1e-4


def test_vcycle_3d_is_symmetric_and_contracts():
    fine = inputs.cube_mesh(8, jitter=0.1, seed=2)
    meshes = inputs.cube_hierarchy(fine, coarsest=2)
    nds = [inputs.boundary_nodes(m, "all") for m in meshes]
    levels, Ps = omg.hierarchy(meshes, nds, 0.5)
    L = levels[0]
    rng = np.random.default_rng(3)
    r1, r2 = rng.standard_normal(L.n_nodes) * L.free, rng.standard_normal(L.n_nodes) * L.free
    z1 = omg.vcycle(levels, Ps, r1, 2, 2.0 / 3.0)
    z2 = omg.vcycle(levels, Ps, r2, 2, 2.0 / 3.0)
    assert abs(r1 @ z2 - r2 @ z1) <= 1e-13 * np.linalg.norm(r1) * np.linalg.norm(z2)
    zero = np.zeros(L.n_nodes)
    e = rng.standard_normal(L.n_nodes) * L.free
    for _ in range(15):
        ae = -L.residual(zero, e)
        e_new = e - omg.vcycle(levels, Ps, ae, 2, 2.0 / 3.0)
        rate = np.sqrt(e_new @ -L.residual(zero, e_new)) / np.sqrt(e @ ae)
        e = e_new
    assert rate < 0.5, rate


# ---- Chebyshev smoothing (the paper's three-level iteration on D^-1 A) ----


def _pencil(L):
    """Eigenpairs of the free-node pencil (A, D): A v = lambda D v, V^T D V = I."""
    import scipy.linalg

    A, f = L.dense_free()
    lam, V = scipy.linalg.eigh(A, np.diag(np.diag(A)))
    return A, f, lam, V


def test_gershgorin_bound_is_two_on_the_uniform_square_mesh():
    """Right isosceles triangles couple their two acute vertices by 0 and all
    other pairs negatively, so at every free node the element absolute row
    sums add up to 2 x the diagonal (the 5-point stencil 4, -1, -1, -1, -1)."""
    m = inputs.square_mesh(8)
    L = omg.Level(m, inputs.boundary_nodes(m), 0.0)
    assert abs(L.gersh - 2.0) <= 1e-14


@pytest.mark.parametrize("dim,nu", [(2, 0.0), (2, 3.0), (3, 0.0), (3, 1.0)])
def test_gershgorin_bound_covers_the_spectrum(dim, nu):
    """lambda_max(D^-1 A) <= g (Gershgorin's theorem), and g is tight enough to
    place the smoother's interval (within 25 %).  Row sums without absolute
    values (a plausible slip) give a 'bound' far below lambda_max."""
    mesh = inputs.square_mesh(10, jitter=0.2, seed=6) if dim == 2 else inputs.cube_mesh(5, jitter=0.1, seed=6)
    L = omg.Level(mesh, inputs.boundary_nodes(mesh), nu)
    _, _, lam, _ = _pencil(L)
    assert lam.max() <= L.gersh * (1.0 + 1e-12)
    assert L.gersh <= 1.25 * lam.max(), (L.gersh, lam.max())
    Ae = L.K + nu * L.M
    signed = np.zeros(L.n_nodes)
    np.add.at(signed, L.elems.astype(np.int64).ravel(), Ae.sum(axis=2).ravel())
    assert (L.dinv * signed)[L.free].max() < 0.9 * lam.max()


@pytest.mark.parametrize("steps", [1, 2, 3, 5])
@pytest.mark.parametrize("start", ["zero", "random"])
def test_chebyshev_smoother_applies_the_scaled_chebyshev_polynomial(steps, start):
    """For A u = r, m steps from z^0 leave the error u - z^m = P_m(D^-1 A)(u - z^0)
    with P_m(x) = T_m((theta - x) / delta) / T_m(theta / delta), theta and delta
    the centre and half-width of [lower g, g]; checked along the pencil's
    eigenvectors with numpy's Chebyshev basis (the recurrence is not used)."""
    mesh = inputs.square_mesh(8, jitter=0.2, seed=3)
    L = omg.Level(mesh, inputs.boundary_nodes(mesh, "x2=0"), 0.5)
    A, f, lam, V = _pencil(L)
    lower = 0.3
    lam1, lam2 = lower * L.gersh, L.gersh
    theta, delta = 0.5 * (lam1 + lam2), 0.5 * (lam2 - lam1)
    T = np.polynomial.chebyshev.Chebyshev.basis(steps)
    P = T((theta - lam) / delta) / T(theta / delta)
    rng = np.random.default_rng(steps)
    u = np.zeros(L.n_nodes)
    u[f] = rng.standard_normal(f.size)
    r = np.zeros(L.n_nodes)
    r[f] = A @ u[f]
    z0 = None
    e0 = u[f].copy()
    if start == "random":
        z0 = np.zeros(L.n_nodes)
        z0[f] = rng.standard_normal(f.size)
        e0 = u[f] - z0[f]
    z = omg.chebyshev_smooth(L, r, z0, steps, lower)
    c = V.T @ (np.diag(A) * e0)  # coefficients in the D-orthonormal eigenbasis
    want = V @ (P * c)
    assert np.abs((u[f] - z[f]) - want).max() <= 1e-11 * np.abs(e0).max()
    assert np.all(z[L.mask == 1] == 0.0)


def test_chebyshev_vcycle_is_symmetric_and_contracts():
    """The same polynomial before and after the correction keeps B symmetric
    and positive definite; its contraction stays mesh-independent and below
    that of two damped-Jacobi steps on the same meshes."""
    rates = {}
    for n in (16, 32, 64):
        _, _, levels, Ps = _hierarchy(n, 4, 0.2, "x2=0", 0.5, seed=n)
        L = levels[0]
        rng = np.random.default_rng(n)
        r1, r2 = rng.standard_normal(L.n_nodes) * L.free, rng.standard_normal(L.n_nodes) * L.free
        z1 = omg.vcycle(levels, Ps, r1, 2, 0.0, smoother="chebyshev")
        z2 = omg.vcycle(levels, Ps, r2, 2, 0.0, smoother="chebyshev")
        assert abs(r1 @ z2 - r2 @ z1) <= 1e-13 * np.linalg.norm(r1) * np.linalg.norm(z2)
        assert r1 @ z1 > 0 and r2 @ z2 > 0
        zero = np.zeros(L.n_nodes)
        for sm in ("chebyshev", "jacobi"):
            e = rng.standard_normal(L.n_nodes) * L.free
            for _ in range(15):
                ae = -L.residual(zero, e)
                e_new = e - omg.vcycle(levels, Ps, ae, 2, 2.0 / 3.0, smoother=sm)
                rate = np.sqrt(e_new @ -L.residual(zero, e_new)) / np.sqrt(e @ ae)
                e = e_new
            rates[(n, sm)] = rate
    assert max(rates[(n, "chebyshev")] for n in (16, 32, 64)) < 0.3, rates
    for n in (16, 32, 64):
        assert rates[(n, "chebyshev")] < rates[(n, "jacobi")], rates
