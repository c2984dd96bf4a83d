"""Geometric multigrid on nested square meshes: the transfer operators against
the Galerkin identity of nested P1 spaces, and MG-preconditioned FCG judged by
the oracle's residual."""
import numpy as np
import pytest
import torch

import oracle
import oracle.mg as omg
from paper_1911_03973_amd import inputs

from problems import Problem, cuda

pytestmark = pytest.mark.gpu

fem = pytest.importorskip("paper_1911_03973_amd.fem")


def _hierarchy(n, jitter, which, nu, coarsest=16, seed=0):
    fine = inputs.square_mesh(n, jitter=jitter, seed=seed)
    meshes = inputs.square_hierarchy(fine, coarsest=coarsest)
    nds = [inputs.boundary_nodes(m, which) for m in meshes]
    return meshes, nds, fem.MG.from_meshes(meshes, nds, nu)


@pytest.mark.parametrize("n,which,nu", [(32, "all", 0.0), (64, "all", 0.5), (64, "x2=0", 2.0)])
def test_galerkin_identity_on_nested_meshes(n, which, nu):
    """Without jitter the coarse P1 space is a subspace of the fine one, so
    P^T A_h P z = A_2h z on every free coarse node, for the stiffness and the
    mass part alike: pins the prolongation weights and that the restriction is
    their transpose."""
    meshes, nds, mg = _hierarchy(n, 0.0, which, nu)
    rng = np.random.default_rng(5)
    for level in range(len(meshes) - 1):
        mc = meshes[level + 1]
        zc = rng.standard_normal(mc.n_nodes)
        zc[nds[level + 1]] = 0.0
        got = mg.galerkin_apply(level, cuda(zc)).cpu().numpy()
        Kc, Mc, _ = oracle.local_matrices(mc.coords, mc.elems)
        mask = oracle.mask_from_nodes(mc.n_nodes, nds[level + 1])
        want = -oracle.residual(mc.n_nodes, mc.elems, Kc, Mc, nu, np.zeros(mc.n_nodes), zc, mask)
        scale = np.abs(want).max()
        assert np.abs(got - want).max() <= 1e-12 * scale, (level, np.abs(got - want).max() / scale)


@pytest.mark.parametrize("jitter", [0.0, 0.2])
def test_mg_fcg_converges_independently_of_the_mesh_size(jitter):
    iters = []
    for n in (64, 128, 256):
        meshes, nds, mg = _hierarchy(n, jitter, "x2=0", 1.0, seed=n)
        prob = Problem(meshes[0], nu=1.0, dirichlet="x2=0", f="sine", seed=n + 1)
        x = torch.zeros(prob.n, dtype=torch.float64, device="cuda")
        info = mg.solve(fem.mg_opts(rtol=1e-8), cuda(prob.b), x)
        print(n, info, flush=True)
        assert info["status"] == fem.FEM_OK
        xs = x.cpu().numpy()
        r = oracle.residual(prob.n, prob.mesh.elems, prob.K, prob.M, prob.nu, prob.b, xs, prob.mask)
        r0 = oracle.residual(prob.n, prob.mesh.elems, prob.K, prob.M, prob.nu, prob.b, np.zeros(prob.n), prob.mask)
        assert np.linalg.norm(r) / np.linalg.norm(r0) <= 1e-8
        iters.append(info["iters"])
    # Jacobi-PCG needs ~2x the iterations per halving of h; the V-cycle keeps them flat
    assert max(iters) <= 30 and max(iters) <= 1.5 * min(iters) + 2, iters


def test_mg_solution_matches_single_level_solver():
    meshes, nds, mg = _hierarchy(64, 0.2, "all", 0.3, seed=3)
    prob = Problem(meshes[0], nu=0.3, dirichlet="all", f="sine", seed=9)
    x0 = np.zeros(prob.n)
    x = cuda(x0)
    mg.solve(fem.mg_opts(rtol=1e-10), cuda(prob.b), x)
    xo, _ = oracle.pcg(prob.n, prob.mesh.elems, prob.K, prob.M, prob.nu, prob.b, prob.mask, x0, rtol=1e-12)
    assert np.abs(x.cpu().numpy() - xo).max() <= 1e-8 * np.abs(xo).max()


def test_mg_rejects_a_hierarchy_that_is_not_nested():
    meshes = [inputs.square_mesh(32), inputs.square_mesh(8)]
    nds = [inputs.boundary_nodes(m) for m in meshes]
    with pytest.raises(fem.FemError):
        fem.MG.from_meshes(meshes, nds, 0.0)
    with pytest.raises(fem.FemError):  # coarsest grid too large for the dense solve
        big = inputs.square_hierarchy(inputs.square_mesh(128), coarsest=64)
        fem.MG.from_meshes(big, [inputs.boundary_nodes(m) for m in big], 0.0)


@pytest.mark.parametrize("n,coarsest,jitter,which,nu,smooth", [
    (16, 8, 0.0, "all", 0.0, 1),       # two levels
    (32, 8, 0.0, "all", 0.0, 2),
    (64, 16, 0.2, "x2=0", 0.5, 1),
    (64, 8, 0.1, "all", 3.0, 3),       # four levels
    (200, 25, 0.2, "x2=0", 1.0, 2),    # odd coarsest grid, many chunks and a ragged tail
])
def test_vcycle_matches_oracle(n, coarsest, jitter, which, nu, smooth):
    """One V-cycle z = B r element by element against the oracle's cycle
    (its own local matrices, sparse P from barycentric evaluation, dense LU on
    the coarsest level).  r is nonzero on Dirichlet nodes too: both sides must
    ignore it there.  Tolerance: every step is a linear map of norm O(1) in
    FP64 except the coarsest solve, whose relative error is bounded by its
    condition number (< 10^3 for at most 33^2 nodes) times 1e-16."""
    seed = n + smooth
    print(f"vcycle n={n} coarsest={coarsest} jitter={jitter} {which} nu={nu} smooth={smooth}", flush=True)
    meshes, nds, mg = _hierarchy(n, jitter, which, nu, coarsest=coarsest, seed=seed)
    levels, Ps = omg.hierarchy(meshes, nds, nu)
    r = np.random.default_rng(seed).standard_normal(meshes[0].n_nodes)
    for omega in (2.0 / 3.0, 0.9):
        got = mg.vcycle(cuda(r), smooth, omega).cpu().numpy()
        want = omg.vcycle(levels, Ps, r, smooth, omega)
        scale = np.abs(want).max()
        assert np.abs(got - want).max() <= 1e-12 * scale, (omega, np.abs(got - want).max() / scale)
        assert np.all(got[nds[0]] == 0.0)


def test_vcycle_rejects_bad_arguments():
    meshes, nds, mg = _hierarchy(32, 0.0, "all", 0.0)
    r = cuda(np.ones(meshes[0].n_nodes))
    for smooth, omega in [(0, 0.5), (65, 0.5), (2, 0.0), (2, 2.0)]:
        with pytest.raises(fem.FemError):
            mg.vcycle(r, smooth, omega)
    with pytest.raises(fem.FemError):
        mg.vcycle(r, 2, 0.5, z=r)


@pytest.mark.parametrize("n,coarsest,smooth", [(64, 16, 1), (128, 16, 2)])
def test_vcycle_with_fp32_heads_stays_close_to_oracle(n, coarsest, smooth):
    """The cycle reading the FP32 heads of the packed operator: every product
    carries entrywise relative errors of at most 2^-24 (one rounding of each
    packed value), and the cycle is a contraction-like linear map, so over its
    2 smooth + 2 products per level the result stays within about
    (levels * (2 smooth + 2)) * 2^-24 of the FP64 cycle; asserted with a 10x
    margin as 1e-5 of max|z|."""
    meshes, nds, mg = _hierarchy(n, 0.2, "x2=0", 1.0, coarsest=coarsest, seed=n)
    levels, Ps = omg.hierarchy(meshes, nds, 1.0)
    r = np.random.default_rng(n).standard_normal(meshes[0].n_nodes)
    want = omg.vcycle(levels, Ps, r, smooth, 2.0 / 3.0)
    got = mg.vcycle(cuda(r), smooth, 2.0 / 3.0, cycle_dtype=fem.F32).cpu().numpy()
    err = np.abs(got - want).max() / np.abs(want).max()
    print("fp32-head cycle rel err", err, flush=True)
    assert err <= 1e-5
    assert err > 0.0  # it really read the FP32 heads


def test_mg_fcg_with_fp32_cycle_meets_target():
    meshes, nds, mg = _hierarchy(256, 0.2, "x2=0", 1.0, seed=7)
    prob = Problem(meshes[0], nu=1.0, dirichlet="x2=0", f="sine", seed=8)
    its = {}
    for cd in (fem.F64, fem.F32):
        x = torch.zeros(prob.n, dtype=torch.float64, device="cuda")
        info = mg.solve(fem.mg_opts(rtol=1e-8, cycle_dtype=cd), cuda(prob.b), x)
        assert info["status"] == fem.FEM_OK
        r = oracle.residual(prob.n, prob.mesh.elems, prob.K, prob.M, prob.nu, prob.b, x.cpu().numpy(), prob.mask)
        r0 = oracle.residual(prob.n, prob.mesh.elems, prob.K, prob.M, prob.nu, prob.b, np.zeros(prob.n), prob.mask)
        assert np.linalg.norm(r) / np.linalg.norm(r0) <= 1e-8
        its[cd] = info["iters"]
    assert its[fem.F32] <= its[fem.F64] + 2, its


# ---- Kuhn cube meshes (3D) ----

def _hierarchy3(n, jitter, which, nu, coarsest, seed=0):
    fine = inputs.cube_mesh(n, jitter=jitter, seed=seed)
    meshes = inputs.cube_hierarchy(fine, coarsest=coarsest)
    nds = [inputs.boundary_nodes(m, which) for m in meshes]
    return meshes, nds, fem.MG.from_meshes(meshes, nds, nu)


@pytest.mark.parametrize("n,nu", [(8, 0.0), (16, 0.7)])
def test_galerkin_identity_on_nested_kuhn_meshes(n, nu):
    meshes, nds, mg = _hierarchy3(n, 0.0, "all", nu, coarsest=2)
    rng = np.random.default_rng(6)
    for level in range(len(meshes) - 1):
        mc = meshes[level + 1]
        zc = rng.standard_normal(mc.n_nodes)
        zc[nds[level + 1]] = 0.0
        got = mg.galerkin_apply(level, cuda(zc)).cpu().numpy()
        Kc, Mc, _ = oracle.local_matrices(mc.coords, mc.elems)
        mask = oracle.mask_from_nodes(mc.n_nodes, nds[level + 1])
        want = -oracle.residual(mc.n_nodes, mc.elems, Kc, Mc, nu, np.zeros(mc.n_nodes), zc, mask)
        scale = np.abs(want).max()
        assert np.abs(got - want).max() <= 1e-12 * scale, (level, np.abs(got - want).max() / scale)


@pytest.mark.parametrize("n,coarsest,jitter,nu,smooth", [(8, 2, 0.0, 0.0, 1), (16, 4, 0.1, 1.0, 2),
                                                          (20, 5, 0.1, 10.0, 1)])
def test_vcycle_3d_matches_oracle(n, coarsest, jitter, nu, smooth):
    print(f"vcycle3 n={n} coarsest={coarsest} jitter={jitter} nu={nu} smooth={smooth}", flush=True)
    meshes, nds, mg = _hierarchy3(n, jitter, "all", nu, coarsest, seed=n)
    levels, Ps = omg.hierarchy(meshes, nds, nu)
    r = np.random.default_rng(n + 1).standard_normal(meshes[0].n_nodes)
    got = mg.vcycle(cuda(r), smooth, 2.0 / 3.0).cpu().numpy()
    want = omg.vcycle(levels, Ps, r, smooth, 2.0 / 3.0)
    scale = np.abs(want).max()
    assert np.abs(got - want).max() <= 1e-12 * scale, np.abs(got - want).max() / scale
    assert np.all(got[nds[0]] == 0.0)


def test_mg_fcg_3d_converges_independently_of_the_mesh_size():
    iters = []
    for n in (16, 32, 64):
        meshes, nds, mg = _hierarchy3(n, 0.1, "all", 10.0, coarsest=4, seed=n)
        prob = Problem(meshes[0], nu=10.0, dirichlet="all", f="sine", seed=n + 1)
        x = torch.zeros(prob.n, dtype=torch.float64, device="cuda")
        info = mg.solve(fem.mg_opts(rtol=1e-8), cuda(prob.b), x)
        print(n, info, flush=True)
        assert info["status"] == fem.FEM_OK
        r = oracle.residual(prob.n, prob.mesh.elems, prob.K, prob.M, prob.nu, prob.b, x.cpu().numpy(), prob.mask)
        r0 = oracle.residual(prob.n, prob.mesh.elems, prob.K, prob.M, prob.nu, prob.b, np.zeros(prob.n), prob.mask)
        assert np.linalg.norm(r) / np.linalg.norm(r0) <= 1e-8
        iters.append(info["iters"])
    assert max(iters) <= 30 and max(iters) <= 1.5 * min(iters) + 2, iters


def test_mg_rejects_mixed_dimensions():
    m2 = inputs.square_mesh(8)
    m3 = inputs.cube_mesh(4)
    with pytest.raises(fem.FemError):
        fem.MG.from_meshes([m2, m3], [inputs.boundary_nodes(m2), inputs.boundary_nodes(m3)], 0.0)


# ---- Chebyshev smoothing ----

def test_level_bounds_match_oracle():
    """g of every level (one |A_e| element pass at setup) against the oracle's
    element absolute row sums; on the uniform square mesh at nu = 0 it is
    exactly the 5-point stencil's 2."""
    meshes, nds, mg = _hierarchy(64, 0.2, "x2=0", 0.5, coarsest=8, seed=2)
    levels, _ = omg.hierarchy(meshes, nds, 0.5)
    for l, L in enumerate(levels):
        assert abs(mg.level_bound(l) - L.gersh) <= 1e-12 * L.gersh, (l, mg.level_bound(l), L.gersh)
    meshes3, nds3, mg3 = _hierarchy3(16, 0.1, "all", 1.0, coarsest=4, seed=3)
    levels3, _ = omg.hierarchy(meshes3, nds3, 1.0)
    for l, L in enumerate(levels3):
        assert abs(mg3.level_bound(l) - L.gersh) <= 1e-12 * L.gersh, (l, mg3.level_bound(l), L.gersh)
    _, _, mgu = _hierarchy(32, 0.0, "all", 0.0, coarsest=8)
    assert all(abs(mgu.level_bound(l) - 2.0) <= 1e-13 for l in range(3))
    with pytest.raises(fem.FemError):
        mgu.level_bound(3)


@pytest.mark.parametrize("dim,n,coarsest,jitter,which,nu,smooth,lower", [
    (2, 16, 8, 0.0, "all", 0.0, 1, 0.3),      # two levels; one step = Jacobi with 1/theta
    (2, 32, 8, 0.0, "all", 0.0, 2, 0.3),
    (2, 64, 16, 0.2, "x2=0", 0.5, 3, 0.2),
    (2, 64, 8, 0.1, "all", 3.0, 2, 0.3),      # four levels
    (2, 200, 25, 0.2, "x2=0", 1.0, 2, 0.3),   # odd coarsest grid, ragged tail
    (3, 8, 2, 0.0, "all", 0.0, 2, 0.3),
    (3, 16, 4, 0.1, "all", 1.0, 3, 0.25),
])
def test_chebyshev_vcycle_matches_oracle(dim, n, coarsest, jitter, which, nu, smooth, lower):
    """One V-cycle with Chebyshev smoothing against the oracle's (its own g,
    recurrence in the paper's three-term form, sparse P, dense coarsest
    solve); tolerance as for the Jacobi cycle: the steps are linear maps of
    norm O(1) and the two g agree to rounding."""
    print(f"cheb vcycle dim={dim} n={n} coarsest={coarsest} nu={nu} smooth={smooth} lower={lower}", flush=True)
    if dim == 2:
        meshes, nds, mg = _hierarchy(n, jitter, which, nu, coarsest=coarsest, seed=n)
    else:
        meshes, nds, mg = _hierarchy3(n, jitter, which, nu, coarsest, seed=n)
    levels, Ps = omg.hierarchy(meshes, nds, nu)
    r = np.random.default_rng(n + 3).standard_normal(meshes[0].n_nodes)
    got = mg.vcycle(cuda(r), smooth, 0.0, smoother=fem.SMOOTH_CHEBYSHEV, cheb_lower=lower).cpu().numpy()
    want = omg.vcycle(levels, Ps, r, smooth, 0.0, smoother="chebyshev", lower=lower)
    scale = np.abs(want).max()
    assert np.abs(got - want).max() <= 1e-12 * scale, np.abs(got - want).max() / scale
    assert np.all(got[nds[0]] == 0.0)
    # a second call reuses the level increments: same result bit for bit
    again = mg.vcycle(cuda(r), smooth, 0.0, smoother=fem.SMOOTH_CHEBYSHEV, cheb_lower=lower).cpu().numpy()
    assert np.array_equal(again, got)


def test_chebyshev_vcycle_with_fp32_heads_stays_close_to_oracle():
    meshes, nds, mg = _hierarchy(128, 0.2, "x2=0", 1.0, coarsest=16, seed=5)
    levels, Ps = omg.hierarchy(meshes, nds, 1.0)
    r = np.random.default_rng(5).standard_normal(meshes[0].n_nodes)
    want = omg.vcycle(levels, Ps, r, 2, 0.0, smoother="chebyshev")
    got = mg.vcycle(cuda(r), 2, 0.0, cycle_dtype=fem.F32, smoother=fem.SMOOTH_CHEBYSHEV).cpu().numpy()
    err = np.abs(got - want).max() / np.abs(want).max()
    print("fp32-head chebyshev cycle rel err", err, flush=True)
    assert 0.0 < err <= 1e-5


@pytest.mark.parametrize("dim", [2, 3])
def test_mg_fcg_with_chebyshev_smoothing(dim):
    """MG-FCG with Chebyshev smoothing meets the target by the oracle's
    residual, in no more iterations than with as many damped-Jacobi steps."""
    if dim == 2:
        meshes, nds, mg = _hierarchy(256, 0.2, "x2=0", 1.0, seed=11)
        prob = Problem(meshes[0], nu=1.0, dirichlet="x2=0", f="sine", seed=12)
    else:
        meshes, nds, mg = _hierarchy3(32, 0.1, "all", 10.0, coarsest=4, seed=11)
        prob = Problem(meshes[0], nu=10.0, dirichlet="all", f="sine", seed=12)
    its = {}
    for sm in (fem.SMOOTH_JACOBI, fem.SMOOTH_CHEBYSHEV):
        x = torch.zeros(prob.n, dtype=torch.float64, device="cuda")
        info = mg.solve(fem.mg_opts(rtol=1e-8, smooth=2, smoother=sm), cuda(prob.b), x)
        assert info["status"] == fem.FEM_OK
        r = oracle.residual(prob.n, prob.mesh.elems, prob.K, prob.M, prob.nu, prob.b, x.cpu().numpy(), prob.mask)
        r0 = oracle.residual(prob.n, prob.mesh.elems, prob.K, prob.M, prob.nu, prob.b, np.zeros(prob.n), prob.mask)
        assert np.linalg.norm(r) / np.linalg.norm(r0) <= 1e-8
        its[sm] = info["iters"]
    print(dim, its, flush=True)
    assert its[fem.SMOOTH_CHEBYSHEV] <= its[fem.SMOOTH_JACOBI], its


def test_chebyshev_options_are_checked():
    meshes, nds, mg = _hierarchy(32, 0.0, "all", 0.0)
    r = cuda(np.ones(meshes[0].n_nodes))
    for smoother, lower in [(2, 0.3), (-1, 0.3), (fem.SMOOTH_CHEBYSHEV, 0.0), (fem.SMOOTH_CHEBYSHEV, 1.0),
                            (fem.SMOOTH_CHEBYSHEV, float("nan"))]:
        with pytest.raises(fem.FemError):
            mg.vcycle(r, 2, 0.5, smoother=smoother, cheb_lower=lower)
    x = torch.zeros(meshes[0].n_nodes, dtype=torch.float64, device="cuda")
    with pytest.raises(fem.FemError):
        mg.solve(fem.mg_opts(smoother=fem.SMOOTH_CHEBYSHEV, cheb_lower=1.5), r, x)
    # omega is not used by the Chebyshev smoother
    mg.vcycle(r, 2, 0.0, smoother=fem.SMOOTH_CHEBYSHEV)
