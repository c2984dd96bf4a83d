"""The paper's iterations on the GPU residual against the FP64 oracle.

The experiment of Section 3: 33^2 nodes, nu = 0, f = 1, u = 1 on the
boundary, eigenvalue bounds from the closed-form spectrum, 124 iterations.
The iterates are sums of the same FP64 terms in a different order (the
element pass sums each node's contributions in chunk order, the oracle in
element order), so stable iterations agree to a few units of rounding per
step; the unstable 2-level ordering with N = 32 amplifies those differences
and is compared through its error instead.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1911_03973_amd import inputs

from problems import Problem, cuda

pytestmark = pytest.mark.gpu

fem = pytest.importorskip("paper_1911_03973_amd.fem")


def _section3(n_side=33, dtype=None):
    N = n_side - 1
    prob = Problem(inputs.square_mesh(N), nu=0.0)
    x0 = np.zeros(prob.n)
    x0[prob.nd] = 1.0
    u, _ = oracle.pcg(prob.n, prob.mesh.elems, prob.K, prob.M, 0.0, prob.b, prob.mask, x0, rtol=1e-12,
                      max_iter=5000)
    lam1 = 8 * math.sin(math.pi / (2 * N)) ** 2
    lam2 = 8 * math.sin((N - 1) * math.pi / (2 * N)) ** 2
    return prob, x0, u, lam1, lam2


def _gpu_run(prob, dtype, method, x0, lam1, lam2, iters, cycle=1, nu=0.0):
    plan = fem.Plan.from_mesh(prob.mesh, prob.nd)
    K = plan.empty_matrix(dtype)
    M = plan.empty_matrix(dtype)
    fem.build_local_matrices(plan, dtype, K, M, None)
    x = cuda(x0)
    info = fem.iterate(plan, fem.iter_opts(method=method, dtype=dtype, nu=nu, lam1=lam1, lam2=lam2, cycle=cycle,
                                           iters=iters), K, M, cuda(prob.b), x)
    return x.cpu().numpy(), info


ORACLE = {
    fem.RICHARDSON: lambda p, x0, l1, l2, it, N: oracle.richardson(p.n, p.mesh.elems, p.K, p.M, p.nu, p.b, p.mask,
                                                                     x0, l1, l2, it),
    fem.CHEBYSHEV2: lambda p, x0, l1, l2, it, N: oracle.cheb2(p.n, p.mesh.elems, p.K, p.M, p.nu, p.b, p.mask, x0,
                                                                l1, l2, N, it),
    fem.CHEBYSHEV3: lambda p, x0, l1, l2, it, N: oracle.cheb3(p.n, p.mesh.elems, p.K, p.M, p.nu, p.b, p.mask, x0,
                                                                l1, l2, it),
    fem.CHEBYSHEV3_LISTING: lambda p, x0, l1, l2, it, N: oracle.cheb3_listing(p.n, p.mesh.elems, p.K, p.M, p.nu,
                                                                                p.b, p.mask, x0, l1, l2, it),
}


@pytest.mark.parametrize("method,N", [(fem.RICHARDSON, 1), (fem.CHEBYSHEV2, 8), (fem.CHEBYSHEV2, 16),
                                      (fem.CHEBYSHEV3, 1), (fem.CHEBYSHEV3_LISTING, 1)])
@pytest.mark.parametrize("dtype", [fem.F64, fem.F32X2])
def test_section3_iterates_match_oracle(method, N, dtype):
    prob, x0, u, l1, l2 = _section3()
    x, info = _gpu_run(prob, dtype, method, x0, l1, l2, 124, cycle=N)
    ref = ORACLE[method](prob, x0, l1, l2, 124, N)
    tol = 1e-11 if dtype == fem.F64 else 1e-9  # the F32X2 pair carries ~2^-48 of each entry
    assert np.abs(x - ref).max() <= tol * np.abs(ref).max()
    # Dirichlet values stay fixed
    assert np.all(x[prob.nd] == 1.0)
    assert info["iters"] == 124


def test_section3_bounds_on_gpu_iterates():
    prob, x0, u, l1, l2 = _section3()
    e0 = np.linalg.norm(x0 - u)
    it = 124
    xr, _ = _gpu_run(prob, fem.F64, fem.RICHARDSON, x0, l1, l2, it)
    x3, i3 = _gpu_run(prob, fem.F64, fem.CHEBYSHEV3, x0, l1, l2, it)
    x2, _ = _gpu_run(prob, fem.F64, fem.CHEBYSHEV2, x0, l1, l2, it, cycle=32)
    q = (math.sqrt(l2) - math.sqrt(l1)) / (math.sqrt(l2) + math.sqrt(l1))
    er, e2, e3 = (np.linalg.norm(v - u) for v in (xr, x2, x3))
    assert er <= ((l2 - l1) / (l2 + l1)) ** it * e0 * (1 + 1e-9)
    assert e3 <= 2 * q ** it * e0 * (1 + 1e-6)
    assert e3 < 1e-2 * er and e3 < e2
    # 2-level N = 32 over one whole cycle meets its bound; three cycles exceed it by far (Section 3)
    x32, _ = _gpu_run(prob, fem.F64, fem.CHEBYSHEV2, x0, l1, l2, 32, cycle=32)
    assert np.linalg.norm(x32 - u) <= 2 * q ** 32 * e0
    x96, _ = _gpu_run(prob, fem.F64, fem.CHEBYSHEV2, x0, l1, l2, 96, cycle=32)
    assert np.linalg.norm(x96 - u) > 5 * (2 * q ** 32) ** 3 * e0
    # the reported residual is the oracle's
    r = oracle.residual(prob.n, prob.mesh.elems, prob.K, prob.M, 0.0, prob.b, x3, prob.mask)
    r0 = oracle.residual(prob.n, prob.mesh.elems, prob.K, prob.M, 0.0, prob.b, x0, prob.mask)
    assert i3["relres"] == pytest.approx(np.linalg.norm(r) / np.linalg.norm(r0), rel=1e-8)


def test_three_level_3d_with_mass_term():
    prob = Problem(inputs.cube_mesh(6), nu=10.0)
    x0 = np.zeros(prob.n)
    # bounds of the masked operator from the oracle's dense matrix (small mesh)
    n = prob.n
    A = np.zeros((n, n))
    for e, el in enumerate(prob.mesh.elems):
        A[np.ix_(el, el)] += prob.K[e] + 10.0 * prob.M[e]
    free = ~prob.mask.astype(bool)
    ev = np.linalg.eigvalsh(A[np.ix_(free, free)])
    l1, l2 = ev[0], ev[-1]
    x, _ = _gpu_run(prob, fem.F64, fem.CHEBYSHEV3, x0, l1, l2, 60, nu=10.0)
    ref = oracle.cheb3(n, prob.mesh.elems, prob.K, prob.M, 10.0, prob.b, prob.mask, x0, l1, l2, 60)
    assert np.abs(x - ref).max() <= 1e-11 * np.abs(ref).max()


def test_richardson_equals_one_root_chebyshev_on_gpu():
    prob, x0, u, l1, l2 = _section3(17)
    xr, _ = _gpu_run(prob, fem.F64, fem.RICHARDSON, x0, l1, l2, 20)
    x1, _ = _gpu_run(prob, fem.F64, fem.CHEBYSHEV2, x0, l1, l2, 20, cycle=1)
    # alpha_0 = d + c cos(pi / 2) equals d up to cos(pi / 2) = 6e-17 in floating point
    np.testing.assert_allclose(xr, x1, rtol=0, atol=1e-14 * np.abs(xr).max())


def test_iterate_rejects_bad_bounds():
    prob, x0, u, l1, l2 = _section3(9)
    with pytest.raises(fem.FemError):
        _gpu_run(prob, fem.F64, fem.CHEBYSHEV3, x0, l2, l1, 5)
    with pytest.raises(fem.FemError):
        _gpu_run(prob, fem.F64, fem.CHEBYSHEV2, x0, l1, l2, 5, cycle=0)
