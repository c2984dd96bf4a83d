"""Solver parity: GPU Jacobi-PCG (FP64 and FP32 with FP64 reliable updates)
against the FP64 oracle.  CG amplifies rounding differences, so the final
iterates are not compared bit for bit; instead
  * the first 10 FP64 iterates match the oracle's to 1e-10,
  * iteration counts agree within 2 %,
  * the oracle's own FP64 residual of the GPU solution meets the target.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1911_03973_amd import inputs

from problems import Problem, cuda, max_rel, to_soa

pytestmark = pytest.mark.gpu

fem = pytest.importorskip("paper_1911_03973_amd.fem")


def _setup(prob, plan, dtype):
    K = plan.empty_matrix(dtype)
    M = plan.empty_matrix(dtype)
    fem.build_local_matrices(plan, dtype, K, M, None)
    return K, M


def _x0(prob, values=None):
    x0 = np.zeros(prob.n)
    if values is not None:
        x0[prob.nd] = values[prob.nd]
    return x0


def _true_relres(prob, x, x0):
    r = oracle.residual(prob.n, prob.mesh.elems, prob.K, prob.M, prob.nu, prob.b, x, prob.mask)
    r0 = oracle.residual(prob.n, prob.mesh.elems, prob.K, prob.M, prob.nu, prob.b, x0, prob.mask)
    return np.linalg.norm(r) / np.linalg.norm(r0)


def test_config1_jacobi_pcg_fp64():
    """64x64 squares, f = 1, nu = 0, homogeneous Dirichlet, FP64 local matrices."""
    mesh = inputs.square_mesh(64)
    prob = Problem(mesh, nu=0.0, dirichlet="all")
    plan = fem.Plan.from_mesh(mesh, prob.nd)
    K, M = _setup(prob, plan, fem.F64)
    b = cuda(prob.b)
    x = cuda(_x0(prob))
    info = fem.pcg_solve(plan, fem.solve_opts(dtype=fem.F64, nu=0.0, rtol=1e-8, check_every=8), K, None, b, x)
    xo, io = oracle.pcg(prob.n, mesh.elems, prob.K, prob.M, 0.0, prob.b, prob.mask, _x0(prob), rtol=1e-8)
    print(info, io)
    assert info["status"] == fem.FEM_OK
    assert info["relres"] <= 1e-8
    assert abs(info["iters"] - io["iters"]) <= max(1, 0.02 * io["iters"])
    assert _true_relres(prob, x.cpu().numpy(), _x0(prob)) <= 1e-8
    assert max_rel(x.cpu().numpy(), xo) <= 1e-6


@pytest.mark.parametrize("dim", [2, 3])
def test_first_iterates_match_oracle(dim):
    mesh = inputs.square_mesh(24, jitter=0.2, seed=9) if dim == 2 else inputs.cube_mesh(8, jitter=0.1, seed=9)
    prob = Problem(mesh, nu=2.5, dirichlet="all", f="sine", seed=3)
    plan = fem.Plan.from_mesh(mesh, prob.nd, chunk_elems=256)
    K, M = _setup(prob, plan, fem.F64)
    u = 1.0 + mesh.coords[:, 0]
    for k in (1, 2, 5, 10):
        x = cuda(_x0(prob, u))
        info = fem.pcg_solve(plan, fem.solve_opts(dtype=fem.F64, nu=prob.nu, max_iter=k, check_every=4), K, M,
                             cuda(prob.b), x)
        xo, io = oracle.pcg(prob.n, mesh.elems, prob.K, prob.M, prob.nu, prob.b, prob.mask, _x0(prob, u),
                            max_iter=k, raise_on_noconv=False)
        assert info["iters"] == io["iters"] == k
        assert max_rel(x.cpu().numpy(), xo) <= 1e-10, k


def test_fp64_solve_3d_and_dirichlet_values():
    mesh = inputs.cube_mesh(10, jitter=0.1, seed=4)
    prob = Problem(mesh, nu=10.0, dirichlet="all")
    plan = fem.Plan.from_mesh(mesh, prob.nd)
    K, M = _setup(prob, plan, fem.F64)
    u = 0.5 - mesh.coords[:, 2]
    x0 = _x0(prob, u)
    x = cuda(x0)
    info = fem.pcg_solve(plan, fem.solve_opts(dtype=fem.F64, nu=prob.nu), K, M, cuda(prob.b), x)
    assert info["status"] == fem.FEM_OK
    xs = x.cpu().numpy()
    np.testing.assert_array_equal(xs[prob.nd], x0[prob.nd])
    assert _true_relres(prob, xs, x0) <= 1e-8
    _, io = oracle.pcg(prob.n, mesh.elems, prob.K, prob.M, prob.nu, prob.b, prob.mask, x0, rtol=1e-8)
    assert abs(info["iters"] - io["iters"]) <= max(1, 0.02 * io["iters"])


@pytest.mark.parametrize("dim,dtype,vectors", [(2, 2, 0), (3, 2, 0), (2, 1, 0), (2, 2, 1), (3, 2, 1)])
def test_mixed_precision_reaches_fp64_target(dim, dtype, vectors):
    """FP32 inner CG with FP64 reliable updates: the oracle's FP64 residual of
    the GPU solution meets 1e-8 (for FP32X2 storage; plain FP32 storage solves
    the FP32-rounded operator, whose own solution is only ~1e-5 accurate, so
    there the GPU's residual is judged against the stored operator)."""
    if dim == 2:
        mesh = inputs.square_mesh(96, jitter=0.2, seed=0)
        prob = Problem(mesh, nu=1.0, dirichlet="x2=0", f="sine", seed=1)
    else:
        mesh = inputs.cube_mesh(14)
        prob = Problem(mesh, nu=10.0, dirichlet="all")
    plan = fem.Plan.from_mesh(mesh, prob.nd)
    K, M = _setup(prob, plan, dtype)
    x = cuda(_x0(prob))
    info = fem.pcg_solve(plan, fem.solve_opts(dtype=dtype, nu=prob.nu, rtol=1e-8, vectors=vectors), K, M,
                         cuda(prob.b), x)
    print(info)
    assert info["status"] == fem.FEM_OK
    assert info["relres"] <= 1e-8
    if dtype == fem.F32X2:
        assert _true_relres(prob, x.cpu().numpy(), _x0(prob)) <= 1e-8
    _, io = oracle.pcg(prob.n, mesh.elems, prob.K, prob.M, prob.nu, prob.b, prob.mask, _x0(prob), rtol=1e-8)
    # FP64 vectors keep the FP64 iteration count; FP32 vectors lose some
    assert info["iters"] <= (1.1 if vectors == 0 else 1.6) * io["iters"]


def test_solver_reports_noconv_and_keeps_iterate():
    mesh = inputs.square_mesh(32)
    prob = Problem(mesh, nu=0.0, dirichlet="all")
    plan = fem.Plan.from_mesh(mesh, prob.nd)
    K, _ = _setup(prob, plan, fem.F64)
    x = cuda(_x0(prob))
    info = fem.pcg_solve(plan, fem.solve_opts(dtype=fem.F64, max_iter=7, check_every=3), K, None, cuda(prob.b), x)
    assert info["status"] == fem.FEM_ENOCONV and info["iters"] == 7
    xo, _ = oracle.pcg(prob.n, mesh.elems, prob.K, prob.M, 0.0, prob.b, prob.mask, _x0(prob), max_iter=7,
                       raise_on_noconv=False)
    assert max_rel(x.cpu().numpy(), xo) <= 1e-10


def test_solve_is_bitwise_reproducible():
    mesh = inputs.square_mesh(40, jitter=0.2, seed=5)
    prob = Problem(mesh, nu=1.0, dirichlet="x2=0", f="sine", seed=2)
    plan = fem.Plan.from_mesh(mesh, prob.nd, chunk_elems=128)
    K, M = _setup(prob, plan, fem.F32X2)
    outs = []
    for _ in range(2):
        x = cuda(_x0(prob))
        fem.pcg_solve(plan, fem.solve_opts(dtype=fem.F32X2, nu=1.0), K, M, cuda(prob.b), x)
        outs.append(x.cpu().numpy())
    np.testing.assert_array_equal(outs[0], outs[1])


@pytest.mark.parametrize("dtype,check_every", [(fem.F64, 7), (fem.F32X2, 16), (fem.F32X2, 1)])
def test_graph_replayed_iterations_equal_eager_launches(dtype, check_every):
    """Without per-pass timing (profile = 0) check_every iterations replay as one
    HIP graph, captured once and reused by later solves; with profile > 0 every
    kernel is launched on its own.  Three graph solves in a row, with the
    refreshes and state reads between the replays, give the eager solve's
    iterate bit for bit and its iteration count."""
    mesh = inputs.square_mesh(48, jitter=0.2, seed=6)
    prob = Problem(mesh, nu=2.0, dirichlet="x2=0", f="sine", seed=3)
    plan = fem.Plan.from_mesh(mesh, prob.nd, chunk_elems=256)
    K, M = _setup(prob, plan, dtype)
    b = cuda(prob.b)
    runs = []
    for profile in (1, 0, 0, 0):
        x = cuda(_x0(prob))
        info = fem.pcg_solve(plan, fem.solve_opts(dtype=dtype, nu=2.0, check_every=check_every, profile=profile),
                             K, M, b, x)
        assert info["status"] == 0
        runs.append((x.cpu().numpy(), info["iters"], info["relres"]))
    for x, it, rr in runs[1:]:
        np.testing.assert_array_equal(x, runs[0][0])
        assert it == runs[0][1] and rr == runs[0][2]
