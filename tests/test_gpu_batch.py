"""The batched persistent solver against the FP64 oracle, problem by problem."""
import numpy as np
import pytest
import torch

import oracle
from paper_1911_03973_amd import inputs

from problems import Problem

pytestmark = pytest.mark.gpu

fem = pytest.importorskip("paper_1911_03973_amd.fem")


def _batch(meshes, nus, fseeds, dirichlet="all", chunk=0):
    probs = [Problem(m, nu=nu, dirichlet=dirichlet, f="sine", seed=s) for m, nu, s in zip(meshes, nus, fseeds)]
    B = fem.Batch(meshes, [p.nd for p in probs], chunk_elems=chunk)
    K = B.empty_matrix(fem.F32X2)
    M = B.empty_matrix(fem.F32X2)
    B.build_local_matrices(fem.F32X2, K, M)
    f = torch.from_numpy(np.concatenate([p.f for p in probs])).cuda()
    b = torch.empty(B.n_nodes, dtype=torch.float64, device="cuda")
    B.assemble_rhs(fem.F32X2, M, f, b)
    return probs, B, K, M, b


def _check_solutions(probs, B, x, res, tol=1e-8):
    xs = x.cpu().numpy()
    for i, p in enumerate(probs):
        xi = xs[B.node_off[i]:B.node_off[i + 1]]
        r = oracle.residual(p.n, p.mesh.elems, p.K, p.M, p.nu, p.b, xi, p.mask)
        r0 = oracle.residual(p.n, p.mesh.elems, p.K, p.M, p.nu, p.b, np.zeros(p.n), p.mask)
        rel = np.linalg.norm(r) / np.linalg.norm(r0)
        assert res[i]["status"] == 0, (i, res[i])
        assert rel <= tol, (i, rel, res[i])
        _, io = oracle.pcg(p.n, p.mesh.elems, p.K, p.M, p.nu, p.b, p.mask, np.zeros(p.n), rtol=1e-8)
        assert res[i]["iters"] <= 1.1 * io["iters"] + 2, (i, res[i]["iters"], io["iters"])


@pytest.mark.parametrize("chunk,inline", [(0, 64), (256, 64), (256, 0), (64, 1)])
def test_batch_2d_uneven_sizes(chunk, inline):
    """inline = 0 runs every shared-node fix-up as separate queue items; 1 mixes both paths."""
    ns = [8, 17, 30, 12, 41, 3]
    nus = [1e-3, 0.5, 10.0, 1e3, 1.0, 0.0]
    meshes = [inputs.square_mesh(n, jitter=0.15, seed=i) for i, n in enumerate(ns)]
    probs, B, K, M, b = _batch(meshes, nus, list(range(100, 106)), chunk=chunk)
    print(B.stats())
    x = torch.zeros(B.n_nodes, dtype=torch.float64, device="cuda")
    rc, res, sec = B.solve(fem.batch_opts(use_graph=0, watchdog_seconds=20.0, inline_segments=inline), K, M, nus,
                           b, x)
    print(rc, res, sec)
    assert rc == 0
    _check_solutions(probs, B, x, res)


def test_batch_3d_and_graph_replay_is_bitwise_stable():
    meshes = [inputs.cube_mesh(n, jitter=0.1, seed=n) for n in (4, 7, 5)]
    nus = [10.0, 0.1, 1.0]
    probs, B, K, M, b = _batch(meshes, nus, [7, 8, 9])
    outs = []
    for _ in range(3):
        x = torch.zeros(B.n_nodes, dtype=torch.float64, device="cuda")
        rc, res, sec = B.solve(fem.batch_opts(use_graph=1, watchdog_seconds=20.0), K, M, nus, b, x)
        assert rc == 0
        outs.append(x.cpu().numpy())
    _check_solutions(probs, B, x, res)
    # replays of the captured graph, with dynamic scheduling, give the same bits
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])


def test_batch_matches_single_problem_solver():
    meshes = [inputs.square_mesh(n, jitter=0.2, seed=n) for n in (20, 33)]
    nus = [2.0, 0.3]
    probs, B, K, M, b = _batch(meshes, nus, [1, 2], chunk=256)
    x = torch.zeros(B.n_nodes, dtype=torch.float64, device="cuda")
    rc, res, _ = B.solve(fem.batch_opts(use_graph=0), K, M, nus, b, x)
    assert rc == 0
    for i, p in enumerate(probs):
        plan = fem.Plan.from_mesh(p.mesh, p.nd, chunk_elems=256)
        Ks = plan.empty_matrix(fem.F32X2)
        Ms = plan.empty_matrix(fem.F32X2)
        fem.build_local_matrices(plan, fem.F32X2, Ks, Ms, None)
        xs = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        bi = b[B.node_off[i]:B.node_off[i + 1]].clone()
        info = fem.pcg_solve(plan, fem.solve_opts(dtype=fem.F32X2, nu=p.nu), Ks, Ms, bi, xs)
        # same algorithm, same chunking: same iteration count
        assert res[i]["iters"] == info["iters"], (res[i], info)
        xb = x[B.node_off[i]:B.node_off[i + 1]].cpu().numpy()
        assert np.abs(xb - xs.cpu().numpy()).max() <= 1e-9 * np.abs(xb).max()


def test_autotuners_return_valid_schedules():
    from paper_1911_03973_amd import autotune

    mesh = inputs.square_mesh(48, jitter=0.1, seed=3)
    nd = inputs.boundary_nodes(mesh)
    r = autotune.autotune_solver(mesh, nd, 1.0, chunks=(256, 512), blocks=(256, 512), iters=16)
    assert r["chunk_elems"] in (256, 512) and r["block"] in (256, 512) and len(r["table"]) == 4
    assert all(t["pass_us"] > 0 for t in r["table"])
    meshes = [inputs.square_mesh(n) for n in (10, 25)]
    dirs = [inputs.boundary_nodes(m) for m in meshes]

    def b_fn(B, K, M):
        b = torch.empty(B.n_nodes, dtype=torch.float64, device="cuda")
        B.assemble_rhs(fem.F32X2, M, torch.ones(B.n_nodes, dtype=torch.float64, device="cuda"), b)
        return b

    rb = autotune.autotune_batch(meshes, dirs, [1.0, 0.1], b_fn, chunks=(256,), blocks=(256,), items=(1, 4), iters=10)
    assert rb["items_per_phase"] in (1, 4) and len(rb["table"]) == 2
    # default: every candidate is scored on whole solves
    rb = autotune.autotune_batch(meshes, dirs, [1.0, 0.1], b_fn, chunks=(256,), blocks=(256,), items=(2, 4))
    assert rb["items_per_phase"] in (2, 4) and len(rb["table"]) == 2 and all(t["seconds"] > 0 for t in rb["table"])


def test_adaptive_grouping_gives_identical_bits():
    """Regrouping a problem's chunks into more work items, and moving its
    fix-up to separate items, once few problems are left (adaptive, the
    default) leaves every sum in the same order: the solutions agree bit for
    bit with the fixed schedule."""
    ns = [40, 9, 25, 33, 14]
    nus = [1.0, 1e-2, 30.0, 0.2, 5.0]
    meshes = [inputs.square_mesh(n, jitter=0.2, seed=i + 20) for i, n in enumerate(ns)]
    probs, B, K, M, b = _batch(meshes, nus, list(range(30, 35)), chunk=128)
    outs = []
    for adaptive in (1, 0):
        x = torch.zeros(B.n_nodes, dtype=torch.float64, device="cuda")
        rc, res, _ = B.solve(fem.batch_opts(use_graph=0, watchdog_seconds=20.0, items_per_phase=2,
                                            adaptive=adaptive), K, M, nus, b, x)
        assert rc == 0
        outs.append((x.cpu().numpy(), [r["iters"] for r in res]))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1]
    _check_solutions(probs, B, x, res)
