"""Tile-schedule autotuner for the element solvers.

A schedule is (chunk_elems, workgroup size) for a single solve, plus the
number of work items per problem phase for a batched solve.  Candidates are
timed on the caller's own inputs with short, capped solves (the iterations
are identical whatever the schedule, so a fixed iteration budget compares like
with like); the fastest is returned together with the full table.  Plans have
to be rebuilt for every chunk size, so the tuner is meant to run once per mesh
family, before the timed work.
"""
from __future__ import annotations

import time

import torch

from . import fem

CHUNKS_2D = (512, 1024, 2048)
CHUNKS_3D = (512, 1024, 1536)
BLOCKS = (256, 512, 1024)


def _valid(nb, E, BS):
    if nb == 4 and E > 1536:
        return False
    return not (BS == 1024 and E < 1024)


def autotune_solver(mesh, dirichlet, nu, dtype=fem.F32X2, chunks=None, blocks=BLOCKS, iters=64, f=None):
    """Pick (chunk_elems, block) for fem_pcg_solve on this mesh.

    Each candidate runs `iters` CG iterations with every element pass timed by
    HIP events; the score is the mean element-pass time.
    Returns {"chunk_elems", "block", "pass_us", "table": [...]}.
    """
    nb = mesh.nb
    chunks = chunks or (CHUNKS_2D if nb == 3 else CHUNKS_3D)
    table = []
    for E in chunks:
        plan = fem.Plan.from_mesh(mesh, dirichlet, chunk_elems=E)
        K = plan.empty_matrix(dtype)
        M = plan.empty_matrix(dtype)
        fem.build_local_matrices(plan, dtype, K, M, None)
        ff = torch.ones(mesh.n_nodes, dtype=torch.float64, device="cuda") if f is None else f
        b = plan.empty_vector()
        fem.assemble_rhs(plan, dtype, M, ff, b)
        for BS in blocks:
            if not _valid(nb, E, BS):
                continue
            x = torch.zeros(mesh.n_nodes, dtype=torch.float64, device="cuda")
            opts = fem.solve_opts(dtype=dtype, nu=nu, max_iter=iters, check_every=iters, profile=1, block=BS,
                                  rtol=1e-12)
            info = fem.pcg_solve(plan, opts, K, M if nu else None, b, x)
            us = info["matvec_ms"] * 1e3 / max(info["matvec_samples"], 1)
            table.append({"chunk_elems": E, "block": BS, "pass_us": round(us, 2)})
        del plan, K, M
    best = min(table, key=lambda r: r["pass_us"])
    return dict(best, table=table)


def autotune_batch(meshes, dirichlets, nus, b_fn, dtype=fem.F32X2, chunks=(1024, 2048), blocks=(256, 512),
                   items=(4, 8, 16), iters=None, rtol=1e-8):
    """Pick (chunk_elems, block, items_per_phase) for fem_batch_solve.

    b_fn(batch, K, M) -> b must return the right-hand side on the batch's node
    numbering.  Each candidate solves every problem to `rtol` inside one
    persistent launch (with `iters`, at most that many CG iterations per
    problem instead) and the score is its wall time.  Whole solves are the
    default because a short run keeps every problem live and never shows the
    tail in which only the largest problems are left, where long work items
    and few queue trips win.
    Returns {"chunk_elems", "block", "items_per_phase", "seconds", "table"}.
    """
    table = []
    for E in chunks:
        B = fem.Batch(meshes, dirichlets, chunk_elems=E)
        K = B.empty_matrix(dtype)
        M = B.empty_matrix(dtype)
        B.build_local_matrices(dtype, K, M)
        b = b_fn(B, K, M)
        for BS in blocks:
            if not _valid(B.nb, E, BS):
                continue
            for it in items:
                x = torch.zeros(B.n_nodes, dtype=torch.float64, device="cuda")
                opts = fem.batch_opts(dtype=dtype, rtol=rtol, max_iter=iters if iters else 100000, block=BS,
                                      items_per_phase=it, use_graph=0, watchdog_seconds=60.0)
                torch.cuda.synchronize()
                t = time.perf_counter()
                B.solve(opts, K, M, nus, b, x, allow=(fem.FEM_ENOCONV, fem.FEM_OK))
                torch.cuda.synchronize()
                table.append({"chunk_elems": E, "block": BS, "items_per_phase": it,
                              "seconds": round(time.perf_counter() - t, 4)})
        del B, K, M
    best = min(table, key=lambda r: r["seconds"])
    return dict(best, table=table)
