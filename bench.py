"""Benchmark of the element-based solver hot path on one MI355X.

Workload (default): 2-D P1, 2048 x 2048 squares cut along their diagonal
(4,198,401 nodes, 8,388,608 triangles), interior nodes jittered by +-0.2h
(seed 0), nu = 1, f = sum of 8 random sines (seed 1), Dirichlet u = 0 on
x2 = 0 and homogeneous Neumann elsewhere; local matrices stored as FP32 hi/lo
pairs, Jacobi-PCG with FP32 element matvec and FP64 reliable-update
refinement to a true relative residual of 1e-8.

One step = the whole hot path on resident device inputs: build all K_e, M_e,
assemble b, combine A_e = K_e + nu M_e, Jacobi diagonal, and the solve.
`value` is the element-operator throughput in GB/s: algorithmic bytes of one
FP32 element matvec divided by its mean duration, timed with HIP events on the
solver's stream (every `--profile`-th matvec of the timed steps).  The
time-to-1e-8 of the solve is reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "element-residual GB/s (% HBM peak); time-to-1e-8 learned-FCG vs Jacobi-PCG"

WORKLOADS = {
    "c2": dict(dim=2, n=2048, jitter=0.2, jseed=0, nu=1.0, f="sine", fseed=1, dirichlet="x2=0", dtype="f32x2",
               name="2D P1 2048x2048 squares (4198401 nodes, 8388608 triangles), jitter 0.2h, nu=1, "
                    "random-sine f, Dirichlet x2=0; FP32 element matvec + FP64 refinement to 1e-8"),
    "c1": dict(dim=2, n=64, jitter=0.0, jseed=0, nu=0.0, f="one", fseed=0, dirichlet="all", dtype="f64",
               name="2D P1 64x64 squares (4225 nodes, 8192 triangles), nu=0, f=1, full Dirichlet; FP64 Jacobi-PCG"),
    "c4": dict(dim=2, n=0, jitter=0.0, jseed=0, nu=None, f="sine", fseed=0, dirichlet="all", dtype="f32x2",
               name="batched: 256 independent 2D P1 problems, N~U{32..512} squares per side, nu log-uniform "
                    "[1e-3,1e3], random-sine f (per-problem seeds), full Dirichlet; one persistent launch, "
                    "FP32 element matvec + FP64 refinement to 1e-8 per problem"),
    "p2": dict(dim=2, n=1024, jitter=0.2, jseed=0, nu=1.0, f="sine", fseed=1, dirichlet="x2=0", dtype="f32x2",
               order=2,
               name="2D quadratic (P2) triangles on 1024x1024 squares (4198401 nodes, 2097152 triangles), "
                    "jitter 0.2h, nu=1, random-sine f, Dirichlet x2=0; FP32 element matvec + FP64 refinement "
                    "to 1e-8"),
    "p2t": dict(dim=3, n=64, jitter=0.15, jseed=0, nu=10.0, f="sine", fseed=1, dirichlet="all", dtype="f32x2",
                order=2,
                name="3D quadratic (P2) tetrahedra on 64^3 cubes x 6 (2146689 nodes, 1572864 tets), jitter 0.15h, "
                     "nu=10, random-sine f, full Dirichlet; FP32 element matvec + FP64 refinement to 1e-8"),
    "c3": dict(dim=3, n=160, jitter=0.0, jseed=0, nu=10.0, f="one", fseed=0, dirichlet="all", dtype="f32x2",
               name="3D P1 160^3 cubes x 6 tets (4173281 nodes, 24576000 tets), nu=10, f=1, full Dirichlet; "
                    "FP32 element matvec + FP64 refinement to 1e-8"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_problem(w):
    import numpy as np

    from paper_1911_03973_amd import inputs

    if w.get("order") == 2 and w["dim"] == 3:
        mesh = inputs.cube_mesh_p2(w["n"], jitter=w["jitter"], seed=w["jseed"])
    elif w.get("order") == 2:
        mesh = inputs.square_mesh_p2(w["n"], jitter=w["jitter"], seed=w["jseed"])
    elif w["dim"] == 2:
        mesh = inputs.square_mesh(w["n"], jitter=w["jitter"], seed=w["jseed"])
    else:
        mesh = inputs.cube_mesh(w["n"], jitter=w["jitter"], seed=w["jseed"])
    nd = inputs.boundary_nodes(mesh, w["dirichlet"])
    f = inputs.random_sine(mesh.coords, w["fseed"]) if w["f"] == "sine" else np.ones(mesh.n_nodes)
    return mesh, nd, f


def cpu_baseline(mesh, w, seconds):
    """The FP64 oracle's element residual on the same mesh (one host thread)."""
    import numpy as np

    import oracle

    t = time.perf_counter()
    if mesh.nb == 6:
        import oracle.p2

        K, M, _ = oracle.p2.local_matrices_p2(mesh.coords, mesh.elems)
    elif mesh.nb == 10:
        import oracle.p2

        K, M, _ = oracle.p2.local_matrices_p2_tet(mesh.coords, mesh.elems)
    else:
        K, M, _ = oracle.local_matrices(mesh.coords, mesh.elems)
    t_local = time.perf_counter() - t
    rng = np.random.default_rng(0)
    x = rng.standard_normal(mesh.n_nodes)
    b = rng.standard_normal(mesh.n_nodes)
    mask = oracle.mask_from_nodes(mesh.n_nodes, inputs_boundary(mesh, w))
    calls, t0 = 0, time.perf_counter()
    while True:
        oracle.residual(mesh.n_nodes, mesh.elems, K, M, w["nu"], b, x, mask)
        calls += 1
        el = time.perf_counter() - t0
        if el >= seconds and calls >= 2:
            break
    per = el / calls
    nb = mesh.nb
    bytes_call = mesh.n_elems * (nb * nb * 8 + 4 * nb) + mesh.n_nodes * 3 * 8
    return {
        "value": round(bytes_call / per / 1e9, 3),
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{calls} calls of the FP64 oracle element residual on the full mesh "
                   f"({mesh.n_elems} elements), {per * 1e3:.1f} ms each, {mesh.n_elems / per:.3e} elements/s; "
                   f"bytes counted as FP64 combined A_e (the oracle reads K_e and M_e separately); "
                   f"oracle local matrices {t_local:.2f} s"),
    }


def host_facts():
    """Host CPU of this run: model name, logical CPUs, CPUs this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0))}


def cpu_allcores(mesh, w, seconds):
    """The FP64 oracle's element residual on every usable host core (at most 16, this machine's CPU share per
    GPU): the element list cut into one contiguous range per thread, each range through the unchanged
    oracle routine with b absent (ctypes releases the GIL during the call), the partial residuals added
    pairwise in a fixed tree.  Checked against the one-thread oracle to 1e-12."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle

    facts = host_facts()
    T = max(1, min(16, facts["usable_cpus"]))
    K, M, _ = oracle.local_matrices(mesh.coords, mesh.elems)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(mesh.n_nodes)
    b = rng.standard_normal(mesh.n_nodes)
    mask = oracle.mask_from_nodes(mesh.n_nodes, inputs_boundary(mesh, w))
    bm = np.where(mask != 0, 0.0, b)
    cut = np.linspace(0, mesh.n_elems, T + 1).astype(np.int64)
    nu = w["nu"]

    def part(t):
        a, e = cut[t], cut[t + 1]
        return oracle.residual(mesh.n_nodes, mesh.elems[a:e], K[a:e], M[a:e], nu, None, x, mask)

    def add(ab):
        a, b = ab
        a += b
        return a

    with ThreadPoolExecutor(T) as pool:
        def call():
            # the partials added pairwise in a fixed tree, each level's sums on the threads
            parts = list(pool.map(part, range(T)))
            while len(parts) > 1:
                nxt = list(pool.map(add, [(parts[i], parts[i + 1]) for i in range(0, len(parts) - 1, 2)]))
                parts = nxt + ([parts[-1]] if len(parts) % 2 else [])
            return parts[0] + bm

        ref = oracle.residual(mesh.n_nodes, mesh.elems, K, M, nu, b, x, mask)
        r = call()
        assert np.abs(r - ref).max() <= 1e-12 * np.abs(ref).max(), "threaded oracle residual differs"
        calls, t0 = 0, time.perf_counter()
        while True:
            call()
            calls += 1
            el = time.perf_counter() - t0
            if el >= seconds and calls >= 2:
                break
    per = el / calls
    nb = mesh.nb
    bytes_call = mesh.n_elems * (nb * nb * 8 + 4 * nb) + mesh.n_nodes * 3 * 8
    return {"value": round(bytes_call / per / 1e9, 3), "unit": "GB/s", "cores": T, "kind": "oracle",
            "sample": f"{calls} calls of the FP64 oracle element residual on the full mesh split over {T} threads, "
                      f"{per * 1e3:.1f} ms each, {mesh.n_elems / per:.3e} elements/s", **facts}


def oracle_pcg_times(seconds, c3_iters=None, c5_iters=None):
    """The FP64 oracle's Jacobi-PCG (one host thread): C1 solved to 1e-8 in full; on C5 (1024^2, nu 35.55,
    random-sine f seed 5002) and C3 the time per iteration from a capped run, and the time to 1e-8
    projected with the GPU's Jacobi-PCG iteration count for the same problem."""
    import numpy as np

    import oracle
    from paper_1911_03973_amd import inputs

    out = {}
    w = WORKLOADS["c1"]
    mesh, nd, f = make_problem(w)
    K, M, _ = oracle.local_matrices(mesh.coords, mesh.elems)
    mask = oracle.mask_from_nodes(mesh.n_nodes, nd)
    b = oracle.rhs(mesh.n_nodes, mesh.elems, M, f)
    t = time.perf_counter()
    _, info = oracle.pcg(mesh.n_nodes, mesh.elems, K, M, w["nu"], b, mask, np.zeros(mesh.n_nodes), rtol=1e-8)
    out["c1"] = {"time_to_1e8_s": round(time.perf_counter() - t, 4), "iters": info["iters"],
                 "relres": info["relres"]}

    def capped(name, mesh, nd, nu, f, iters_gpu):
        K, M, _ = oracle.local_matrices(mesh.coords, mesh.elems)
        mask = oracle.mask_from_nodes(mesh.n_nodes, nd)
        b = oracle.rhs(mesh.n_nodes, mesh.elems, M, f)
        x0 = np.zeros(mesh.n_nodes)
        t = time.perf_counter()
        oracle.pcg(mesh.n_nodes, mesh.elems, K, M, nu, b, mask, x0, rtol=1e-30, max_iter=3, raise_on_noconv=False)
        per = (time.perf_counter() - t) / 3
        k = max(3, min(2000, int(seconds / max(per, 1e-9))))
        t = time.perf_counter()
        _, info = oracle.pcg(mesh.n_nodes, mesh.elems, K, M, nu, b, mask, x0, rtol=1e-30, max_iter=k,
                             raise_on_noconv=False)
        per = (time.perf_counter() - t) / max(info["iters"], 1)
        out[name] = {"iters_run": info["iters"], "s_per_iter": round(per, 5),
                     "gpu_jacobi_pcg_iters": iters_gpu,
                     "projected_time_to_1e8_s": round(per * iters_gpu, 2) if iters_gpu else None}

    m5 = inputs.square_mesh(1024)
    capped("c5", m5, inputs.boundary_nodes(m5, "all"), 35.547, inputs.random_sine(m5.coords, 5002), c5_iters)
    del m5
    w = WORKLOADS["c3"]
    m3, nd3, f3 = make_problem(w)
    capped("c3", m3, nd3, w["nu"], f3, c3_iters)
    return out


def other_configs(args):
    """C3, C1 and C4 on the same GPU after the headline workload (fewer timed steps)."""
    import argparse

    out = {}
    r = measure_single(args, "c3", steps=3, warmup=1)
    out["c3"] = {"workload": r["config"]["workload"], "fused_pass_GBps": r["value"], "frac": r["roofline"]["frac"],
                 "matvec_us": r["matvec_us"], "matvec_bytes": r["matvec_bytes"],
                 "elements_per_s": r["elements_per_s"], "time_to_1e8_s": r["time_to_1e8_s"],
                 "iters": r["iters"][-1], "relres": max(r["relres"]), "converged": r["converged"],
                 "residual_kernels": r["residual_kernels"]}
    a1 = argparse.Namespace(**vars(args))
    a1.profile = 0  # no per-pass events: the iterations replay as HIP graphs
    r = measure_single(a1, "c1", steps=10, warmup=2, residual=False)
    out["c1"] = {"workload": r["config"]["workload"], "time_to_1e8_s": r["time_to_1e8_s"], "iters": r["iters"][-1],
                 "relres": max(r["relres"]), "converged": r["converged"],
                 "note": "0.8 MB of element data: cache-resident, launch-latency bound"}
    a4 = argparse.Namespace(**vars(args))
    a4.steps, a4.warmup = 1, 1
    r = run_batched(a4, WORKLOADS["c4"])
    out["c4"] = {"workload": r["config"]["workload"], "time_to_1e8_s": r["time_to_1e8_s"], "GBps": r["value"],
                 "frac": r["roofline"]["frac"], "all_converged": r["all_converged"], "max_relres": r["max_relres"],
                 "iters_total": r["iters_total"], "schedule": r["schedule"]}
    return out


def residual_kernels(fem, plan, mesh, K, M, nu, dt, calls):
    """Standalone element residuals r = b - A x on the same mesh (full n_b x n_b storage)."""
    import torch

    nb = mesh.nb
    out = {}
    g = torch.Generator(device="cuda").manual_seed(0)
    x32 = torch.rand(mesh.n_nodes, device="cuda", generator=g, dtype=torch.float32)
    b32 = torch.rand(mesh.n_nodes, device="cuda", generator=g, dtype=torch.float32)
    r32 = torch.empty_like(x32)
    x64, b64, r64 = x32.double(), b32.double(), torch.empty(mesh.n_nodes, dtype=torch.float64, device="cuda")
    A32 = Ap = None
    cases = []
    if dt != fem.MFREE:
        A32 = plan.empty_matrix(fem.F32)
        fem.combine_local(plan, dt, K, M, nu, fem.F32, A32)
        Ap = plan.empty_matrix(fem.F32X2)
        fem.combine_local(plan, dt, K, M, nu, fem.F32X2, Ap)
        cases += [
            ("f32", lambda: fem.element_residual_f32(plan, A32, b32, x32, r32, mask=True),
             mesh.n_elems * (nb * nb * 4 + 4 * nb) + mesh.n_nodes * 3 * 4),
            ("f64_from_hi_lo", lambda: fem.element_residual(plan, fem.F32X2, Ap, None, 0.0, b64, x64, r64, mask=True),
             mesh.n_elems * (nb * nb * 8 + 4 * nb) + mesh.n_nodes * 3 * 8),
        ]
    # matrix-free FP64: connectivity-equivalent index, coordinates, x and b read, r written
    cases.append(("f64_mfree", lambda: fem.element_residual(plan, fem.MFREE, None, None, nu, b64, x64, r64, mask=True),
                  mesh.n_elems * 4 * nb + mesh.n_nodes * (mesh.dim + 3) * 8))
    for name, fn, nbytes in cases:
        try:
            fn()
        except fem.FemError as e:  # chunk LDS above the workgroup limit
            out[name] = {"refused": str(e)}
            continue
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(calls):
            fn()
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / calls
        out[name] = {"us": round(us, 2), "bytes": nbytes, "GB/s": round(nbytes / us / 1e3, 1),
                     "frac": round(nbytes / us / 1e3 / HBM_PEAK_GBS, 4)}
    del A32, Ap
    return out


def inputs_boundary(mesh, w):
    from paper_1911_03973_amd import inputs

    return inputs.boundary_nodes(mesh, w["dirichlet"])


def run_batched(args, w):
    """Config with 256 problems: one step = local matrices + rhs + the persistent batched solve."""
    import numpy as np
    import torch

    from paper_1911_03973_amd import fem, inputs

    params = inputs.batched_params(args.n_problems)
    log(f"[bench] {len(params)} problems, building meshes")
    meshes, dirs, fs, nus = [], [], [], []
    for n, nu, seed in params:
        m = inputs.square_mesh(n)
        meshes.append(m)
        dirs.append(inputs.boundary_nodes(m))
        fs.append(inputs.random_sine(m.coords, seed))
        nus.append(nu)
    tuned = None
    if args.autotune:
        from paper_1911_03973_amd import autotune

        log("[bench] autotuning the batched schedule (untimed)")
        fcat = torch.from_numpy(np.concatenate(fs)).cuda()

        def b_fn(Bt, Kt, Mt):
            bb = torch.empty(Bt.n_nodes, dtype=torch.float64, device="cuda")
            Bt.assemble_rhs(fem.F32X2, Mt, fcat, bb)
            return bb

        tuned = autotune.autotune_batch(meshes, dirs, nus, b_fn)
        log(f"[bench] autotuned: {dict((k, v) for k, v in tuned.items() if k != 'table')}")
        args.chunk, args.block, args.items = tuned["chunk_elems"], tuned["block"], tuned["items_per_phase"]
    t = time.perf_counter()
    B = fem.Batch(meshes, dirs, chunk_elems=args.chunk or args.batch_chunk)
    t_plan = time.perf_counter() - t
    st = B.stats()
    log(f"[bench] batch plan {t_plan:.2f} s: {st}")
    K = B.empty_matrix(fem.F32X2)
    M = B.empty_matrix(fem.F32X2)
    f = torch.from_numpy(np.concatenate(fs)).cuda()
    b = torch.empty(B.n_nodes, dtype=torch.float64, device="cuda")
    x = torch.empty(B.n_nodes, dtype=torch.float64, device="cuda")
    opts = fem.batch_opts(rtol=1e-8, block=args.block, use_graph=1, watchdog_seconds=60.0, group=args.group,
                          items_per_phase=args.items, inline_segments=args.inline_segs, adaptive=args.adaptive,
                          max_iter=min(args.max_iter, 100000))

    def step():
        B.build_local_matrices(fem.F32X2, K, M)
        B.assemble_rhs(fem.F32X2, M, f, b)
        x.zero_()
        return B.solve(opts, K, M, nus, b, x)

    for i in range(args.warmup):
        rc, res, sec = step()
        log(f"[bench] warmup {i}: rc {rc} solve {sec:.3f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = []
    for i in range(args.steps):
        outs.append(step())
        log(f"[bench] step {i}: rc {outs[-1][0]} solve {outs[-1][2]:.3f} s")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    rc, res, sec = outs[-1]
    iters = np.array([r["iters"] for r in res])
    ne = np.diff(B.elem_off)
    nn = np.diff(B.node_off)
    # algorithmic bytes of the element passes actually run: per problem and
    # iteration the fused pass (6 packed FP32 values + 12 index bytes per
    # element, 9 FP64 vector streams per node)
    pass_bytes = float(np.sum(iters * (ne * (6 * 4 + 12) + nn * 9 * 8)))
    gbs = pass_bytes / sec / 1e9
    out = {
        "metric": METRIC, "value": round(gbs, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w["name"], "n_problems": len(params), "n_nodes": B.n_nodes, "n_elems": B.n_elems,
                   "chunk_elems": st["chunk_elems"], "block": args.block},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None},
        "time_to_1e8_s": round(sec, 4),
        "all_converged": bool(rc == 0 and all(r["status"] == 0 for r in res)),
        "max_relres": max(r["relres"] for r in res),
        "iters_total": int(iters.sum()), "iters_max": int(iters.max()), "iters_min": int(iters.min()),
        "plan_seconds": round(t_plan, 3),
        "note": "value = algorithmic bytes of all element passes of the solve / solve wall time (whole job)",
        "schedule": {"chunk_elems": st["chunk_elems"], "block": args.block, "items_per_phase": args.items,
                     "adaptive": args.adaptive},
        "autotune": tuned,
    }
    return out


MFMA_BF16_PEAK_TFLOPS = 2500.0


def unet_flops(H, W, c=16, real_in=2):
    """Multiply-add flops (2 per MAC) of one U-Net forward on an H x W image."""
    px = lambda lvl: (H >> lvl) * (W >> lvl)  # noqa: E731
    conv = lambda lvl, cin, cout: 2 * 9 * cin * cout * px(lvl)  # noqa: E731
    up = lambda lvl_low, cin, cout: 2 * cin * 4 * cout * px(lvl_low)  # noqa: E731
    f = conv(0, real_in, c) + conv(0, c, c) + conv(1, c, 2 * c) + conv(1, 2 * c, 2 * c)
    f += conv(2, 2 * c, 4 * c) + conv(2, 4 * c, 4 * c) + conv(3, 4 * c, 8 * c) + conv(3, 8 * c, 8 * c)
    f += up(3, 8 * c, 4 * c) + conv(2, 8 * c, 4 * c) + conv(2, 4 * c, 4 * c)
    f += up(2, 4 * c, 2 * c) + conv(1, 4 * c, 2 * c) + conv(1, 2 * c, 2 * c)
    f += up(1, 2 * c, c) + conv(0, 2 * c, c) + conv(0, c, c) + 2 * c * px(0)
    return f


def run_unet(args):
    """U-Net kernels alone: forward (batch 1) and training step (batch 4) at 1024^2, HIP-event timed."""
    import torch

    from paper_1911_03973_amd import fem

    N = args.learned_n
    fwd_flops = unet_flops(N, N)
    net = fem.UNet(N, N, max_batch=4, channels=16, seed=0)
    g = torch.Generator(device="cuda").manual_seed(0)
    inp = torch.randn((4, N, N, 2), generator=g, device="cuda")
    tgt = torch.randn((4, N, N), generator=g, device="cuda")
    x1 = inp[:1].contiguous()
    for _ in range(args.warmup + 1):
        net.forward(x1)
        net.train_step(inp, tgt, 1e-4)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(args.steps, 1) * 10
    s.record()
    for _ in range(reps):
        net.forward(x1)
    e.record()
    torch.cuda.synchronize()
    fwd_ms = s.elapsed_time(e) / reps
    s.record()
    for _ in range(reps):
        net.train_step(inp, tgt, 1e-4)
    e.record()
    torch.cuda.synchronize()
    train_ms = s.elapsed_time(e) / reps
    tf = fwd_flops / (fwd_ms * 1e-3) / 1e12
    train_tf = 3 * 4 * fwd_flops / (train_ms * 1e-3) / 1e12
    out = {
        "metric": "U-Net forward TFLOP/s (BF16 MFMA, FP32 accumulation)", "value": round(tf, 2),
        "unit": "TFLOP/s", "n_gpus": 1, "steps": reps, "warmup": args.warmup,
        "ms_per_step": round(fwd_ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"U-Net 4 levels 16-128 channels, {N}x{N} image, forward batch 1, "
                               f"training step batch 4 (forward + backward + Adam)"},
        "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tf / MFMA_BF16_PEAK_TFLOPS, 4), "traffic": None},
        "forward_gflop": round(fwd_flops / 1e9, 2), "train_step_ms": round(train_ms, 3),
        "train_tflops_3x_forward": round(train_tf, 2),
    }
    print(json.dumps(out), flush=True)


def run_iterations(args):
    """The paper's iterations (Section 2, experiment of Section 3 scaled up): f = 1,
    u = 1 on the boundary of an n x n diagonal-cut mesh, nu = 0, spectral bounds
    of K_II from the closed form 4 sin^2(i pi / 2n) + 4 sin^2(j pi / 2n).  Times
    the 3-level Chebyshev iteration; each step is one element pass that forms the
    FP64 residual (packed difference form) and applies the three-term update."""
    import numpy as np
    import torch

    from paper_1911_03973_amd import fem, inputs

    n = args.iter_n
    mesh = inputs.square_mesh(n)
    nd = inputs.boundary_nodes(mesh, "all")
    plan = fem.Plan.from_mesh(mesh, nd)
    K = plan.empty_matrix(fem.F64)
    M = plan.empty_matrix(fem.F64)
    fem.build_local_matrices(plan, fem.F64, K, M, None)
    b = plan.empty_vector()
    fem.assemble_rhs(plan, fem.F64, M, torch.ones(mesh.n_nodes, dtype=torch.float64, device="cuda"), b)
    x0 = torch.zeros(mesh.n_nodes, dtype=torch.float64, device="cuda")
    x0[torch.from_numpy(nd.astype(np.int64)).cuda()] = 1.0
    lam1 = 8.0 * np.sin(np.pi / (2 * n)) ** 2
    lam2 = 8.0 * np.sin((n - 1) * np.pi / (2 * n)) ** 2

    def solve(iters):
        x = x0.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        info = fem.iterate(plan, fem.iter_opts(method=fem.CHEBYSHEV3, dtype=fem.F64, nu=0.0, lam1=lam1, lam2=lam2,
                                               iters=iters), K, None, b, x)
        torch.cuda.synchronize()
        return time.perf_counter() - t, info

    s1, s2 = args.iter_steps, 2 * args.iter_steps
    for _ in range(args.warmup):
        solve(s1)
    t1 = min(solve(s1)[0] for _ in range(max(args.steps, 1)))
    t2, info = min((solve(s2) for _ in range(max(args.steps, 1))), key=lambda r: r[0])
    per_step = (t2 - t1) / (s2 - s1)  # setup (packing, workspace) cancels
    nb = 3
    n_pk = nb + nb * (nb - 1) // 2
    # one fused pass: packed FP64 values + connectivity per element; per node read x, b,
    # x_prev and write x_new
    step_bytes = mesh.n_elems * (n_pk * 8 + 4 * nb) + mesh.n_nodes * 4 * 8
    gbs = step_bytes / per_step / 1e9
    q = (np.sqrt(lam2) - np.sqrt(lam1)) / (np.sqrt(lam2) + np.sqrt(lam1))
    out = {
        "metric": METRIC, "value": round(gbs, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(per_step * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"Section 3 iterations scaled up: {n}x{n} diagonal-cut squares, f=1, u=1 on the "
                               f"boundary, nu=0; 3-level Chebyshev, FP64 packed operator",
                   "n_nodes": mesh.n_nodes, "n_elems": mesh.n_elems, "lam1": lam1, "lam2": lam2},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None},
        "iteration_us": round(per_step * 1e6, 2), "step_bytes": step_bytes, "elements_per_s": round(
            mesh.n_elems / per_step, 1), "iters": s2, "relres_after": info["relres"],
        "chebyshev_bound_2q_to_the_k": float(2 * q ** s2),
    }
    print(json.dumps(out), flush=True)


def run_multigrid(args):
    """The C2 (or C3) problem solved by FCG with the geometric multigrid
    V-cycle (the hierarchy 2048^2 -> 16^2 of nested square meshes that keep the
    jitter, or 160^3 -> 5^3 of Kuhn cube meshes), against the single-level
    Jacobi-PCG solve of the same problem on the same GPU."""
    import numpy as np
    import torch

    from paper_1911_03973_amd import fem, inputs

    w = WORKLOADS[args.mg_base]
    mesh, nd, f = make_problem(w)
    t = time.perf_counter()
    if w["dim"] == 3:
        meshes = inputs.cube_hierarchy(mesh, coarsest=args.mg_coarsest or 5)
    else:
        meshes = inputs.square_hierarchy(mesh, coarsest=args.mg_coarsest or 16)
    nds = [inputs.boundary_nodes(m, w["dirichlet"]) for m in meshes]
    mg = fem.MG.from_meshes(meshes, nds, w["nu"])
    t_setup = time.perf_counter() - t
    plan = mg.plans[0]
    b = plan.empty_vector()
    fem.assemble_rhs(plan, fem.F64, mg.M[0], torch.from_numpy(f).cuda(), b)
    x = plan.empty_vector()
    smoother = fem.SMOOTH_CHEBYSHEV if args.mg_smoother == "chebyshev" else fem.SMOOTH_JACOBI
    opts = fem.mg_opts(rtol=1e-8, smooth=args.mg_smooth, cycle_dtype=fem.F32 if args.mg_cycle == "f32" else fem.F64,
                       smoother=smoother)

    def mg_solve():
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = mg.solve(opts, b, x)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, info

    for _ in range(args.warmup):
        mg_solve()
    runs = [mg_solve() for _ in range(max(args.steps, 1))]
    sec = float(np.median([r[0] for r in runs]))
    info = runs[-1][1]
    # the single-level reference: Jacobi-PCG, FP32 operator heads in FP64 refinement (the C2 solver)
    K32 = plan.empty_matrix(fem.F32X2)
    M32 = plan.empty_matrix(fem.F32X2)
    fem.build_local_matrices(plan, fem.F32X2, K32, M32, None)
    xj = plan.empty_vector()
    info_j = fem.pcg_solve(plan, fem.solve_opts(dtype=fem.F32X2, nu=w["nu"], rtol=1e-8, check_every=64), K32, M32,
                           b, xj)
    out = {
        "metric": METRIC, "value": round(sec, 4), "unit": "s", "n_gpus": 1, "steps": len(runs),
        "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 3), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w["name"].replace("FP32 element matvec + FP64 refinement to 1e-8",
                                                 "FCG with a geometric multigrid V-cycle, FP64 operators, to 1e-8"),
                   "levels": [m.n for m in meshes], "smooth": args.mg_smooth, "smoother": args.mg_smoother,
                   "cycle": args.mg_cycle},
        "roofline": None,
        "time_to_1e8_s": round(sec, 4), "iters": info["iters"], "relres": info["relres"],
        "vcycles": info["precond_calls"], "setup_s": round(t_setup, 3),
        "jacobi_pcg": {"time_to_1e8_s": round(info_j["seconds"], 4), "iters": info_j["iters"],
                       "relres": info_j["relres"]},
        "speedup_vs_jacobi_pcg": round(info_j["seconds"] / sec, 2),
    }
    print(json.dumps(out), flush=True)


def measured_traffic():
    """HBM bytes per fused CG pass from the committed rocprofv3 counter summary, if it is current.

    profiles/c2_hbm_counters.md carries a line `traffic: {json}` with the
    element-pass source hash the counters were taken with and the calibrated
    FETCH_SIZE + WRITE_SIZE bytes per pass (k_chunk_main + k_chunk_fixup of
    the iteration); any change to those sources makes it stale (None).
    """
    from paper_1911_03973_amd.build import sources_hash

    path = os.path.join(ROOT, "profiles", "c2_hbm_counters.md")
    try:
        with open(path) as f:
            for line in f:
                if line.startswith("traffic: "):
                    rec = json.loads(line[len("traffic: "):])
                    if rec.get("sources") == sources_hash():
                        return rec
    except (OSError, ValueError):
        pass
    return None


def parse_segments(spec):
    """"4x25,8x25" -> [4]*25 + [8]*25 (segment lengths of the pair generator)."""
    out = []
    for part in spec.split(","):
        if "x" in part:
            k, c = part.split("x")
            out += [int(k)] * int(c)
        else:
            out.append(int(part))
    return out


def learned_fcg(args):
    """Learned-preconditioner workload: 1024^2 squares, nu ~ U(0, 100), random-sine f, u = 0 on the boundary.

    Training pairs come from the plain FP64 Jacobi-PCG solver (restarted
    segments from x0 = 0; the error against a multigrid reference solution, see
    paper_1911_03973_amd/learn.py), streamed round by round into the training
    of the network with the library's BF16 MFMA kernels; every pair is used
    once.  Then every held-out problem is solved to a true relative residual of
    1e-8 by (a) Jacobi-PCG with FP32 element passes and FP64 refinement (the
    optimized solver of the main workload) and (b) learned FCG on the same FP32
    hi/lo element matrices.  Training time is reported separately from the
    solve times.
    """
    import numpy as np
    import torch

    from paper_1911_03973_amd import fem, learn

    N = args.learned_n
    segs = parse_segments(args.learned_segments)
    params = learn.problem_params(args.learned_problems, 100)
    log(f"[bench] learned: {len(params)} problems x {len(segs)} snapshots at {N}^2 in {args.learned_rounds} rounds")
    fam = learn.GridFamily(N, fem.F64, mg=True)
    net = fem.UNet(N, N, max_batch=args.learned_batch, channels=16, seed=0)
    if args.learned_loss == "energy":
        learn.use_energy_loss(net, args.learned_out_smooth)
    else:
        net.set_output_smoothing(args.learned_out_smooth)
    hist, n_pairs, t_data, t_train = learn.train_streaming(fam, net, params, segs, args.learned_batch,
                                                           args.learned_lr, args.learned_rounds, log=log,
                                                           epochs=args.learned_epochs)
    del fam
    torch.cuda.empty_cache()
    log(f"[bench] learned: {n_pairs} pairs in {t_data:.1f} s, {len(hist)} steps in {t_train:.1f} s")
    efam = learn.GridFamily(N, fem.F32X2)
    fopts = dict(smooth=args.learned_smooth, cycle_dtype=fem.F32 if args.learned_cycle == "f32" else fem.F64)
    # the same cycle without the network (all its parameters zero: N(r) = 0, s = 0),
    # on the first held-out problems: what the trained network adds to the smoothing
    net0 = fem.UNet(N, N, max_batch=1, channels=16, seed=0)
    net0.set_params(torch.zeros(net0.n_params, dtype=torch.float32, device="cuda"))
    rows = []
    for i, (nu, seed) in enumerate(learn.problem_params(args.learned_eval, 5000)):
        gp = efam.problem(nu, seed)
        x = torch.zeros(gp.n_nodes, dtype=torch.float64, device="cuda")
        if i == 0:  # warm-ups: workspace allocation, code loading
            gp.pcg(x)
            x.zero_()
            gp.fcg(net, x, max_iter=2, **fopts)
            x.zero_()
        a = gp.pcg(x)
        x.zero_()
        b = gp.fcg(net, x, **fopts)
        row = {"nu": round(nu, 3), "pcg_iters": a["iters"], "pcg_s": round(a["seconds"], 4),
               "pcg_relres": a["relres"], "fcg_iters": b["iters"], "fcg_pcg_iters": b["pcg_iters"],
               "fcg_fell_back": b["fell_back"], "fcg_s": round(b["seconds"], 4), "fcg_relres": b["relres"]}
        msg = (f"[bench] learned: nu {nu:.2f} Jacobi-PCG {a['iters']} it {a['seconds']:.3f} s | "
               f"learned FCG {b['iters']}+{b['pcg_iters']} it {b['seconds']:.3f} s")
        if i < args.learned_ablate:
            x.zero_()
            z = gp.fcg(net0, x, stall_iters=1 << 30, max_iter=args.learned_max_iter, **fopts)
            row.update({"cycle_without_network_iters": z["iters"], "cycle_without_network_s": round(z["seconds"], 4),
                        "cycle_without_network_status": z["status"]})
            msg += f" | same cycle without the network {z['iters']} it {z['seconds']:.3f} s"
        if b["fell_back"] >= 0 and i < args.learned_nohandover:
            x.zero_()
            c = gp.fcg(net, x, stall_iters=1 << 30, max_iter=args.learned_max_iter, **fopts)
            row.update({"fcg_no_handover_iters": c["iters"], "fcg_no_handover_s": round(c["seconds"], 4),
                        "fcg_no_handover_status": c["status"], "fcg_no_handover_relres": c["relres"]})
            msg += f" | without hand-over {c['iters']} it {c['seconds']:.3f} s"
        rows.append(row)
        log(msg)
        del gp
    t_pcg = float(np.median([r["pcg_s"] for r in rows]))
    t_fcg = float(np.median([r["fcg_s"] for r in rows]))
    fcg_it = [r["fcg_iters"] + r["fcg_pcg_iters"] for r in rows]
    fcg_only = [r["fcg_s"] / max(r["fcg_iters"], 1) for r in rows if r["fcg_fell_back"] < 0]
    return {
        "workload": f"2D P1 {N}x{N} squares ({(N + 1) ** 2} nodes, {2 * N * N} triangles), nu~U(0,100), "
                    "random-sine f, u=0 on the boundary; held-out problems",
        "network": "U-Net 4 levels, 16-128 channels, BF16 MFMA / FP32 accumulation, 482753 parameters",
        "loss": ("energy: 1 - (y.Ae)^2 / ((y.Ay)(e.Ae)) per pair" if args.learned_loss == "energy"
                 else "relative L2 of the scaled error"),
        "output_smoothing_passes": args.learned_out_smooth,
        "preconditioner": f"FCG(1), two-level cycle: {args.learned_smooth} damped-Jacobi steps (omega 2/3), network "
                          f"correction, {args.learned_smooth} Jacobi steps, {args.learned_cycle.upper()} cycle passes; "
                          "hand-over to Jacobi-PCG (restarted from x0) after 200 iterations without halving ||r||",
        "pairs": n_pairs, "train_problems": len(params), "snapshots_per_problem": len(segs),
        "eval_problems": len(rows),
        "train_steps": len(hist), "train_batch": args.learned_batch, "train_epochs": args.learned_epochs,
        "train_loss_first": round(float(hist[:50].mean()), 4), "train_loss_last": round(float(hist[-200:].mean()), 4),
        "data_s": round(t_data, 2), "train_s": round(t_train, 2),
        "time_to_1e8_jacobi_pcg_s": round(t_pcg, 4), "time_to_1e8_learned_fcg_s": round(t_fcg, 4),
        "speedup_vs_jacobi_pcg": round(t_pcg / t_fcg, 3),
        "iters_jacobi_pcg_mean": round(float(np.mean([r["pcg_iters"] for r in rows])), 1),
        "iters_learned_fcg_mean": round(float(np.mean(fcg_it)), 1),
        "handovers": sum(1 for r in rows if r["fcg_fell_back"] >= 0),
        "max_total_minus_cold_pcg_iters": int(max(t - r["pcg_iters"] for t, r in zip(fcg_it, rows))),
        "fcg_ms_per_iter_median": round(1e3 * float(np.median(fcg_only)), 4) if fcg_only else None,
        "network_gain_iters": (round(float(np.mean([r["cycle_without_network_iters"] / max(r["fcg_iters"], 1)
                                                    for r in rows if "cycle_without_network_iters" in r
                                                    and r["fcg_fell_back"] < 0])), 3)
                               if any("cycle_without_network_iters" in r and r["fcg_fell_back"] < 0 for r in rows)
                               else None),
        "problems": rows,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + ["unet", "cheb", "mg", "learned"], default="c2")
    ap.add_argument("--mg-base", choices=["c2", "c3"], default="c2", help="mg workload: the problem (2D or 3D)")
    ap.add_argument("--mg-coarsest", type=int, default=0,
                    help="mg workload: cells per side of the coarsest grid (0: 16 in 2D, 5 in 3D)")
    ap.add_argument("--mg-smooth", type=int, default=1, help="mg workload: smoothing steps before and after")
    ap.add_argument("--mg-smoother", choices=["jacobi", "chebyshev"], default="jacobi",
                    help="mg workload: damped Jacobi or Chebyshev smoothing")
    ap.add_argument("--mg-cycle", choices=["f64", "f32"], default="f32",
                    help="mg workload: precision of the V-cycle's operator products")
    ap.add_argument("--iter-n", type=int, default=2048, help="cheb workload: squares per side")
    ap.add_argument("--iter-steps", type=int, default=200, help="cheb workload: iterations of the shorter run")
    ap.add_argument("--profile", type=int, default=4, help="time every k-th matvec with HIP events")
    ap.add_argument("--check-every", type=int, default=64)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--vectors", type=int, default=0, help="mixed precision: 0 FP64, 1 FP32 iteration vectors")
    ap.add_argument("--block", type=int, default=0, help="workgroup size of the element pass (0 = default)")
    ap.add_argument("--operator", choices=["stored", "mfree"], default="stored",
                    help="c1-c3: stored local matrices (the workload's storage) or the matrix-free operator")
    ap.add_argument("--residual-calls", type=int, default=20)
    ap.add_argument("--max-iter", type=int, default=200000, help="cap on CG iterations (profiling runs)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="copy a buffer of this size once before the timed steps (HBM counter calibration)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n-problems", type=int, default=256, help="batched workload: number of problems")
    ap.add_argument("--group", type=int, default=0, help="batched: chunks per work item (0 = per-problem schedule)")
    ap.add_argument("--items", type=int, default=4, help="batched: target work items per problem phase")
    ap.add_argument("--batch-chunk", type=int, default=2048, help="batched: elements per chunk")
    ap.add_argument("--inline-segs", type=int, default=64,
                    help="batched: fix-up segments the last chunk item of a phase runs itself")
    ap.add_argument("--adaptive", type=int, default=1,
                    help="batched: regroup work items as problems finish (1) or keep the fixed schedule (0)")
    ap.add_argument("--autotune", action="store_true", help="batched: pick the schedule with the autotuner first")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-FCG vs Jacobi-PCG comparison")
    ap.add_argument("--no-extra", action="store_true",
                    help="c2: skip the C3 / C1 / C4 legs and the all-core and PCG oracle timings")
    ap.add_argument("--learned-n", type=int, default=1024)
    ap.add_argument("--learned-problems", type=int, default=160, help="training problems")
    ap.add_argument("--learned-segments", default="4x25,8x25,12x25,16x25,20x25",
                    help="Jacobi-PCG segment lengths between snapshots, 'length x count' items")
    ap.add_argument("--learned-rounds", type=int, default=10, help="rounds of pair generation + training")
    ap.add_argument("--learned-smooth", type=int, default=2)
    ap.add_argument("--learned-cycle", choices=["f32", "f64"], default="f32")
    ap.add_argument("--learned-max-iter", type=int, default=4000)
    ap.add_argument("--learned-batch", type=int, default=4)
    ap.add_argument("--learned-lr", type=float, default=2e-3)
    ap.add_argument("--learned-eval", type=int, default=32, help="held-out problems")
    ap.add_argument("--learned-loss", choices=["energy", "l2"], default="energy")
    ap.add_argument("--learned-epochs", type=int, default=2, help="passes over each round's pool of pairs")
    ap.add_argument("--learned-out-smooth", type=int, default=2,
                    help="binomial smoothing passes on the network output")
    ap.add_argument("--learned-ablate", type=int, default=4,
                    help="held-out problems also solved with the same cycle and a zero network")
    ap.add_argument("--learned-nohandover", type=int, default=3,
                    help="of the held-out problems that hand over, the first few are also solved without hand-over")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library runs its hot path on a single MI355X "
              "(multi-GPU sharding is a design note, not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1911_03973_amd import fem

    if args.workload == "unet":
        return run_unet(args)
    if args.workload == "cheb":
        return run_iterations(args)
    if args.workload == "mg":
        return run_multigrid(args)
    if args.workload == "learned":
        print(json.dumps({"learned_fcg": learned_fcg(args)}), flush=True)
        return
    if args.workload == "c4":
        print(json.dumps(run_batched(args, WORKLOADS["c4"])), flush=True)
        return
    torch.cuda.set_device(0)
    out = measure_single(args, args.workload, args.steps, args.warmup)
    out["learned_fcg"] = None if args.no_learned else learned_fcg(args)
    if args.workload == "c2" and not args.no_extra:
        out["other_configs"] = other_configs(args)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        w = WORKLOADS[args.workload]
        mesh, _, _ = make_problem(w)
        out["cpu_baseline"] = cpu_baseline(mesh, w, args.cpu_seconds)
        if args.workload == "c2" and not args.no_extra:
            out["cpu_allcores"] = cpu_allcores(mesh, w, args.cpu_seconds / 2)
            del mesh
            c3 = (out.get("other_configs") or {}).get("c3") or {}
            lf = out.get("learned_fcg") or {}
            c5 = next((p["pcg_iters"] for p in lf.get("problems", []) if abs(p["nu"] - 35.547) < 1e-3), None)
            out["oracle_pcg"] = oracle_pcg_times(args.cpu_seconds / 2, c3.get("iters"), c5)
    print(json.dumps(out), flush=True)


def measure_single(args, wname, steps, warmup, residual=True):
    """One single-problem workload: `steps` timed solves after `warmup` ones; the line's fields."""
    import numpy as np
    import torch

    from paper_1911_03973_amd import fem

    w = WORKLOADS[wname]
    mfree = args.operator == "mfree"
    dt = fem.MFREE if mfree else {"f64": fem.F64, "f32x2": fem.F32X2}[w["dtype"]]
    log(f"[bench] workload {wname}: building inputs")
    mesh, nd, f = make_problem(w)
    log(f"[bench] mesh {mesh.n_nodes} nodes {mesh.n_elems} elements; plan")
    t = time.perf_counter()
    # matrix-free in 3D: 512-tet chunks (the coordinate table and slot index
    # of 1536-tet chunks leave one workgroup per CU)
    chunk = args.chunk or (512 if mfree and mesh.dim == 3 else 0)
    plan = fem.Plan.from_mesh(mesh, nd, chunk_elems=chunk)
    t_plan = time.perf_counter() - t
    st = plan.stats()
    K = None if mfree else plan.empty_matrix(dt)
    M = None if mfree else plan.empty_matrix(dt)
    fg = torch.from_numpy(f).cuda()
    b = plan.empty_vector()
    x = plan.empty_vector()
    opts = fem.solve_opts(dtype=dt, nu=w["nu"], rtol=1e-8, check_every=args.check_every, profile=args.profile,
                          max_iter=args.max_iter, vectors=args.vectors, block=args.block)

    def step():
        if not mfree:
            fem.build_local_matrices(plan, dt, K, M, None)
        fem.assemble_rhs(plan, dt, M, fg, b)
        x.zero_()  # Dirichlet data u = 0
        return fem.pcg_solve(plan, opts, K, M, b, x)

    if args.calib_copy_mb:
        nel = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for i in range(warmup):
        info = step()
        log(f"[bench] warmup {i}: {info}")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for i in range(steps):
        infos.append(step())
        log(f"[bench] step {i}: iters {infos[-1]['iters']} relres {infos[-1]['relres']:.3e} "
            f"solve {infos[-1]['seconds']:.3f} s")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / steps
    # the same solve without the per-pass events: its iterations replay as HIP graphs
    if args.profile > 0:
        opts.profile = 0
        t_noev = step()["seconds"]
        opts.profile = args.profile
    else:
        t_noev = float(np.median([i["seconds"] for i in infos]))
    mv_ms = sum(i["matvec_ms"] for i in infos)
    mv_n = sum(i["matvec_samples"] for i in infos)
    nb = mesh.nb
    n_pk = nb + nb * (nb - 1) // 2  # packed symmetric difference form: row sums + upper off-diagonals
    s_a = 0 if mfree else 4 if dt != fem.F64 else 8
    s_v = 4 if (dt not in (fem.F64, fem.MFREE) and args.vectors == 1) else 8
    # one fused CG pass: matrix heads (none when matrix-free) + the connectivity-equivalent
    # index + 9 vector streams (read r, q, x, p, D^-1; write r, x, p, q) + the coordinates
    # when matrix-free
    bytes_mv = mesh.n_elems * (n_pk * s_a + 4 * nb) + mesh.n_nodes * (9 * s_v + (8 * mesh.dim if mfree else 0))
    avg_mv_s = (mv_ms / mv_n) / 1e3 if mv_n else float("nan")
    gbs = bytes_mv / avg_mv_s / 1e9
    ok = all(i["status"] == 0 and i["relres"] <= 1e-8 for i in infos)
    if args.max_iter < 200000:
        log("[bench] capped iterations: a profiling run, not a time-to-1e-8 measurement")
    resid = residual_kernels(fem, plan, mesh, K, M, w["nu"], dt, args.residual_calls) if residual else None
    rec = (measured_traffic() if wname == "c2" and args.vectors == 0 and args.block == 0 and not mfree
           else None)
    traffic = rec["bytes_per_pass"] if rec and rec.get("chunk_elems") == st["chunk_elems"] else None
    out = {
        "metric": METRIC,
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if dt not in (fem.F64, fem.MFREE) else "f64",
        "data": "synthetic",
        "config": {
            "workload": w["name"],
            "n_nodes": mesh.n_nodes,
            "n_elems": mesh.n_elems,
            "chunk_elems": st["chunk_elems"],
            "storage": "matrix-free (K_e, M_e rebuilt per pass, FP64)" if mfree else w["dtype"],
            "block": args.block,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(gbs, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": traffic,
        },
        "elements_per_s": round(mesh.n_elems / avg_mv_s, 1),
        "matvec_us": round(avg_mv_s * 1e6, 2),
        "matvec_bytes": bytes_mv,
        "matvec_samples": mv_n,
        "time_to_1e8_s": round(float(np.median([i["seconds"] for i in infos])), 4),
        "time_to_1e8_s_no_events": round(t_noev, 4),
        "iters": [i["iters"] for i in infos],
        "refreshes": [i["outer"] for i in infos],
        "relres": [i["relres"] for i in infos],
        "converged": ok,
        "plan_seconds": round(t_plan, 3),
        "pass_kind": ("fused CG pass, matrix-free (packed form rebuilt from coordinates), FP64 vectors" if mfree
                      else "fused CG pass, packed difference form (%d values/elem, %s), %s vectors"
                      % (n_pk, "FP32 heads" if dt != fem.F64 else "FP64", "FP32" if s_v == 4 else "FP64")),
        "residual_kernels": resid,
    }
    del K, M, plan
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
