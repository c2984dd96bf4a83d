"""Training and evaluation of the learned preconditioner.

Problems are the structured 2D ones of the learned workload: the unit square
with N x N cells cut by their (0,0)-(1,1) diagonal, (N+1)^2 nodes numbered
i + j (N+1), homogeneous Dirichlet data on the whole boundary, nu uniform in
[0, 100], f a random sum of sines.  One GridFamily holds the mesh's plan and
its K_e, M_e, built once: the problems differ only in nu (an argument of
every solver call) and in b = sum_e C_e^T M_e f_e.

Training pairs come from the plain solver: Jacobi-PCG is run in restarted
segments from x0 = 0 and after every segment the residual r_k = b - A x_k
and the error e_k = u* - x_k are recorded, u* the solution from multigrid-
preconditioned FCG to a relative residual of 1e-11 (the nested meshes
N, N/2, ..., 16 of the family).  fem_unet_make_pair turns (r_k, u*, x_k) into
the network input -- r_k scaled to unit RMS over the interior nodes plus the
constant channel nu / 100, exactly as the preconditioner feeds the network --
and the target, e_k scaled to unit RMS.  Flexible CG only uses the direction
of z = N(r) (its step length is re-optimised every iteration), so the scale
of the error is not learned.

The loss is either the relative L2 error of the scaled error image or its
energy-norm counterpart: the fraction of ||e||_A^2 left after the
energy-optimal step along the network output, which is the step the
preconditioner's cycle takes (fem_unet_set_loss).

The training set is streamed: the problems are taken in rounds; each round's
pairs fill a pool on the device and the network takes one Adam step per
`batch` pairs of the pool, in a random order without repetition, so every
pair is used once.  The learning rate decays along a cosine over all steps.

The solver, pair and network arithmetic runs in libfem's kernels; this module
orders the calls, draws the problem parameters and minibatch orders, and
moves images between the pool and the batch buffers.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import torch

from . import fem, inputs


NU_PER_CVAL = 100.0  # nu = NU_PER_CVAL * the network's constant input channel


def cval_of(nu):
    """Constant second input channel of the network for coefficient nu."""
    return float(nu) / NU_PER_CVAL


def use_energy_loss(net, out_smooth=2):
    """Trains `net` on the energy loss of the learned problems' operator (the
    constant channel carries nu / NU_PER_CVAL), with `out_smooth` binomial
    passes on its output: they damp the BF16 rounding noise whose energy norm
    would otherwise swamp that of the smooth errors."""
    net.set_loss(fem.LOSS_ENERGY, NU_PER_CVAL)
    net.set_output_smoothing(out_smooth)


@dataclasses.dataclass
class GridProblem:
    N: int
    nu: float
    seed: int
    dtype: int
    plan: object
    K: torch.Tensor
    M: torch.Tensor
    b: torch.Tensor
    mask: torch.Tensor

    @classmethod
    def make(cls, N, nu, seed, dtype=fem.F64, chunk_elems=0):
        return GridFamily(N, dtype, chunk_elems=chunk_elems).problem(nu, seed)

    @property
    def n_nodes(self):
        return (self.N + 1) ** 2

    def residual(self, x, r=None):
        r = self.plan.empty_vector() if r is None else r
        fem.element_residual(self.plan, self.dtype, self.K, self.M, self.nu, self.b, x, r, mask=True)
        return r

    def pcg(self, x, rtol=1e-8, max_iter=100000, dtype=None, **kw):
        o = fem.solve_opts(dtype=self.dtype if dtype is None else dtype, nu=self.nu, rtol=rtol, max_iter=max_iter,
                           **kw)
        return fem.pcg_solve(self.plan, o, self.K, self.M, self.b, x)

    def fcg(self, net, x, rtol=1e-8, max_iter=100000, **kw):
        o = fem.fcg_opts(dtype=self.dtype, nu=self.nu, rtol=rtol, max_iter=max_iter, grid_n=self.N,
                         cval=cval_of(self.nu), **kw)
        return fem.fcg_solve(self.plan, o, net, self.K, self.M, self.b, x)


class GridFamily:
    """Plan, K_e and M_e of the N x N grid (built once), the Dirichlet mask, and
    with mg=True the nested grids N, N/2, ..., `coarsest` for reference solves."""

    def __init__(self, N, dtype=fem.F64, chunk_elems=0, mg=False, coarsest=16):
        self.N, self.dtype = int(N), dtype
        mesh = inputs.square_mesh(self.N)
        self.coords = mesh.coords
        nd = inputs.boundary_nodes(mesh, "all")
        self.plan = fem.Plan.from_mesh(mesh, nd, chunk_elems=chunk_elems)
        self.K = self.plan.empty_matrix(dtype)
        self.M = self.plan.empty_matrix(dtype)
        fem.build_local_matrices(self.plan, dtype, self.K, self.M, None)
        mask = torch.zeros(mesh.n_nodes, dtype=torch.uint8)
        mask[torch.from_numpy(nd.astype(np.int64))] = 1
        self.mask = mask.cuda()
        self.levels = None
        if mg:
            self.levels = [self.N]
            while self.levels[-1] // 2 >= coarsest and self.levels[-1] % 2 == 0:
                self.levels.append(self.levels[-1] // 2)
            self.mg_plans, self.mg_K, self.mg_M = [self.plan], [self.K], [self.M]
            for n in self.levels[1:]:
                m = inputs.square_mesh(n)
                p = fem.Plan.from_mesh(m, inputs.boundary_nodes(m, "all"))
                k, mm = p.empty_matrix(dtype), p.empty_matrix(dtype)
                fem.build_local_matrices(p, dtype, k, mm, None)
                self.mg_plans.append(p)
                self.mg_K.append(k)
                self.mg_M.append(mm)

    @property
    def n_nodes(self):
        return (self.N + 1) ** 2

    def problem(self, nu, seed):
        f = torch.from_numpy(inputs.random_sine(self.coords, seed)).cuda()
        b = self.plan.empty_vector()
        fem.assemble_rhs(self.plan, self.dtype, self.M, f, b)
        return GridProblem(self.N, float(nu), seed, self.dtype, self.plan, self.K, self.M, b, self.mask)

    def reference(self, prob, rtol=1e-11):
        """u* of a problem of this family by multigrid-preconditioned FCG."""
        if self.levels is None:
            raise ValueError("family built without multigrid levels")
        Ms = self.mg_M if prob.nu != 0.0 else None
        mg = fem.MG(self.mg_plans, self.levels, self.dtype, self.mg_K, Ms, prob.nu)
        u = torch.zeros(self.n_nodes, dtype=torch.float64, device="cuda")
        info = mg.solve(fem.mg_opts(rtol=rtol, smooth=1), prob.b, u)
        mg.destroy()
        if info["status"] != 0:
            raise RuntimeError(f"reference solve failed: {info}")
        return u


def snapshot_pairs(prob, segments, net, u_star, ins, tgs, start=0):
    """Restarted Jacobi-PCG segments of the given lengths from x0 = 0; after each
    one the pair of (r_k, e_k = u* - x_k) goes into ins[start + j], tgs[start + j]
    (float32 [.., N, N, 2] and [.., N, N]) through the library.  Returns the count."""
    x = torch.zeros(prob.n_nodes, dtype=torch.float64, device="cuda")
    r = prob.plan.empty_vector()
    for j, k in enumerate(segments):
        prob.pcg(x, max_iter=int(k), rtol=1e-14)
        prob.residual(x, r)
        net.make_pair(prob.N, r, u_star, x, cval_of(prob.nu), ins[start + j], tgs[start + j])
    return len(segments)


def problem_params(count, base_seed, nu_max=100.0):
    """(nu, seed) pairs: nu ~ U(0, nu_max), seeds base_seed + 1 + i."""
    rng = np.random.default_rng(base_seed)
    return [(float(rng.uniform(0.0, nu_max)), base_seed + 1 + i) for i in range(count)]


def make_dataset(fam, net, count, base_seed, segments):
    """All pairs of `count` problems at once (small grids): (inputs, targets)."""
    S = len(segments)
    ins = torch.empty((count * S, fam.N, fam.N, 2), dtype=torch.float32, device="cuda")
    tgs = torch.empty((count * S, fam.N, fam.N), dtype=torch.float32, device="cuda")
    for i, (nu, seed) in enumerate(problem_params(count, base_seed)):
        prob = fam.problem(nu, seed)
        snapshot_pairs(prob, segments, net, fam.reference(prob), ins, tgs, i * S)
    return ins, tgs


def _lr(s, steps, lr, lr_final):
    return lr_final + 0.5 * (lr - lr_final) * (1.0 + np.cos(np.pi * s / max(steps - 1, 1)))


def train(net, ins, tgs, steps, batch, lr, seed=0, lr_final=None, log_every=0):
    """Adam on random minibatches of a fixed set; cosine decay from lr to lr_final.
    Returns the per-step losses."""
    gen = torch.Generator().manual_seed(seed)
    n = ins.shape[0]
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    hist = torch.zeros(steps, dtype=torch.float64, device="cuda")
    lr_final = lr * 0.05 if lr_final is None else lr_final
    for s in range(steps):
        idx = torch.randint(0, n, (batch,), generator=gen).cuda()
        xb = ins.index_select(0, idx).contiguous()
        tb = tgs.index_select(0, idx).contiguous()
        net.train_step(xb, tb, _lr(s, steps, lr, lr_final), loss)
        hist[s] = loss[0]
        if log_every and (s + 1) % log_every == 0:
            print(f"step {s + 1}/{steps} loss {float(loss):.4f}", flush=True)
    return hist.cpu().numpy()


def train_streaming(fam, net, params, segments, batch, lr, rounds, seed=0, lr_final=None, log=None, epochs=1):
    """Generates the pairs of the (nu, seed) problems round by round and trains on
    each round's pool `epochs` times, each time in a fresh random order (one
    Adam step per `batch` pairs; a last partial batch is dropped).  Returns
    (losses, pairs, data seconds, training seconds)."""
    S = len(segments)
    per_round = (len(params) + rounds - 1) // rounds
    pool = per_round * S
    ins = torch.empty((pool, fam.N, fam.N, 2), dtype=torch.float32, device="cuda")
    tgs = torch.empty((pool, fam.N, fam.N), dtype=torch.float32, device="cuda")
    xb = torch.empty((batch, fam.N, fam.N, 2), dtype=torch.float32, device="cuda")
    tb = torch.empty((batch, fam.N, fam.N), dtype=torch.float32, device="cuda")
    total_steps = epochs * sum((min(per_round, len(params) - i) * S) // batch for i in range(0, len(params), per_round))
    lr_final = lr * 0.05 if lr_final is None else lr_final
    gen = torch.Generator().manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    hist = torch.zeros(max(total_steps, 1), dtype=torch.float64, device="cuda")
    step, pairs, t_data, t_train = 0, 0, 0.0, 0.0
    for r0 in range(0, len(params), per_round):
        chunk = params[r0:r0 + per_round]
        torch.cuda.synchronize()
        t = time.perf_counter()
        n = 0
        for nu, sd in chunk:
            prob = fam.problem(nu, sd)
            n += snapshot_pairs(prob, segments, net, fam.reference(prob), ins, tgs, n)
        torch.cuda.synchronize()
        t_data += time.perf_counter() - t
        pairs += n
        t = time.perf_counter()
        for _ in range(epochs):
            order = torch.randperm(n, generator=gen).cuda()
            for k in range(n // batch):
                idx = order[k * batch:(k + 1) * batch]
                torch.index_select(ins[:n], 0, idx, out=xb)
                torch.index_select(tgs[:n], 0, idx, out=tb)
                net.train_step(xb, tb, _lr(step, total_steps, lr, lr_final), loss)
                hist[step] = loss[0]
                step += 1
        torch.cuda.synchronize()
        t_train += time.perf_counter() - t
        if log:
            log(f"[learn] round {r0 // per_round + 1}: {pairs} pairs, {step} steps, loss {float(loss):.4f}")
    return hist[:step].cpu().numpy(), pairs, t_data, t_train
