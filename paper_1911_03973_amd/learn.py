"""Training and evaluation of the learned preconditioner.

Problems are the structured 2D ones of the learned workload: the unit square
with N x N cells cut by their (0,0)-(1,1) diagonal, (N+1)^2 nodes numbered
i + j (N+1), homogeneous Dirichlet data on the whole boundary, nu uniform in
[0, 100], f a random sum of sines.  Training pairs come from the plain
solver: Jacobi-PCG is run in restarted segments from x0 = 0 and after every
segment the residual r_k = b - A x_k and the error e_k = u* - x_k (u* the
converged FP64 solution) are recorded.  The network input is r_k scaled to
unit RMS over the interior nodes plus the constant channel nu / 100; the
target is e_k scaled to unit RMS.  Flexible CG only uses the direction of
z = N(r) (its step length is re-optimised every iteration), so the scale of
the error is not learned.

Inside the two-level cycle of fem_fcg_solve (opts.smooth = k > 0) the network
sees the residual left after k damped-Jacobi steps.  snapshot_pairs(smooth=k)
can pass the pairs through the same steps first (z = the k-step Jacobi
approximation of A^-1 r_k, input r_k - A z, target e_k - z); measured on 64^2
and 128^2 grids this does not beat training on the raw pairs, which stay the
default.

All solver and network arithmetic runs in libfem's kernels; torch only moves
the nodal vectors into the image layout of the training batches.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import fem, inputs


def cval_of(nu):
    """Constant second input channel of the network for coefficient nu."""
    return float(nu) / 100.0


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
        mesh = inputs.square_mesh(N)
        nd = inputs.boundary_nodes(mesh, "all")
        plan = fem.Plan.from_mesh(mesh, nd, chunk_elems=chunk_elems)
        K = plan.empty_matrix(dtype)
        M = plan.empty_matrix(dtype)
        fem.build_local_matrices(plan, dtype, K, M, None)
        f = torch.from_numpy(inputs.random_sine(mesh.coords, seed)).cuda()
        b = plan.empty_vector()
        fem.assemble_rhs(plan, dtype, M, f, b)
        mask = torch.zeros(mesh.n_nodes, dtype=torch.uint8)
        mask[torch.from_numpy(nd.astype(np.int64))] = 1
        return cls(N, float(nu), seed, dtype, plan, K, M, b, mask.cuda())

    @property
    def n_nodes(self):
        return (self.N + 1) ** 2

    def dinv(self):
        if getattr(self, "_dinv", None) is None:
            d = self.plan.empty_vector()
            fem.jacobi_diag(self.plan, self.dtype, self.K, self.M, self.nu, d)
            self._dinv = torch.where(self.mask.bool(), torch.zeros_like(d), 1.0 / d)
        return self._dinv

    def presmooth(self, r, steps, omega):
        """(z, r - A z) after `steps` damped-Jacobi steps z += omega D^-1 (r - A z) from z = 0."""
        dinv = self.dinv()
        z = omega * dinv * r
        rz = self.plan.empty_vector()
        fem.element_residual(self.plan, self.dtype, self.K, self.M, self.nu, r, z, rz, mask=True)
        for _ in range(steps - 1):
            z = z + omega * dinv * rz
            fem.element_residual(self.plan, self.dtype, self.K, self.M, self.nu, r, z, rz, mask=True)
        return z, rz

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


def interior_image(v, N):
    """Nodal vector on (N+1)^2 nodes -> N x N image of the interior, unit RMS, zero last row/column."""
    g = v.view(N + 1, N + 1)[1:N, 1:N]
    rms = torch.sqrt(torch.mean(g * g))
    img = torch.zeros((N, N), dtype=torch.float32, device=v.device)
    img[: N - 1, : N - 1] = (g / torch.clamp(rms, min=1e-300)).float()
    return img


def snapshot_pairs(prob, segments, u_star=None, smooth=0, omega=2.0 / 3.0):
    """(inputs [S, N, N, 2], targets [S, N, N]) from restarted Jacobi-PCG segments of the given lengths,
    pre-smoothed by `smooth` damped-Jacobi steps (0: the raw pairs)."""
    N = prob.N
    if u_star is None:
        u_star = torch.zeros(prob.n_nodes, dtype=torch.float64, device="cuda")
        prob.pcg(u_star, rtol=1e-11)
    x = torch.zeros_like(u_star)
    ins, tgs = [], []
    r = prob.plan.empty_vector()
    for k in segments:
        prob.pcg(x, max_iter=int(k), rtol=1e-12)
        prob.residual(x, r)
        e = u_star - x
        if smooth:
            z, r = prob.presmooth(r, smooth, omega)
            e = e - z
        if float(torch.linalg.vector_norm(e)) == 0.0 or float(torch.linalg.vector_norm(r)) == 0.0:
            break
        img = torch.empty((N, N, 2), dtype=torch.float32, device="cuda")
        img[..., 0] = interior_image(r, N)
        img[..., 1] = cval_of(prob.nu)
        ins.append(img)
        tgs.append(interior_image(e, N))
    return torch.stack(ins), torch.stack(tgs)


def problem_params(count, base_seed, nu_max=100.0):
    """(nu, seed) pairs: nu ~ U(0, nu_max), seeds base_seed + 1 + i."""
    rng = np.random.default_rng(base_seed)
    return [(float(rng.uniform(0.0, nu_max)), base_seed + 1 + i) for i in range(count)]


def make_dataset(N, count, base_seed, segments, dtype=fem.F64, smooth=0, omega=2.0 / 3.0):
    ins, tgs = [], []
    for nu, seed in problem_params(count, base_seed):
        prob = GridProblem.make(N, nu, seed, dtype)
        a, t = snapshot_pairs(prob, segments, smooth=smooth, omega=omega)
        ins.append(a)
        tgs.append(t)
        del prob
    return torch.cat(ins), torch.cat(tgs)


def train(net, ins, tgs, steps, batch, lr, seed=0, lr_final=None, log_every=0):
    """Adam on random minibatches; cosine decay from lr to lr_final. Returns the per-step losses."""
    gen = torch.Generator().manual_seed(seed)
    n = ins.shape[0]
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    hist = torch.zeros(steps, dtype=torch.float64, device="cuda")
    lr_final = lr * 0.05 if lr_final is None else lr_final
    for s in range(steps):
        idx = torch.randint(0, n, (batch,), generator=gen).cuda()
        xb = ins.index_select(0, idx).contiguous()
        tb = tgs.index_select(0, idx).contiguous()
        cur = lr_final + 0.5 * (lr - lr_final) * (1.0 + np.cos(np.pi * s / max(steps - 1, 1)))
        net.train_step(xb, tb, cur, loss)
        hist[s] = loss[0]
        if log_every and (s + 1) % log_every == 0:
            print(f"step {s + 1}/{steps} loss {float(loss):.4f}", flush=True)
    return hist.cpu().numpy()
