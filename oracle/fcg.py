"""Flexible conjugate gradients and the two-level network cycle, in FP64
(test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of the
benchmark may import this module; it shares no code with the GPU library.
Every operator product is the oracle's element residual (Section 2, eq. (4),
Algorithm 1) with b = 0, so A p = -residual(0, p), with the Dirichlet rows
masked as in the problem statement of Section 1.

FCG(1) -- flexible CG truncated to one previous direction (Notay, SIAM J. Sci.
Comput. 22 (2000), the method with m_max = 1):
    z_k = B(r_k)
    p_0 = z_0,   p_k = z_k - (z_k . q_{k-1}) / (p_{k-1} . q_{k-1}) p_{k-1}
    q_k = A p_k,  alpha_k = (p_k . r_k) / (p_k . q_k)
    x_{k+1} = x_k + alpha_k p_k,  r_{k+1} = r_k - alpha_k q_k
With a fixed symmetric positive definite B this is the preconditioned CG
method in exact arithmetic, so its iterates equal those of ``oracle.pcg``.

The two-level cycle B(r) with a network N as the coarse correction:
    z = 0;  k times  z <- z + omega D^-1 (r - A z)          (pre-smoothing)
    r_z = r - A z;  n = N(r_z)
    s = (n . r_z) / (n . A n)   (0 if n . A n <= 0 or not finite)
    z <- z + s n                                             (coarse correction)
    k times  z <- z + omega D^-1 (r - A z)                   (post-smoothing)
s is the step that minimises the A-norm of the error A^-1 r - z - s n left by
the correction.  N is the FP64 U-Net of ``oracle.unet`` on the structured grid
(``grid_input`` / ``grid_output``): the learned preconditioner is not in the
paper, which motivates preconditioning in Section 3 and names it in its
Outlooks; the cycle is this project's reading of how the network enters.
"""
from __future__ import annotations

import numpy as np

from . import jacobi_diag, residual
from . import unet as _unet


class Operator:
    """A p = (K + nu M) p with the Dirichlet rows (mask != 0) set to zero."""

    def __init__(self, n_nodes, elems, K, M, nu, mask):
        self.n = int(n_nodes)
        self.elems = elems
        self.K, self.M, self.nu = K, M, float(nu)
        self.mask = np.asarray(mask, dtype=np.uint8)
        self.free = self.mask == 0

    def apply(self, p):
        return -residual(self.n, self.elems, self.K, self.M, self.nu, None, p, self.mask)

    def residual(self, b, x):
        return residual(self.n, self.elems, self.K, self.M, self.nu, b, x, self.mask)

    def dinv(self):
        """D^-1 on free nodes, 0 on Dirichlet nodes."""
        d = jacobi_diag(self.n, self.elems, self.K, self.M, self.nu)
        out = np.zeros(self.n)
        out[self.free] = 1.0 / d[self.free]
        return out


def jacobi(op):
    """The preconditioner z = D^-1 r (0 on Dirichlet nodes)."""
    dinv = op.dinv()
    return lambda r: dinv * r


def damped_jacobi_steps(op, r, z, steps, omega, dinv=None):
    """`steps` updates z <- z + omega D^-1 (r - A z)."""
    dinv = op.dinv() if dinv is None else dinv
    z = np.array(z, dtype=np.float64)
    for _ in range(steps):
        z = z + omega * dinv * (r - op.apply(z))
    return z


def two_level_cycle(op, r, coarse, smooth, omega=2.0 / 3.0, dinv=None, detail=False):
    """z = B(r) of the two-level cycle above; with detail=True also (s, n, z before the correction)."""
    dinv = op.dinv() if dinv is None else dinv
    z = damped_jacobi_steps(op, r, np.zeros(op.n), smooth, omega, dinv)
    rz = r - op.apply(z)
    n = np.asarray(coarse(rz), dtype=np.float64)
    An = op.apply(n)
    num, den = float(n @ rz), float(n @ An)
    s = num / den if den > 0.0 and np.isfinite(num / den) else 0.0
    z_pre = z
    z = z + s * n
    z = damped_jacobi_steps(op, r, z, smooth, omega, dinv)
    return (z, s, n, z_pre) if detail else z


def network_coarse(params, N, cval, mask=None, channels=16):
    """n = N(r) on the (N+1)^2 grid: the interior residual scaled to unit RMS in,
    the network's output image on the interior nodes out (0 on the boundary and
    on masked nodes)."""

    def apply(r):
        y = _unet.forward(params, _unet.grid_input(r, N, cval), channels)
        return _unet.grid_output(y, N, mask)

    return apply


def fcg(op, b, x0, precond, iters=None, rtol=1e-8, max_iter=10000, history=False):
    """FCG(1) from x0; stops after `iters` iterations if given, else at ||r|| <= rtol ||r0||
    (recursive residual).  Returns x, or (x, [x_1, x_2, ...]) with history=True."""
    x = np.array(x0, dtype=np.float64)
    r = op.residual(b, x)
    r0 = float(np.linalg.norm(r))
    hist = []
    p_prev = q_prev = None
    pq_prev = 1.0
    limit = iters if iters is not None else max_iter
    for _ in range(limit):
        if iters is None and np.linalg.norm(r) <= rtol * r0:
            break
        z = np.asarray(precond(r), dtype=np.float64)
        if p_prev is None:
            p = z.copy()
        else:
            p = z - (float(z @ q_prev) / pq_prev) * p_prev
        q = op.apply(p)
        pq = float(p @ q)
        if not pq > 0.0:
            raise FloatingPointError("p.q <= 0 in FCG")
        alpha = float(p @ r) / pq
        x = x + alpha * p
        r = r - alpha * q
        p_prev, q_prev, pq_prev = p, q, pq
        if history:
            hist.append(x.copy())
    return (x, hist) if history else x
