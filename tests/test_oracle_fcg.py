"""Pins of the oracle's flexible CG and two-level cycle (oracle/fcg.py) and of
its Adam step (oracle/unet.py), against what the mathematics fixes: FCG(1)
with a fixed SPD preconditioner is PCG; the cycle without a coarse correction
is 2k damped-Jacobi steps, i.e. the polynomial (I - (I - w D^-1 A)^2k) A^-1 in
closed form; its step s minimises the A-norm error of the correction; an exact
coarse solve makes the cycle the exact inverse; Adam's bias correction makes
a constant gradient move every weight by lr_t g / (|g| + eps)."""
import numpy as np
import pytest

import oracle
import oracle.fcg as ofcg
from oracle import unet as U
from paper_1911_03973_amd import inputs


def _problem(mesh, nu, which="all", seed=4):
    n = mesh.n_nodes
    K, M, _ = oracle.local_matrices(mesh.coords, mesh.elems)
    nd = inputs.boundary_nodes(mesh, which)
    mask = oracle.mask_from_nodes(n, nd)
    f = inputs.random_sine(mesh.coords, seed) if mesh.dim == 2 else np.ones(n)
    b = oracle.rhs(n, mesh.elems, M, f)
    op = ofcg.Operator(n, mesh.elems, K, M, nu, mask)
    return op, b, K, M, mask


def _dense(op):
    """The free-node block of A, column by column from the operator."""
    free = np.flatnonzero(op.free)
    A = np.zeros((len(free), len(free)))
    for k, j in enumerate(free):
        e = np.zeros(op.n)
        e[j] = 1.0
        A[:, k] = op.apply(e)[free]
    return A, free


@pytest.mark.parametrize("dim", [2, 3])
def test_fcg_with_jacobi_is_pcg(dim):
    mesh = inputs.square_mesh(12, jitter=0.2, seed=2) if dim == 2 else inputs.cube_mesh(5, jitter=0.15, seed=2)
    op, b, K, M, mask = _problem(mesh, 1.5, "x2=0" if dim == 2 else "all")
    x0 = np.zeros(op.n)
    _, hist = ofcg.fcg(op, b, x0, ofcg.jacobi(op), iters=10, history=True)
    scale = None
    for k in range(1, 11):
        xk, _ = oracle.pcg(op.n, mesh.elems, K, M, 1.5, b, mask, x0, rtol=1e-300, max_iter=k,
                           raise_on_noconv=False)
        scale = np.abs(xk).max() if scale is None else max(scale, np.abs(xk).max())
        assert np.abs(hist[k - 1] - xk).max() <= 1e-10 * scale, k
    # and to convergence: same solution as a dense solve
    A, free = _dense(op)
    x = ofcg.fcg(op, b, x0, ofcg.jacobi(op), rtol=1e-12)
    u = np.linalg.solve(A, b[free])
    assert np.abs(x[free] - u).max() <= 1e-9 * np.abs(u).max()


@pytest.mark.parametrize("k", [1, 2, 4])
def test_cycle_without_coarse_correction_is_2k_jacobi_steps(k):
    mesh = inputs.square_mesh(8, jitter=0.2, seed=5)
    op, _, _, _, _ = _problem(mesh, 3.0)
    rng = np.random.default_rng(11)
    r = rng.standard_normal(op.n) * op.free
    omega = 2.0 / 3.0
    z, s, n, _ = ofcg.two_level_cycle(op, r, lambda v: np.zeros_like(v), k, omega, detail=True)
    assert s == 0.0 and not n.any()
    # closed form on the free nodes: z = (I - (I - w D^-1 A)^(2k)) A^-1 r
    A, free = _dense(op)
    Dinv = np.diag(1.0 / np.diag(A))
    E = np.eye(len(free)) - omega * Dinv @ A
    want = (np.eye(len(free)) - np.linalg.matrix_power(E, 2 * k)) @ np.linalg.solve(A, r[free])
    assert np.abs(z[free] - want).max() <= 1e-12 * np.abs(want).max()
    assert not z[~op.free].any()


def test_cycle_step_minimises_the_energy_error():
    """On the 9 x 9 grid with a random-weight network: s from the cycle is the
    minimiser of ||A^-1 r - z_pre - s n||_A found by a dense scan."""
    N = 8
    mesh = inputs.square_mesh(N)
    op, _, _, _, mask = _problem(mesh, 20.0)
    rng = np.random.default_rng(3)
    params = rng.standard_normal(U.param_count(16)) * 0.2
    coarse = ofcg.network_coarse(params, N, 0.2, mask)
    r = rng.standard_normal(op.n) * op.free
    z, s, n, z_pre = ofcg.two_level_cycle(op, r, coarse, 2, detail=True)
    assert n.any() and s != 0.0
    A, free = _dense(op)
    e = np.linalg.solve(A, r[free]) - z_pre[free]
    nf = n[free]

    def energy(t):
        d = e - t * nf
        return d @ A @ d

    grid = s + np.linspace(-1.0, 1.0, 2001) * abs(s)
    vals = np.array([energy(t) for t in grid])
    t_best = grid[np.argmin(vals)]
    assert abs(t_best - s) <= 1.5e-3 * abs(s)
    assert energy(s) <= vals.min() * (1 + 1e-12)


def test_exact_coarse_solve_makes_the_cycle_the_inverse():
    mesh = inputs.square_mesh(8, jitter=0.1, seed=6)
    op, b, _, _, _ = _problem(mesh, 0.5)
    A, free = _dense(op)

    def exact(v):
        out = np.zeros(op.n)
        out[free] = np.linalg.solve(A, v[free])
        return out

    rng = np.random.default_rng(8)
    r = rng.standard_normal(op.n) * op.free
    z, s, _, _ = ofcg.two_level_cycle(op, r, exact, 3, detail=True)
    assert abs(s - 1.0) <= 1e-12
    np.testing.assert_allclose(z[free], np.linalg.solve(A, r[free]), rtol=0, atol=1e-12 * np.abs(z).max())
    # FCG with it converges in one iteration
    x = ofcg.fcg(op, b, np.zeros(op.n), lambda v: ofcg.two_level_cycle(op, v, exact, 3), iters=1)
    assert np.linalg.norm(op.residual(b, x)) <= 1e-12 * np.linalg.norm(b)


def test_fcg_converges_with_the_network_cycle():
    """A variable (nonlinear) preconditioner: FCG(1) with the cycle around a
    random-weight network still reaches the tolerance, no slower than Jacobi-PCG."""
    N = 16
    mesh = inputs.square_mesh(N)
    op, b, K, M, mask = _problem(mesh, 10.0)
    rng = np.random.default_rng(9)
    params = rng.standard_normal(U.param_count(16)) * 0.1
    coarse = ofcg.network_coarse(params, N, 0.1, mask)
    x = ofcg.fcg(op, b, np.zeros(op.n), lambda v: ofcg.two_level_cycle(op, v, coarse, 2), rtol=1e-8)
    assert np.linalg.norm(op.residual(b, x)) <= 1e-8 * np.linalg.norm(b) * 1.0001
    _, info = oracle.pcg(op.n, mesh.elems, K, M, 10.0, b, mask, np.zeros(op.n), rtol=1e-8)
    assert info["relres"] <= 1e-8


# --------------------------------------------------------------------------
# Adam (Kingma & Ba, Algorithm 1)
# --------------------------------------------------------------------------

def test_adam_constant_gradient_moves_by_lr_times_sign():
    """With a constant gradient the bias-corrected moments are exactly g and g^2,
    so step t moves every weight by -lr_t g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    theta0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lrs = [1e-3, 5e-4, 2e-4, 1e-4]
    hist = U.adam(theta0, [g] * 4, lrs, history=True)
    prev = theta0
    for th, lr in zip(hist, lrs):
        np.testing.assert_allclose(th - prev, -lr * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15)
        prev = th


def test_adam_sign_flip_second_step():
    """g_1 = a, g_2 = -a: m^_2 = -(1 - b1) a / (1 + b1) and v^_2 = a^2, so the
    second step moves by +lr (1 - b1) / (1 + b1) sign(a) (up to eps)."""
    a = np.array([0.5, -2.0, 3.0])
    th = U.adam(np.zeros(3), [a, -a], [1.0, 1.0], history=True)
    step2 = th[1] - th[0]
    np.testing.assert_allclose(step2, (0.1 / 1.9) * np.sign(a) * np.abs(a) / (np.abs(a) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(th[0], -np.sign(a) * np.abs(a) / (np.abs(a) + 1e-8), rtol=1e-12)
