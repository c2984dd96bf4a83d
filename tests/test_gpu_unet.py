"""U-Net kernels (BF16 MFMA, FP32 accumulation) against the FP64 oracle.

The GPU rounds weights and activations to BF16 (unit roundoff u = 2^-9) and
accumulates in FP32; the oracle runs the same network in float64 on the same
weights rounded to BF16 (the biases stay FP32 on both sides), so what is left
is the rounding of the activations and activation gradients between layers.
With L = 21 rounding stages on the longest path, independent roundings give a
relative error of about sqrt(L) u = 0.9 % in the output; the bounds below
allow 2x (forward 2e-2) and, for the backward pass, which rounds once more per
layer and multiplies two rounded factors per weight gradient, 5e-2 per layer
in the relative L2 norm.  A weight gradient sums over the pixels of its level,
so the rounding errors (and the ReLU masks that flip between BF16 and FP64
activations) average out only when that level has enough pixels: at 16 x 16
the 2 x 2 bottom level gives 14 % on its layers, at 64 x 64 4 %, at 128 x 128
1 %; the gradient checks therefore use images of 64 x 64 and larger (at least
64 pixels per sample at the bottom level).
"""
import numpy as np
import pytest
import torch

from oracle import unet as U

from problems import bf16_params

pytestmark = pytest.mark.gpu

fem = pytest.importorskip("paper_1911_03973_amd.fem")

FWD_TOL = 2e-2
GRAD_TOL = 5e-2


def _bf16_params(net):
    """The network's parameters with the weights rounded to BF16 as the kernels use them."""
    return bf16_params(net)


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _inputs(B, H, W, seed, cval=0.4):
    rng = np.random.default_rng(seed)
    inp = np.zeros((B, H, W, 2), dtype=np.float32)
    # smooth-plus-noise residual-like images
    yy, xx = np.mgrid[0:H, 0:W] / max(H, W)
    for b in range(B):
        inp[b, :, :, 0] = (np.sin(2 * np.pi * (b + 1) * xx) * np.cos(3 * np.pi * yy) + 0.5 * rng.normal(size=(H, W)))
        inp[b, :, :, 1] = cval
    t = rng.normal(size=(B, H, W)).astype(np.float32)
    return inp, t


@pytest.mark.parametrize("H,W,B", [(16, 16, 2), (32, 24, 1), (64, 64, 2)])
def test_forward_matches_oracle(H, W, B):
    net = fem.UNet(H, W, max_batch=B, channels=16, seed=11)
    inp, _ = _inputs(B, H, W, 1)
    y = net.forward(torch.from_numpy(inp).cuda())
    torch.cuda.synchronize()
    ref = U.forward(_bf16_params(net), inp.astype(np.float64), 16)
    assert _rel(y.cpu().numpy(), ref) < FWD_TOL


def test_forward_wide_network():
    net = fem.UNet(16, 16, max_batch=1, channels=32, seed=3)
    inp, _ = _inputs(1, 16, 16, 2)
    y = net.forward(torch.from_numpy(inp).cuda())
    torch.cuda.synchronize()
    ref = U.forward(_bf16_params(net), inp.astype(np.float64), 32)
    assert _rel(y.cpu().numpy(), ref) < FWD_TOL


@pytest.mark.parametrize("H,B", [(64, 2), (128, 1)])
def test_gradients_match_oracle(H, B):
    net = fem.UNet(H, H, max_batch=B, channels=16, seed=5)
    inp, t = _inputs(B, H, H, 3)
    loss, g = net.loss_grad(torch.from_numpy(inp).cuda(), torch.from_numpy(t).cuda())
    torch.cuda.synchronize()
    p = _bf16_params(net)
    val, gref = U.loss_grad(p, inp.astype(np.float64), t.astype(np.float64), 16)
    assert abs(loss.item() - val) <= FWD_TOL * val
    g = g.double().cpu().numpy()
    offs = np.cumsum([0] + [W.size + b.size for W, b in U.unpack(p, 16)])
    worst = 0.0
    for k in range(len(offs) - 1):
        gk, rk = g[offs[k]:offs[k + 1]], gref[offs[k]:offs[k + 1]]
        if np.linalg.norm(rk) == 0:
            continue
        worst = max(worst, _rel(gk, rk))
    assert worst < GRAD_TOL, worst
    cos = float(g @ gref / (np.linalg.norm(g) * np.linalg.norm(gref)))
    assert cos > 0.999


def test_training_step_is_bitwise_reproducible_and_adam_exact():
    H, B = 32, 2
    inp, t = _inputs(B, H, H, 4)
    inp, t = torch.from_numpy(inp).cuda(), torch.from_numpy(t).cuda()
    runs = []
    for _ in range(2):
        net = fem.UNet(H, H, max_batch=B, channels=16, seed=9)
        w0 = net.get_params()
        _, g = net.loss_grad(inp, t)
        lr = 1e-3
        net.train_step(inp, t, lr)
        w1 = net.get_params()
        torch.cuda.synchronize()
        runs.append((w0.cpu(), g.cpu(), w1.cpu()))
        # first Adam step: m^ = g, v^ = g^2  =>  w1 = w0 - lr g / (|g| + eps)
        want = (w0.double() - lr * g.double() / (g.double().abs() + 1e-8)).cpu()
        assert torch.allclose(w1.cpu().double(), want, rtol=0, atol=2e-7 + 1e-6 * float(want.abs().max()))
    assert torch.equal(runs[0][1], runs[1][1])
    assert torch.equal(runs[0][2], runs[1][2])


def test_three_adam_steps_match_oracle_adam():
    """Three training steps with cosine-decayed learning rates against the
    oracle's Adam (bias-corrected moments) fed with the gradients the library
    reports at each step's starting point: the moment recursions and the bias
    corrections of steps 2 and 3, not only the first step's g / |g|."""
    from paper_1911_03973_amd import learn

    H, B = 32, 2
    inp, t = _inputs(B, H, H, 5)
    inp, t = torch.from_numpy(inp).cuda(), torch.from_numpy(t).cuda()
    net = fem.UNet(H, H, max_batch=B, channels=16, seed=12)
    w0 = net.get_params().double().cpu().numpy()
    lrs = [learn._lr(s, 3, 1e-4, 5e-6) for s in range(3)]
    grads = []
    for lr in lrs:
        _, g = net.loss_grad(inp, t)
        grads.append(g.double().cpu().numpy())
        net.train_step(inp, t, lr)
    w3 = net.get_params().double().cpu().numpy()
    want = U.adam(w0, grads, lrs)
    tol = 2e-7 + 1e-6 * np.abs(want).max()
    assert np.abs(w3 - want).max() <= tol
    # a wrong bias correction or moment recursion moves the weights by O(lr)
    wrong = U.adam(w0, grads, [lr * 0.8 for lr in lrs])
    assert np.abs(wrong - want).max() > 10 * tol


def test_training_reduces_loss():
    H, B = 32, 4
    inp, t = _inputs(B, H, H, 6)
    # a learnable target: a smoothed copy of the input
    from scipy.ndimage import uniform_filter

    t = np.stack([uniform_filter(inp[b, :, :, 0], size=5, mode="constant") for b in range(B)]).astype(np.float32)
    inp, t = torch.from_numpy(inp).cuda(), torch.from_numpy(t).cuda()
    net = fem.UNet(H, H, max_batch=B, channels=16, seed=1)
    l0, _ = net.loss_grad(inp, t)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(60):
        net.train_step(inp, t, 2e-3, loss)
    torch.cuda.synchronize()
    assert loss.item() < 0.5 * l0.item()


def test_grid_precondition_matches_oracle():
    N = 32
    net = fem.UNet(N, N, channels=16, seed=2)
    rng = np.random.default_rng(8)
    r = rng.normal(size=(N + 1) ** 2)
    mask = np.zeros((N + 1) ** 2, dtype=np.uint8)
    mask[5 * (N + 1) + 7] = 1
    z = torch.empty((N + 1) ** 2, dtype=torch.float64, device="cuda")
    net.precondition(N, torch.from_numpy(r).cuda(), 0.25, z, mask=torch.from_numpy(mask).cuda())
    torch.cuda.synchronize()
    img = U.grid_input(r, N, 0.25)
    ref = U.grid_output(U.forward(_bf16_params(net), img, 16), N, mask)
    zz = z.cpu().numpy()
    assert zz[5 * (N + 1) + 7] == 0.0
    z2 = zz.reshape(N + 1, N + 1)
    assert np.all(z2[0] == 0) and np.all(z2[N] == 0) and np.all(z2[:, 0] == 0) and np.all(z2[:, N] == 0)
    assert _rel(zz, ref) < FWD_TOL


def test_invalid_arguments():
    with pytest.raises(fem.FemError):
        fem.UNet(12, 16)
    with pytest.raises(fem.FemError):
        fem.UNet(16, 16, channels=24)
    net = fem.UNet(16, 16, max_batch=1)
    inp = torch.zeros((2, 16, 16, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(fem.FemError):
        net.forward(inp)
    r = torch.zeros(17 * 17, dtype=torch.float64, device="cuda")
    z = torch.zeros(33 * 33, dtype=torch.float64, device="cuda")
    with pytest.raises(fem.FemError):
        net.precondition(32, torch.zeros(33 * 33, dtype=torch.float64, device="cuda"), 0.0, z)
    with pytest.raises(fem.FemError):
        net.train_step(torch.zeros((1, 16, 16, 2), dtype=torch.float32, device="cuda"),
                       torch.zeros((1, 16, 16), dtype=torch.float32, device="cuda"), -1.0)
    del r


def test_make_pair_matches_oracle_grid_mapping():
    """fem_unet_make_pair: the input image is the oracle's grid_input of r, the
    target the interior of u - x over its RMS (FP32 rounding apart)."""
    N = 48
    net = fem.UNet(N, N, channels=16, seed=1)
    rng = np.random.default_rng(4)
    n = (N + 1) ** 2
    r, u, x = rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(n)
    inp = torch.empty((N, N, 2), dtype=torch.float32, device="cuda")
    tgt = torch.empty((N, N), dtype=torch.float32, device="cuda")
    net.make_pair(N, torch.from_numpy(r).cuda(), torch.from_numpy(u).cuda(), torch.from_numpy(x).cuda(), 0.3,
                  inp, tgt)
    torch.cuda.synchronize()
    ref = U.grid_input(r, N, 0.3)[0]
    assert np.abs(inp.cpu().numpy() - ref).max() <= 1e-6 * np.abs(ref).max()
    e = (u - x).reshape(N + 1, N + 1)[1:N, 1:N]
    t = np.zeros((N, N))
    t[:N - 1, :N - 1] = e / np.sqrt(np.mean(e ** 2))
    assert np.abs(tgt.cpu().numpy() - t).max() <= 1e-6 * np.abs(t).max()
