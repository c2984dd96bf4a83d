"""Pins of the FP64 U-Net oracle: each layer against a library routine, the
whole backward pass against central finite differences (float64)."""
import numpy as np
import pytest
from scipy import signal

from oracle import unet as U


def _rand_params(c, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    layers = []
    for kind, _, groups, cout in U.architecture(c):
        cin = sum(groups)
        shape = (3, 3, cin, cout) if kind == "conv" else (cin, 2, 2, cout)
        fan = 9 * cin if kind == "conv" else cin
        layers.append((rng.normal(0, scale * np.sqrt(2.0 / fan), shape), rng.normal(0, 0.1, cout)))
    layers.append((rng.normal(0, np.sqrt(1.0 / c), c), rng.normal(0, 0.1, 1)))
    return U.pack(layers)


def test_param_count_and_layout():
    c = 16
    n = U.param_count(c)
    # 0.48M parameters at c = 16
    assert n == 482753  # hand count: 1168+2320+4640+9248+18496+36928+73856+147584+32832+73792+36928+8224+18464+9248+2064+4624+2320+17
    p = np.arange(n, dtype=np.float64)
    L = U.unpack(p, c)
    assert np.array_equal(U.pack(L), p)
    W0, b0 = L[0]
    # W[ky*3+kx][ci][co]: flat index ((ky*3+kx)*8 + ci)*16 + co
    assert W0[1, 2, 3, 4] == ((1 * 3 + 2) * 8 + 3) * 16 + 4
    assert b0[0] == 9 * 8 * 16
    Wu, _ = L[8]
    off = L[8][0].ravel()[0]
    # W[ci][a*2+b][co]
    assert Wu[5, 1, 0, 7] - off == (5 * 4 + 2) * 64 + 7


def test_conv3x3_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 8, 16, 3))
    W = rng.normal(size=(3, 3, 3, 4))
    b = rng.normal(size=4)
    out = U.conv3x3(x, W, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(signal.correlate(x[n, :, :, i], W[:, :, i, o], mode="same", method="direct")
                             for i in range(3))
            np.testing.assert_allclose(out[n, :, :, o], ref, rtol=1e-13, atol=1e-13)


def test_upconv_matches_kron():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 4, 8, 3))
    W = rng.normal(size=(3, 2, 2, 5))
    b = rng.normal(size=5)
    out = U.upconv(x, W, b)
    for n in range(2):
        for o in range(5):
            ref = b[o] + sum(np.kron(x[n, :, :, i], W[i, :, :, o]) for i in range(3))
            np.testing.assert_allclose(out[n, :, :, o], ref, rtol=1e-13, atol=1e-13)


def test_pool_matches_box_filter():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 8, 8, 3))
    out = U.pool(x)
    for n in range(2):
        for i in range(3):
            box = signal.correlate(x[n, :, :, i], np.full((2, 2), 0.25), mode="valid", method="direct")
            np.testing.assert_allclose(out[n, :, :, i], box[::2, ::2], rtol=1e-14, atol=1e-14)


def test_constant_network_output():
    """All weights zero: the output is the output bias everywhere; the loss has a closed form."""
    c = 16
    p = np.zeros(U.param_count(c))
    p[-1] = 0.75
    rng = np.random.default_rng(4)
    inp = rng.normal(size=(2, 8, 8, 2))
    y = U.forward(p, inp, c)
    assert np.all(y == 0.75)
    t = rng.normal(size=(2, 8, 8))
    want = np.mean([np.sum((0.75 - t[i]) ** 2) / np.sum(t[i] ** 2) for i in range(2)])
    assert U.loss(y, t) == pytest.approx(want, rel=1e-14)


def _fd(f, p, idx, h):
    e = np.zeros_like(p)
    e[idx] = h
    return (f(p + e) - f(p - e)) / (2 * h)


def test_backward_matches_finite_differences():
    """dL/dparams and dL/dinput against central differences (float64, relative 1e-6)."""
    c = 16
    rng = np.random.default_rng(5)
    p = _rand_params(c, 6)
    inp = rng.normal(size=(2, 16, 16, 2))
    inp[..., 1] = 0.3
    t = rng.normal(size=(2, 16, 16))
    val, g, gin = U.loss_grad(p, inp, t, c, input_grad=True)
    assert val == pytest.approx(U.loss(U.forward(p, inp, c), t), rel=1e-14)
    f = lambda q: U.loss(U.forward(q, inp, c), t)  # noqa: E731
    # a sample of parameters from every layer: weights and biases
    offs = np.cumsum([0] + [W.size + b.size for W, b in U.unpack(p, c)])
    idx = []
    for k in range(len(offs) - 1):
        lo, hi = offs[k], offs[k + 1]
        idx += list(rng.integers(lo, hi, size=3)) + [hi - 1]
    worst = 0.0
    for i in idx:
        fd = _fd(f, p, i, 1e-6)
        worst = max(worst, abs(fd - g[i]) / max(abs(fd), 1e-3 * np.abs(g).max()))
    assert worst < 1e-6, worst
    fin = lambda q: U.loss(U.forward(p, q, c), t)  # noqa: E731
    for _ in range(6):
        i = tuple(int(v) for v in (rng.integers(2), rng.integers(16), rng.integers(16), 0))
        e = np.zeros_like(inp)
        e[i] = 1e-6
        fd = (fin(inp + e) - fin(inp - e)) / 2e-6
        assert abs(fd - gin[i]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gin).max())


def test_padding_channels_have_zero_gradient():
    c = 16
    rng = np.random.default_rng(7)
    p = _rand_params(c, 8)
    inp = rng.normal(size=(1, 8, 8, 2))
    t = rng.normal(size=(1, 8, 8))
    _, g = U.loss_grad(p, inp, t, c)
    W0g = g[: 9 * 8 * 16].reshape(9, 8, 16)
    assert np.all(W0g[:, 2:, :] == 0.0)


def test_grid_mapping_round_trip():
    N = 8
    rng = np.random.default_rng(9)
    r = rng.normal(size=(N + 1) ** 2)
    img = U.grid_input(r, N, 0.5)
    r2 = r.reshape(N + 1, N + 1)
    inner = r2[1:N, 1:N]
    np.testing.assert_allclose(img[0, :N - 1, :N - 1, 0] * np.sqrt(np.mean(inner ** 2)), inner, rtol=1e-14)
    assert np.all(img[0, N - 1, :, 0] == 0) and np.all(img[0, :, N - 1, 0] == 0)
    assert np.all(img[0, :, :, 1] == 0.5)
    z = U.grid_output(img[..., 0], N)
    z2 = z.reshape(N + 1, N + 1)
    assert np.all(z2[0] == 0) and np.all(z2[N] == 0) and np.all(z2[:, 0] == 0) and np.all(z2[:, N] == 0)
    np.testing.assert_allclose(z2[1:N, 1:N], img[0, :N - 1, :N - 1, 0])
