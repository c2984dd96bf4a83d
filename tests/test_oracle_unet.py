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


# ---------------------------------------------------------------------------
# Energy loss
# ---------------------------------------------------------------------------

def test_unit_square_grid_is_the_learned_workload_mesh():
    from paper_1911_03973_amd import inputs

    n = 6
    coords, elems, bnd = U.unit_square_grid(n)
    m = inputs.square_mesh(n)
    np.testing.assert_allclose(coords, m.coords, rtol=0, atol=1e-15)
    as_set = lambda E: {tuple(sorted(int(v) for v in e)) for e in E}  # noqa: E731
    assert as_set(elems) == as_set(m.elems)
    np.testing.assert_array_equal(np.flatnonzero(bnd), np.sort(inputs.boundary_nodes(m, "all")))


@pytest.mark.parametrize("n,nu", [(8, 0.0), (8, 37.0), (12, 100.0)])
def test_grid_operator_is_the_p1_stencil(n, nu):
    """On the diagonal-cut grid the assembled P1 stiffness is the 5-point
    Laplacian (the diagonal edges have cotangent weight 0) and the mass matrix
    has h^2/2 on the diagonal and h^2/12 for each of the six edge neighbours."""
    rng = np.random.default_rng(1)
    v = rng.normal(size=(n, n))
    v[n - 1, :] = 0.0
    v[:, n - 1] = 0.0
    h = 1.0 / n
    pad = np.zeros((n + 2, n + 2))
    pad[1:n, 1:n] = v[: n - 1, : n - 1]
    want = np.zeros((n, n))
    for y in range(n - 1):
        for x in range(n - 1):
            P = lambda dy, dx: pad[y + 1 + dy, x + 1 + dx]  # noqa: E731
            axis = P(0, 1) + P(0, -1) + P(1, 0) + P(-1, 0)
            want[y, x] = 4 * P(0, 0) - axis + nu * h * h * (P(0, 0) / 2 + (axis + P(1, 1) + P(-1, -1)) / 12)
    np.testing.assert_allclose(U.grid_operator(n, nu)(v), want, rtol=1e-13, atol=1e-13)


def test_energy_loss_is_the_energy_left_after_the_optimal_step():
    """Each term equals min_s ||s y - t||_A^2 / ||t||_A^2 found by a scalar
    minimiser; the loss ignores the scale and sign of y, is 0 for y = t and 1
    (zero gradient) for a zero output."""
    from scipy.optimize import minimize_scalar

    n = 8
    rng = np.random.default_rng(2)
    y = rng.normal(size=(2, n, n))
    t = rng.normal(size=(2, n, n)) + 0.5 * y
    nus = [3.0, 60.0]
    val, _ = U.energy_loss(y, t, nus)
    inner = np.zeros((n, n))
    inner[: n - 1, : n - 1] = 1
    terms = []
    for k in range(2):
        A = U.grid_operator(n, nus[k])
        yk, tk = y[k] * inner, t[k] * inner
        e = lambda s: float(np.sum((s * yk - tk) * A(s * yk - tk)))  # noqa: E731
        best = minimize_scalar(e, bracket=(-10, 10), tol=1e-12).fun
        terms.append(best / float(np.sum(tk * A(tk))))
    assert val == pytest.approx(np.mean(terms), rel=1e-8)
    assert 0.0 <= val <= 1.0
    assert U.energy_loss(-3.7 * y, t, nus)[0] == pytest.approx(val, rel=1e-12)
    assert U.energy_loss(y, 0.2 * t, nus)[0] == pytest.approx(val, rel=1e-12)
    assert U.energy_loss(t, t, nus)[0] == pytest.approx(0.0, abs=1e-14)
    v0, g0 = U.energy_loss(np.zeros_like(y), t, nus)
    assert v0 == 1.0 and np.all(g0 == 0.0)
    # values on the last row and column do not enter
    y2 = y.copy()
    y2[:, n - 1, :] = 5.0
    y2[:, :, n - 1] = -5.0
    assert U.energy_loss(y2, t, nus)[0] == pytest.approx(val, rel=1e-14)


def test_energy_backward_matches_finite_differences():
    """dL/dy and dL/dparams of the energy loss against central differences (relative 1e-6)."""
    c = 16
    rng = np.random.default_rng(11)
    p = _rand_params(c, 12)
    inp = rng.normal(size=(2, 16, 16, 2))
    inp[0, ..., 1] = 0.3
    inp[1, ..., 1] = 0.8
    t = rng.normal(size=(2, 16, 16))
    nus = [30.0, 80.0]
    y = U.forward(p, inp, c)
    _, gy = U.energy_loss(y, t, nus)
    for _ in range(8):
        i = tuple(int(v) for v in (rng.integers(2), rng.integers(16), rng.integers(16)))
        e = np.zeros_like(y)
        e[i] = 1e-6
        fd = (U.energy_loss(y + e, t, nus)[0] - U.energy_loss(y - e, t, nus)[0]) / 2e-6
        assert abs(fd - gy[i]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gy).max())
    val, g = U.loss_grad(p, inp, t, c, kind="energy", nu_scale=100.0)
    f = lambda q: U.energy_loss(U.forward(q, inp, c), t, nus)[0]  # noqa: E731
    assert val == pytest.approx(f(p), rel=1e-14)
    offs = np.cumsum([0] + [W.size + b.size for W, b in U.unpack(p, c)])
    worst = 0.0
    for k in range(len(offs) - 1):
        for i in list(rng.integers(offs[k], offs[k + 1], size=2)) + [offs[k + 1] - 1]:
            fd = _fd(f, p, i, 1e-6)
            worst = max(worst, abs(fd - g[i]) / max(abs(fd), 1e-3 * np.abs(g).max()))
    assert worst < 1e-6, worst


def test_output_filter_matches_correlate_and_is_symmetric():
    rng = np.random.default_rng(21)
    y = rng.normal(size=(2, 10, 12))
    k = np.array([[1.0, 2.0, 1.0], [2.0, 4.0, 2.0], [1.0, 2.0, 1.0]]) / 16.0
    mask = np.zeros((10, 12))
    mask[:9, :11] = 1.0
    want = y.copy()
    for _ in range(2):
        want = np.stack([signal.correlate2d(w * mask, k, mode="same") * mask for w in want])
    np.testing.assert_allclose(U.output_filter(y, 2), want, rtol=1e-13, atol=1e-15)
    u, v = rng.normal(size=(2, 1, 10, 12))
    assert np.sum(U.output_filter(u, 3) * v) == pytest.approx(np.sum(u * U.output_filter(v, 3)), rel=1e-12)
    # a constant inside the region is kept away from its edge; the row sums are 1
    c = np.ones((1, 10, 12))
    assert np.allclose(U.output_filter(c, 1)[0, 2:7, 2:9], 1.0)


def test_smoothed_network_backward_matches_finite_differences():
    c = 16
    rng = np.random.default_rng(13)
    p = _rand_params(c, 14)
    inp = rng.normal(size=(1, 16, 16, 2))
    inp[..., 1] = 0.5
    # a target near the output keeps the energy loss away from 1, where its
    # gradient (proportional to y.At) is too small for difference quotients
    y0 = U.forward(p, inp, c, smooth=2)
    t = y0 + 0.3 * np.std(y0) * rng.normal(size=(1, 16, 16))
    for kind in ("l2", "energy"):
        val, g = U.loss_grad(p, inp, t, c, kind=kind, nu_scale=100.0, smooth=2)

        def f(q):
            y = U.forward(q, inp, c, smooth=2)
            return U.energy_loss(y, t, [50.0])[0] if kind == "energy" else U.loss(y, t)

        assert val == pytest.approx(f(p), rel=1e-14)
        offs = np.cumsum([0] + [W.size + b.size for W, b in U.unpack(p, c)])
        worst = 0.0
        for k in (0, 8, 16, 17):
            for i in list(rng.integers(offs[k], offs[k + 1], size=2)) + [offs[k + 1] - 1]:
                fd = _fd(f, p, i, 1e-5)
                worst = max(worst, abs(fd - g[i]) / max(abs(fd), 1e-3 * np.abs(g).max()))
        assert worst < 1e-6, (kind, worst)
