"""FP64 reference of the U-Net preconditioner (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of the
benchmark may import this module.  It shares no code with the GPU library:
the network is written out here from its definition in numpy, in float64,
with every layer a plain sum over taps and channels and the backward pass a
hand-written reverse sweep through the same layers.

Network (base width c, images H x W with H, W multiples of 8, NHWC):
  encoder   level 0: conv3x3(2 -> c) ReLU, conv3x3(c -> c) ReLU            -> e0
            level 1: pool, conv3x3(c -> 2c) ReLU, conv3x3(2c -> 2c) ReLU   -> e1
            level 2: pool, conv3x3(2c -> 4c) ReLU, conv3x3(4c -> 4c) ReLU  -> e2
            level 3: pool, conv3x3(4c -> 8c) ReLU, conv3x3(8c -> 8c) ReLU  -> m
  decoder   k = 4c, 2c, c:  u = upconv2x2(2k -> k) of the level below,
            conv3x3([u, e] -> k) ReLU, conv3x3(k -> k) ReLU
  output    1x1 conv (c -> 1)
  pool = 2x2 average; conv3x3 zero-pads by one pixel; upconv2x2 is the
  transposed convolution with kernel 2 and stride 2.
  The first layer's weights are stored for 8 input channels of which only the
  first two carry data (the other six are zero in every input).

Flat parameter layout (float, layer by layer, weights then bias):
  conv3x3   W[ky*3 + kx][ci][co], output (y, x) reads input (y+ky-1, x+kx-1)
  upconv    W[ci][a*2 + b][co], output (2y+a, 2x+b) from input (y, x)
  output    w[c], then one bias
Optional output filter: passes of the 3x3 binomial filter after the output
layer (``output_filter``).
Losses: L = (1/B) sum_b ||y_b - t_b||^2 / ||t_b||^2 (``loss``), or the
energy loss (``energy_loss``) L = (1/B) sum_b [1 - (y_b.A t_b)^2 / ((y_b.A y_b)
(t_b.A t_b))] with A the P1 operator -Delta + nu I of Section 2 (eq. (4)) on
the interior nodes of the unit square's n x n diagonal-cut grid, applied here
through the element residual of this package (``grid_operator``).
Optimiser: Adam (Kingma & Ba, ICLR 2015, Algorithm 1) with bias-corrected
moments, ``adam`` below.

Parity pins (tests/test_oracle_unet.py): every layer type against a library
routine (scipy.signal.correlate for conv3x3, numpy.kron for the transposed
convolution, a box filter for pooling), and the whole backward pass against
central finite differences in float64.
"""
from __future__ import annotations

import numpy as np

IN_STORED = 8  # input channels stored for the first layer


def architecture(c):
    """List of layers: (kind, level, input channel groups, Cout); kind 'conv' or 'up'."""
    return [
        ("conv", 0, (IN_STORED,), c), ("conv", 0, (c,), c),
        ("conv", 1, (c,), 2 * c), ("conv", 1, (2 * c,), 2 * c),
        ("conv", 2, (2 * c,), 4 * c), ("conv", 2, (4 * c,), 4 * c),
        ("conv", 3, (4 * c,), 8 * c), ("conv", 3, (8 * c,), 8 * c),
        ("up", 3, (8 * c,), 4 * c), ("conv", 2, (4 * c, 4 * c), 4 * c), ("conv", 2, (4 * c,), 4 * c),
        ("up", 2, (4 * c,), 2 * c), ("conv", 1, (2 * c, 2 * c), 2 * c), ("conv", 1, (2 * c,), 2 * c),
        ("up", 1, (2 * c,), c), ("conv", 0, (c, c), c), ("conv", 0, (c,), c),
    ]


def param_count(c):
    n = 0
    for kind, _, groups, cout in architecture(c):
        cin = sum(groups)
        n += (9 * cin * cout if kind == "conv" else cin * 4 * cout) + cout
    return n + c + 1


def unpack(params, c):
    """Flat vector -> list of (W, b): conv W (3, 3, Cin, Cout); up W (Cin, 2, 2, Cout); output (w (c,), b)."""
    p = np.asarray(params, dtype=np.float64)
    assert p.shape == (param_count(c),)
    out, o = [], 0
    for kind, _, groups, cout in architecture(c):
        cin = sum(groups)
        if kind == "conv":
            nw = 9 * cin * cout
            W = p[o:o + nw].reshape(3, 3, cin, cout)
        else:
            nw = cin * 4 * cout
            W = p[o:o + nw].reshape(cin, 2, 2, cout)
        o += nw
        out.append((W, p[o:o + cout]))
        o += cout
    out.append((p[o:o + c], p[o + c:o + c + 1]))
    return out


def pack(layers):
    """Inverse of unpack."""
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


# --------------------------------------------------------------------------
# Layers (forward and backward), batch-first NHWC float64 arrays
# --------------------------------------------------------------------------

def conv3x3(x, W, b):
    """out[n, y, x, o] = b[o] + sum_{ky, kx, i} xpad[n, y + ky, x + kx, i] W[ky, kx, i, o]."""
    N, H, Wd, _ = x.shape
    xp = np.zeros((N, H + 2, Wd + 2, x.shape[3]))
    xp[:, 1:H + 1, 1:Wd + 1, :] = x
    out = np.zeros((N, H, Wd, W.shape[3])) + b
    for ky in range(3):
        for kx in range(3):
            out += xp[:, ky:ky + H, kx:kx + Wd, :] @ W[ky, kx]
    return out


def conv3x3_backward(x, W, g):
    """Gradients (dx, dW, db) of conv3x3 for the output gradient g."""
    N, H, Wd, _ = x.shape
    xp = np.zeros((N, H + 2, Wd + 2, x.shape[3]))
    xp[:, 1:H + 1, 1:Wd + 1, :] = x
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    gm = g.reshape(-1, g.shape[3])
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + H, kx:kx + Wd, :].reshape(-1, x.shape[3])
            dW[ky, kx] = patch.T @ gm
            dxp[:, ky:ky + H, kx:kx + Wd, :] += g @ W[ky, kx].T
    return dxp[:, 1:H + 1, 1:Wd + 1, :], dW, g.sum(axis=(0, 1, 2))


def upconv(x, W, b):
    """out[n, 2y + a, 2x + c, o] = b[o] + sum_i x[n, y, x, i] W[i, a, c, o]."""
    N, H, Wd, _ = x.shape
    out = np.zeros((N, 2 * H, 2 * Wd, W.shape[3]))
    for a in range(2):
        for c in range(2):
            out[:, a::2, c::2, :] = x @ W[:, a, c, :] + b
    return out


def upconv_backward(x, W, g):
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    xm = x.reshape(-1, x.shape[3])
    for a in range(2):
        for c in range(2):
            ga = g[:, a::2, c::2, :]
            dx += ga @ W[:, a, c, :].T
            dW[:, a, c, :] = xm.T @ ga.reshape(-1, g.shape[3])
    return dx, dW, g.sum(axis=(0, 1, 2))


def pool(x):
    """2x2 average."""
    return 0.25 * (x[:, 0::2, 0::2] + x[:, 1::2, 0::2] + x[:, 0::2, 1::2] + x[:, 1::2, 1::2])


def pool_backward(g):
    N, H, Wd, C = g.shape
    out = np.zeros((N, 2 * H, 2 * Wd, C))
    for a in range(2):
        for c in range(2):
            out[:, a::2, c::2] = 0.25 * g
    return out


def relu(v):
    return np.maximum(v, 0.0)


# --------------------------------------------------------------------------
# Network
# --------------------------------------------------------------------------

def _input8(inp):
    inp = np.asarray(inp, dtype=np.float64)
    N, H, Wd, two = inp.shape
    assert two == 2 and H % 8 == 0 and Wd % 8 == 0
    x = np.zeros((N, H, Wd, IN_STORED))
    x[..., :2] = inp
    return x


def output_filter(y, passes):
    """``passes`` passes of the 3x3 binomial filter (1 2 1; 2 4 2; 1 2 1) / 16 over
    the pixels x < W-1, y < H-1 of each image (B, H, W); the last row and
    column are read and written as 0.  Each output pixel is the weighted sum of
    its (up to nine) neighbours inside that region."""
    y = np.array(y, dtype=np.float64)
    B, H, W = y.shape
    wts = {-1: 1.0, 0: 2.0, 1: 1.0}
    for _ in range(passes):
        src = np.zeros_like(y)
        src[:, : H - 1, : W - 1] = y[:, : H - 1, : W - 1]
        out = np.zeros_like(y)
        for yy in range(H - 1):
            for xx in range(W - 1):
                acc = np.zeros(B)
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        if 0 <= yy + dy < H - 1 and 0 <= xx + dx < W - 1:
                            acc += wts[dy] * wts[dx] * src[:, yy + dy, xx + dx]
                out[:, yy, xx] = acc / 16.0
        y = out
    return y


def forward(params, inp, c, keep=False, smooth=0):
    """inp (B, H, W, 2) -> y (B, H, W); with keep=True also the activations for
    backward.  smooth: passes of ``output_filter`` after the output layer."""
    L = unpack(params, c)
    a = {"x": _input8(inp)}
    a["e0a"] = relu(conv3x3(a["x"], *L[0]))
    a["e0"] = relu(conv3x3(a["e0a"], *L[1]))
    a["p0"] = pool(a["e0"])
    a["e1a"] = relu(conv3x3(a["p0"], *L[2]))
    a["e1"] = relu(conv3x3(a["e1a"], *L[3]))
    a["p1"] = pool(a["e1"])
    a["e2a"] = relu(conv3x3(a["p1"], *L[4]))
    a["e2"] = relu(conv3x3(a["e2a"], *L[5]))
    a["p2"] = pool(a["e2"])
    a["ma"] = relu(conv3x3(a["p2"], *L[6]))
    a["m"] = relu(conv3x3(a["ma"], *L[7]))
    a["u2"] = upconv(a["m"], *L[8])
    a["c2"] = np.concatenate([a["u2"], a["e2"]], axis=3)
    a["d2a"] = relu(conv3x3(a["c2"], *L[9]))
    a["d2"] = relu(conv3x3(a["d2a"], *L[10]))
    a["u1"] = upconv(a["d2"], *L[11])
    a["c1"] = np.concatenate([a["u1"], a["e1"]], axis=3)
    a["d1a"] = relu(conv3x3(a["c1"], *L[12]))
    a["d1"] = relu(conv3x3(a["d1a"], *L[13]))
    a["u0"] = upconv(a["d1"], *L[14])
    a["c0"] = np.concatenate([a["u0"], a["e0"]], axis=3)
    a["d0a"] = relu(conv3x3(a["c0"], *L[15]))
    a["d0"] = relu(conv3x3(a["d0a"], *L[16]))
    w, b = L[17]
    y = a["d0"] @ w + b[0]
    if smooth:
        y = output_filter(y, smooth)
    return (y, a) if keep else y


def loss(y, t):
    """(1/B) sum_b ||y_b - t_b||^2 / ||t_b||^2."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    B = y.shape[0]
    return float(sum(np.sum((y[i] - t[i]) ** 2) / np.sum(t[i] ** 2) for i in range(B)) / B)


def unit_square_grid(n):
    """The unit square cut into n x n squares, each split by its diagonal from
    the lower-left to the upper-right corner: node i + j (n + 1) at (i/n, j/n);
    triangles (a, a+1, a+n+2) and (a, a+n+2, a+n+1) with a = i + j (n + 1).
    Returns (coords (n_nodes, 2), elems (2 n^2, 3), boundary node mask)."""
    m = n + 1
    j, i = np.divmod(np.arange(m * m), m)
    coords = np.stack([i / n, j / n], axis=1).astype(np.float64)
    cj, ci = np.divmod(np.arange(n * n), n)
    a = ci + cj * m
    elems = np.concatenate([np.stack([a, a + 1, a + m + 1], 1), np.stack([a, a + m + 1, a + m], 1)])
    bnd = ((i == 0) | (i == n) | (j == 0) | (j == n)).astype(np.uint8)
    return coords, elems.astype(np.int32), bnd


def grid_operator(n, nu):
    """v -> A v for images (n, n): pixel (y, x) is interior node (x + 1, y + 1)
    of ``unit_square_grid(n)`` (the last row and column hold no node and are
    read and written as 0); A v is minus the element residual of eq. (4) with
    b = 0 and the boundary rows masked (Section 2's Dirichlet treatment)."""
    from . import local_matrices, residual  # the oracle's element code

    coords, elems, bnd = unit_square_grid(n)
    K, M, _ = local_matrices(coords, elems)
    nn = coords.shape[0]
    zero = np.zeros(nn)

    def apply(v):
        x = np.zeros((n + 1, n + 1))
        x[1:n, 1:n] = np.asarray(v, dtype=np.float64)[: n - 1, : n - 1]
        r = -residual(nn, elems, K, M, nu, zero, x.ravel(), bnd).reshape(n + 1, n + 1)
        out = np.zeros((n, n))
        out[: n - 1, : n - 1] = r[1:n, 1:n]
        return out

    return apply


def energy_loss(y, t, nus):
    """(L, dL/dy) of the energy loss for outputs y, targets t (B, n, n) and the
    per-sample coefficients nus: per sample with a = y.At, b = y.Ay, c = t.At
    (y, t restricted to the interior pixels) the term is 1 - a^2 / (b c), and 1
    with zero gradient when b <= 0 or c <= 0; dL/dy = (1/B) (2 a^2 / (b^2 c) Ay -
    2 a / (b c) At) on the interior pixels, 0 on the last row and column."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    B, n, _ = y.shape
    inner = np.zeros((n, n))
    inner[: n - 1, : n - 1] = 1.0
    val = 0.0
    gy = np.zeros_like(y)
    for k in range(B):
        A = grid_operator(n, float(nus[k]))
        yk, tk = y[k] * inner, t[k] * inner
        Ay, At = A(yk), A(tk)
        a, b, c = np.sum(yk * At), np.sum(yk * Ay), np.sum(tk * At)
        if b > 0 and c > 0:
            val += 1.0 - a * a / (b * c)
            gy[k] = (2.0 * a * a / (b * b * c) * Ay - 2.0 * a / (b * c) * At) * inner / B
        else:
            val += 1.0
    return val / B, gy


def loss_grad(params, inp, target, c, input_grad=False, kind="l2", nu_scale=100.0, smooth=0):
    """(L, dL/dparams flat [, dL/dinput (B, H, W, 2)]) for the loss ``kind``
    ("l2" or "energy"; the energy loss takes nu_b = nu_scale * inp[b, 0, 0, 1])
    of the network with ``smooth`` output-filter passes."""
    t = np.asarray(target, dtype=np.float64)
    y, a = forward(params, inp, c, keep=True, smooth=smooth)
    B = y.shape[0]
    if kind == "energy":
        val, gy = energy_loss(y, t, [nu_scale * float(np.asarray(inp)[b, 0, 0, 1]) for b in range(B)])
    else:
        val = loss(y, t)
        gy = np.stack([2.0 * (y[i] - t[i]) / (B * np.sum(t[i] ** 2)) for i in range(B)])
    out = backward(params, a, gy, c, input_grad, smooth)
    return (val,) + out if input_grad else (val, out)


def backward(params, a, gy, c, input_grad=False, smooth=0):
    """Reverse sweep from the output gradient gy (B, H, W) through the
    activations ``a`` of ``forward(..., keep=True)``: dL/dparams flat
    [, dL/dinput (B, H, W, 2)].  The output filter is symmetric (a masked
    convolution with a symmetric kernel), so its passes carry gy back to the
    output layer unchanged in form."""
    L = unpack(params, c)
    if smooth:
        gy = output_filter(gy, smooth)
    G = [None] * len(L)
    w, _ = L[17]
    G[17] = ((a["d0"] * gy[..., None]).sum(axis=(0, 1, 2)), np.array([gy.sum()]))
    g = gy[..., None] * w  # d loss / d d0

    def conv_relu_back(idx, xin, out, g_out):
        gz = g_out * (out > 0)
        dx, dW, db = conv3x3_backward(xin, L[idx][0], gz)
        G[idx] = (dW, db)
        return dx

    g = conv_relu_back(16, a["d0a"], a["d0"], g)
    g = conv_relu_back(15, a["c0"], a["d0a"], g)
    c0 = a["u0"].shape[3]
    g_u0, g_e0 = g[..., :c0], g[..., c0:]
    g, dW, db = upconv_backward(a["d1"], L[14][0], g_u0)
    G[14] = (dW, db)
    g = conv_relu_back(13, a["d1a"], a["d1"], g)
    g = conv_relu_back(12, a["c1"], a["d1a"], g)
    c1 = a["u1"].shape[3]
    g_u1, g_e1 = g[..., :c1], g[..., c1:]
    g, dW, db = upconv_backward(a["d2"], L[11][0], g_u1)
    G[11] = (dW, db)
    g = conv_relu_back(10, a["d2a"], a["d2"], g)
    g = conv_relu_back(9, a["c2"], a["d2a"], g)
    c2 = a["u2"].shape[3]
    g_u2, g_e2 = g[..., :c2], g[..., c2:]
    g, dW, db = upconv_backward(a["m"], L[8][0], g_u2)
    G[8] = (dW, db)
    g = conv_relu_back(7, a["ma"], a["m"], g)
    g = conv_relu_back(6, a["p2"], a["ma"], g)
    g = g_e2 + pool_backward(g)
    g = conv_relu_back(5, a["e2a"], a["e2"], g)
    g = conv_relu_back(4, a["p1"], a["e2a"], g)
    g = g_e1 + pool_backward(g)
    g = conv_relu_back(3, a["e1a"], a["e1"], g)
    g = conv_relu_back(2, a["p0"], a["e1a"], g)
    g = g_e0 + pool_backward(g)
    g = conv_relu_back(1, a["e0a"], a["e0"], g)
    g = conv_relu_back(0, a["x"], a["e0a"], g)
    flat = pack(G)
    if input_grad:
        return flat, g[..., :2]
    return flat


def grid_input(r, N, cval):
    """Network input of the nodal residual r on the (N+1)^2 grid (node i + j (N+1)):
    interior node (i, j) -> pixel (y, x) = (j - 1, i - 1), scaled to unit RMS over
    the interior; last row and column zero; channel 1 = cval.  Shape (1, N, N, 2)."""
    r = np.asarray(r, dtype=np.float64).reshape(N + 1, N + 1)
    inner = r[1:N, 1:N]
    rms = np.sqrt(np.mean(inner ** 2))
    img = np.zeros((1, N, N, 2))
    img[0, :N - 1, :N - 1, 0] = inner / rms if rms > 0 else 0.0
    img[0, :, :, 1] = cval
    return img


def grid_output(y, N, mask=None):
    """Network output image (1, N, N) -> nodal vector; boundary and masked nodes 0."""
    z = np.zeros((N + 1, N + 1))
    z[1:N, 1:N] = np.asarray(y, dtype=np.float64)[0, :N - 1, :N - 1]
    z = z.ravel()
    if mask is not None:
        z[np.asarray(mask, dtype=bool)] = 0.0
    return z


def adam(params, grads, lrs, beta1=0.9, beta2=0.999, eps=1e-8, history=False):
    """Adam steps t = 1, 2, ... on a flat parameter vector (Kingma & Ba, Algorithm 1):
        m_t = beta1 m_{t-1} + (1 - beta1) g_t,   v_t = beta2 v_{t-1} + (1 - beta2) g_t^2
        m^_t = m_t / (1 - beta1^t),               v^_t = v_t / (1 - beta2^t)
        theta_t = theta_{t-1} - lr_t m^_t / (sqrt(v^_t) + eps)
    from m_0 = v_0 = 0, with grads[t-1] and lrs[t-1] the gradient and learning
    rate of step t.  Returns theta after the last step, or every theta_t with
    history=True."""
    theta = np.array(params, dtype=np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    out = []
    for t, (g, lr) in enumerate(zip(grads, lrs), start=1):
        g = np.asarray(g, dtype=np.float64)
        m = beta1 * m + (1.0 - beta1) * g
        v = beta2 * v + (1.0 - beta2) * g * g
        mhat = m / (1.0 - beta1 ** t)
        vhat = v / (1.0 - beta2 ** t)
        theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
        out.append(theta.copy())
    return out if history else theta
