"""Pins of the network's CPU statement (oracle/cnn.py): the analytic gradient
against central finite differences, and the forward pass against an
independent NumPy im2col implementation."""

import numpy as np
import pytest

from oracle import cnn


def _rand(seed, B=3):
    rng = np.random.default_rng(seed)
    p = np.zeros(cnn.NPARAM, np.float32)
    k = 0
    for name, shape in cnn.SHAPES:
        n = int(np.prod(shape))
        fan = {"W1": 9, "W2": 144, "W3": 288, "Wfc": 64}.get(name)
        p[k:k + n] = rng.normal(0, np.sqrt(2.0 / fan), n) if fan else rng.normal(0, 0.1, n)
        k += n
    img = rng.gamma(1.0, 1.0, (B, 64, 64)).astype(np.float32)
    bits = (img.view(np.uint32) >> 16).astype(np.uint16)  # bf16 by truncation: any bf16 values will do
    labels = rng.uniform(0.05, 0.8, B).astype(np.float32)
    return p, bits, labels


def test_gradient_matches_finite_differences():
    p, x, y = _rand(0)
    loss, g, _ = cnn.loss_and_grad(p, x, y, rounding=False)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(np.arange(0, 160), 6), rng.choice(np.arange(160, 4800), 6),
                          rng.choice(np.arange(4800, 23296), 6), [23296 + 5, 23360]])
    p64 = p.astype(np.float64)
    import torch

    xx = torch.tensor(cnn.bf16_to_f64(x))
    yy = torch.tensor(y.astype(np.float64))

    def L(v):
        with torch.no_grad():
            d = cnn.forward(torch.tensor(v), xx, rounding=False)
            return float(((d - yy) ** 2).mean())

    for i in idx:
        h = 1e-6 * max(1.0, abs(p64[i]))
        a, b = p64.copy(), p64.copy()
        a[i] += h
        b[i] -= h
        fd = (L(a) - L(b)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-9), (i, fd, g[i])


def _conv_np(x, W, b):
    """stride-2, pad-1, 3x3 convolution by im2col (x: [C, H, H])."""
    C, H, _ = x.shape
    Ho = H // 2
    xp = np.zeros((C, H + 2, H + 2))
    xp[:, 1:-1, 1:-1] = x
    cols = np.empty((C * 9, Ho * Ho))
    r = 0
    for c in range(C):
        for ky in range(3):
            for kx in range(3):
                cols[r] = xp[c, ky:ky + 2 * Ho:2, kx:kx + 2 * Ho:2].ravel()
                r += 1
    out = W.reshape(W.shape[0], -1) @ cols + b[:, None]
    return out.reshape(W.shape[0], Ho, Ho)


def test_forward_matches_independent_im2col():
    import torch

    p, x, y = _rand(2, B=2)
    P = {k: v.numpy() for k, v in cnn.unpack(torch.tensor(p.astype(np.float64))).items()}

    def bfr(a):
        return torch.tensor(a).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()

    want = []
    for b in range(2):
        x0 = cnn.bf16_to_f64(x[b])[None]
        a1 = np.maximum(_conv_np(x0, bfr(P["W1"]), P["b1"]), 0)
        a2 = np.maximum(_conv_np(bfr(a1), bfr(P["W2"]), P["b2"]), 0)
        a3 = np.maximum(_conv_np(bfr(a2), bfr(P["W3"]), P["b3"]), 0)
        g = a3.mean(axis=(1, 2))
        want.append(bfr(g) @ bfr(P["Wfc"]) + P["bfc"][0])
    got = cnn.predict(p, x)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12)
