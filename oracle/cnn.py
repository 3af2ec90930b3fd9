"""CPU statement of the learned-incumbent network (fp64, PyTorch CPU ops).

TEST INFRASTRUCTURE ONLY.  The network is not in the paper: it proposes a
starting incumbent for Algorithm 1 (the branch and bound still certifies the optimum).

Definition (parameters as one fp32 vector, layout below):
  x0 = image (64x64, values already bfloat16)
  z1 = conv3x3/s2/p1(x0; bf(W1)) + b1,   a1 = relu(z1)      16 x 32 x 32
  z2 = conv3x3/s2/p1(bf(a1); bf(W2)) + b2, a2 = relu(z2)   32 x 16 x 16
  z3 = conv3x3/s2/p1(bf(a2); bf(W3)) + b3, a3 = relu(z3)   64 x 8 x 8
  g  = mean over the 8x8 positions of a3                    64
  d  = bf(g) . bf(Wfc) + bfc
where bf() rounds to bfloat16 (nearest even).  Training loss: mean squared
error over the batch.  Gradients treat bf() as the identity (the usual
mixed-precision rule); ``rounding=False`` drops bf() altogether, giving a
smooth function whose gradient finite differences can check.
"""

from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

SHAPES = [
    ("W1", (16, 1, 3, 3)), ("b1", (16,)),
    ("W2", (32, 16, 3, 3)), ("b2", (32,)),
    ("W3", (64, 32, 3, 3)), ("b3", (64,)),
    ("Wfc", (64,)), ("bfc", (1,)),
]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p: torch.Tensor):
    out, k = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = p[k:k + n].reshape(shape)
        k += n
    return out


class _STE(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x):
        return x.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    @staticmethod
    def backward(ctx, g):
        return g


def bf(x: torch.Tensor, rounding: bool) -> torch.Tensor:
    return _STE.apply(x) if rounding else x


def forward(params, imgs, rounding: bool = True) -> torch.Tensor:
    """params: fp64 tensor [NPARAM]; imgs: fp64 [B, 64, 64]. Returns [B]."""
    P = unpack(params)
    x = imgs.unsqueeze(1)
    a1 = F.relu(F.conv2d(x, bf(P["W1"], rounding), P["b1"], stride=2, padding=1))
    a2 = F.relu(F.conv2d(bf(a1, rounding), bf(P["W2"], rounding), P["b2"], stride=2, padding=1))
    a3 = F.relu(F.conv2d(bf(a2, rounding), bf(P["W3"], rounding), P["b3"], stride=2, padding=1))
    g = a3.mean(dim=(2, 3))
    return bf(g, rounding) @ bf(P["Wfc"], rounding) + P["bfc"]


def loss_and_grad(params_f32: np.ndarray, imgs_bf16: np.ndarray, labels: np.ndarray, rounding: bool = True):
    """MSE loss and its gradient w.r.t. the parameters (fp64)."""
    p = torch.tensor(np.asarray(params_f32, np.float64), requires_grad=True)
    x = torch.tensor(bf16_to_f64(imgs_bf16))
    y = torch.tensor(np.asarray(labels, np.float64))
    d = forward(p, x, rounding)
    loss = ((d - y) ** 2).mean()
    loss.backward()
    return float(loss.item()), p.grad.numpy().copy(), d.detach().numpy()


def predict(params_f32: np.ndarray, imgs_bf16: np.ndarray, rounding: bool = True) -> np.ndarray:
    with torch.no_grad():
        p = torch.tensor(np.asarray(params_f32, np.float64))
        return forward(p, torch.tensor(bf16_to_f64(imgs_bf16)), rounding).numpy()


def bf16_to_f64(bits: np.ndarray) -> np.ndarray:
    b = np.asarray(bits, np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)
