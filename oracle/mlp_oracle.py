"""CPU reference of the surrogate network (FP64 numpy), for the gradient checks.

TEST INFRASTRUCTURE ONLY: used by the test suite, never by the product library.

Network (per member): x -> standardise -> [Linear 6->H, SiLU] -> [Linear H->H, SiLU] ->
[Linear H->H, SiLU] -> Linear H->1; loss = mean over rows of (output - (y - mu_y)/sd_y)^2.
Parameters flattened as W1 [H][6], b1 [H], W2 [H][H], b2, W3 [H][H], b3, W4 [H], b4 [1].
With ``bf16=True`` the values that enter each product (the standardised input, the
weights, every hidden activation, the output gradient and every pre-activation
gradient) are rounded to BF16 (round to nearest, ties to even) as the device kernels
round them; everything else stays FP64.
"""
from __future__ import annotations

import numpy as np


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def n_params(H: int, n_in: int = 6) -> int:
    return H * n_in + H + 2 * (H * H + H) + H + 1


def unpack(p: np.ndarray, H: int, n_in: int = 6):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    out = []
    for shape in ((H, n_in), (H,), (H, H), (H,), (H, H), (H,), (H,), (1,)):
        k = int(np.prod(shape))
        out.append(p[o:o + k].reshape(shape))
        o += k
    assert o == len(p)
    return out


def _silu(z):
    return z / (1.0 + np.exp(-z))


def _dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def loss_and_grad(p, x, y, mu_x, sd_x, mu_y, sd_y, H: int, bf16_points: bool = False):
    """Loss (mean squared error of the standardised output) and its gradient with
    respect to the flattened parameters, by back-propagation."""
    r = bf16 if bf16_points else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(p, H, len(mu_x))
    W1q, W2q, W3q, W4q = r(W1), r(W2), r(W3), r(W4)
    n = len(y)
    X = r((np.asarray(x, np.float64) - mu_x) / sd_x)
    Z1 = X @ W1q.T + b1
    H1 = r(_silu(Z1))
    Z2 = H1 @ W2q.T + b2
    H2 = r(_silu(Z2))
    Z3 = H2 @ W3q.T + b3
    H3 = r(_silu(Z3))
    out = H3 @ W4q + b4[0]
    t = (np.asarray(y, np.float64) - mu_y) / sd_y
    d = out - t
    loss = float(np.mean(d * d))
    dy = r(2.0 * d / n)
    gW4 = dy @ H3
    gb4 = np.array([np.sum(2.0 * d / n)])
    dZ3 = np.outer(dy, W4q) * _dsilu(Z3)
    dZ3q = r(dZ3)
    gW3 = dZ3q.T @ H2
    gb3 = dZ3.sum(0)
    dZ2 = (dZ3q @ W3q) * _dsilu(Z2)
    dZ2q = r(dZ2)
    gW2 = dZ2q.T @ H1
    gb2 = dZ2.sum(0)
    dZ1 = (dZ2q @ W2q) * _dsilu(Z1)
    dZ1q = r(dZ1)
    gW1 = dZ1q.T @ X
    gb1 = dZ1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3, gW4, gb4])
    return loss, g


def forward(p, x, mu_x, sd_x, H: int, bf16_points: bool = False) -> np.ndarray:
    """Standardised network output per row (same rounding points as loss_and_grad)."""
    r = bf16 if bf16_points else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(p, H, len(mu_x))
    X = r((np.asarray(x, np.float64) - mu_x) / sd_x)
    H1 = r(_silu(X @ r(W1).T + b1))
    H2 = r(_silu(H1 @ r(W2).T + b2))
    H3 = r(_silu(H2 @ r(W3).T + b3))
    return H3 @ r(W4) + b4[0]


def loss_only(p, x, y, mu_x, sd_x, mu_y, sd_y, H: int) -> float:
    return loss_and_grad(p, x, y, mu_x, sd_x, mu_y, sd_y, H)[0]
