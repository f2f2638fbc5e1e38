"""Pins of the surrogate network's CPU reference: back-propagated gradients against
central differences (FP64, tiny widths), and the BF16 rounding."""
import numpy as np
import pytest

from oracle import mlp_oracle as M


def _setup(H, n, seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(size=M.n_params(H)) * 0.5
    x = rng.normal(size=(n, 6)) * 3.0 + 1.0
    y = np.sin(x[:, 0]) + x[:, 1] * x[:, 2] * 0.1
    mu_x, sd_x = x.mean(0), x.std(0)
    return p, x, y, mu_x, sd_x, float(y.mean()), float(y.std())


@pytest.mark.parametrize("H,seed", [(5, 0), (3, 1), (8, 2)])
def test_backprop_matches_central_differences(H, seed):
    p, x, y, mx, sx, my, sy = _setup(H, 23, seed)
    loss, g = M.loss_and_grad(p, x, y, mx, sx, my, sy, H)
    num = np.empty_like(g)
    h = 1e-6
    for k in range(len(p)):
        e = np.zeros_like(p)
        e[k] = h
        num[k] = (M.loss_only(p + e, x, y, mx, sx, my, sy, H) -
                  M.loss_only(p - e, x, y, mx, sx, my, sy, H)) / (2 * h)
    assert np.max(np.abs(g - num)) <= 1e-7 * max(1.0, np.max(np.abs(num)))
    assert loss == pytest.approx(M.loss_only(p, x, y, mx, sx, my, sy, H))


def test_bf16_rounding():
    one = 1.0
    ulp = 2.0 ** -7          # spacing of BF16 at 1
    assert M.bf16(np.array([one + ulp / 2]))[0] == one            # tie -> even (1.0)
    assert M.bf16(np.array([one + 3 * ulp / 2]))[0] == one + 2 * ulp  # tie -> even
    assert M.bf16(np.array([one + 0.51 * ulp]))[0] == one + ulp
    assert M.bf16(np.array([-3.0]))[0] == -3.0
    assert M.bf16(np.array([255.5]))[0] == 256.0                  # carry into the exponent
    x = np.random.default_rng(0).normal(size=1000)
    r = M.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)


def test_forward_matches_loss_path():
    p, x, y, mx, sx, my, sy = _setup(5, 17, 4)
    out = M.forward(p, x, mx, sx, 5)
    t = (y - my) / sy
    assert M.loss_only(p, x, y, mx, sx, my, sy, 5) == pytest.approx(float(np.mean((out - t) ** 2)))
