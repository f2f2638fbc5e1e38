"""The surrogate network's kernels on the GPU: matrix-core product, gradients against
the CPU reference with BF16 rounding emulated, training."""
import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_1608_01125_amd import tril as T

pytestmark = pytest.mark.gpu

H = 256


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    return _t


def _bits(a):
    """BF16 bit patterns (int16) of float values, rounded to nearest even."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16).view(np.int16)


@pytest.mark.parametrize("M_,N,K,transA,transB", [
    (1, 1, 1, False, False), (17, 33, 45, False, False), (64, 64, 32, False, False),
    (130, 70, 300, True, False), (65, 129, 7, False, True), (200, 1, 256, True, True),
    # strides that take the 16-byte load paths (contiguous along k, and along rows)
    (256, 256, 256, False, False), (128, 64, 512, True, True), (64, 256, 4096, True, False),
    (72, 200, 264, False, True)])
def test_gemm_matches_numpy(torch, M_, N, K, transA, transB):
    rng = np.random.default_rng(M_ * 1000 + N + K)
    a = M.bf16(rng.normal(size=(M_, K)))
    b = M.bf16(rng.normal(size=(K, N)))
    A_store = a.T.copy() if transA else a
    B_store = b.T.copy() if transB else b
    sam, sak = (1, M_) if transA else (K, 1)
    sbk, sbn = (1, K) if transB else (N, 1)
    Ad = torch.from_numpy(_bits(A_store).ravel().copy()).cuda()
    Bd = torch.from_numpy(_bits(B_store).ravel().copy()).cuda()
    C = torch.zeros((M_, N), dtype=torch.float32, device="cuda")
    T.tril_dbg_gemm_bf16(Ad, sam, sak, Bd, sbk, sbn, M_, N, K, C)
    ref = a @ b
    got = C.cpu().numpy().astype(np.float64)
    scale = np.abs(a) @ np.abs(b) + 1e-30
    assert np.all(np.abs(got - ref) <= 1e-5 * scale)


def _data(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, 6)) * [1.0, 2.0, 0.5, 3.0, 1.0, 0.2] + [0.0, 1.0, -1.0, 4.0, 0.0, 2.0]
    y = np.sin(x[:, 0]) + 0.3 * x[:, 1] * x[:, 2] + np.log1p(np.abs(x[:, 3])) - x[:, 5]
    return x.astype(np.float32), y.astype(np.float32)


def test_gradients_match_reference_with_bf16_rounding(torch):
    x, y = _data(512, 1)
    mu_x, sd_x = x.mean(0), x.std(0) + 0.1
    mu_y, sd_y = float(y.mean()), float(y.std())
    net = T.Mlp(2, seed=5)
    try:
        net.set_norm(mu_x, sd_x, mu_y, sd_y)
        p = net.get_params(1)
        loss, g = net.grad(1, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    finally:
        net.close()
    mx = mu_x.astype(np.float32).astype(np.float64)
    sx = sd_x.astype(np.float32).astype(np.float64)
    loss_ref, g_ref = M.loss_and_grad(p.astype(np.float64), x.astype(np.float64),
                                      y.astype(np.float64), mx, sx, np.float32(mu_y),
                                      np.float32(sd_y), H, bf16_points=True)
    assert loss == pytest.approx(loss_ref, rel=1e-4)
    blocks = [H * 6, H, H * H, H, H * H, H, H, 1]
    o = 0
    for k in blocks:
        a, b = g[o:o + k].astype(np.float64), g_ref[o:o + k]
        assert np.linalg.norm(a - b) <= 1e-3 * np.linalg.norm(b) + 1e-12, (o, k)
        o += k


def test_params_round_trip(torch):
    net = T.Mlp(3, seed=1)
    try:
        p = np.random.default_rng(0).normal(size=T.MLP_PARAMS).astype(np.float32)
        net.set_params(2, p)
        assert np.array_equal(net.get_params(2), p)
        assert not np.array_equal(net.get_params(1), p)
    finally:
        net.close()


def test_training_fits_a_smooth_function(torch):
    x, y = _data(20000, 2)
    xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    net = T.Mlp(4, seed=3)
    try:
        net.fit_norm(xd, yd)
        l0 = net.train(xd, yd, n_steps=1, batch=1024, lr=1e-4)
        l1 = net.train(xd, yd, n_steps=1500, batch=1024, lr=2e-3, seed=1)
        xt, yt = _data(4000, 3)
        mean, sd = net.predict(torch.from_numpy(xt).cuda())
    finally:
        net.close()
    mean = mean.cpu().numpy()
    rmse = float(np.sqrt(np.mean((mean - yt) ** 2)))
    assert np.all(l1 < 0.05 * l0)
    assert rmse < 0.1 * float(np.std(yt))
    assert np.all(sd.cpu().numpy() >= 0)


@pytest.mark.parametrize("n", [1, 127, 129, 5000])
def test_predict_matches_reference(torch, n):
    """Ensemble mean and spread of the de-standardised output against the CPU reference
    with BF16 rounding emulated (all four layers fused in one kernel on the device)."""
    x, y = _data(n, 7)
    mu_x, sd_x = x.mean(0) if n > 1 else np.zeros(6, np.float32), (x.std(0) + 0.5 if n > 1 else np.ones(6, np.float32))
    mu_y, sd_y = 0.3, 1.7
    net = T.Mlp(3, seed=9)
    try:
        net.set_norm(mu_x, sd_x, mu_y, sd_y)
        ps = [net.get_params(k) for k in range(3)]
        mean, sd = net.predict(torch.from_numpy(x).cuda())
    finally:
        net.close()
    mx = np.asarray(mu_x, np.float32).astype(np.float64)
    sx = np.asarray(sd_x, np.float32).astype(np.float64)
    outs = np.stack([M.forward(p.astype(np.float64), x.astype(np.float64), mx, sx, H, bf16_points=True)
                     for p in ps]) * np.float32(sd_y) + np.float32(mu_y)
    ref_mean = outs.mean(0)
    ref_sd = outs.std(0, ddof=1)
    scale = np.abs(outs).max() + 1e-6
    assert np.max(np.abs(mean.cpu().numpy() - ref_mean)) <= 2e-3 * scale
    assert np.max(np.abs(sd.cpu().numpy() - ref_sd)) <= 2e-3 * scale
