"""Surrogate path of the statistical regime on the GPU: coverage of the candidate cell
pairs, training targets, and what the trained ensemble gains over the bin-level estimate
without it, with the gate holding the total within 1% of the exact path."""
import numpy as np
import pytest

from paper_1608_01125_amd import beams, surrogate
from paper_1608_01125_amd import tril as T

pytestmark = pytest.mark.gpu

N_MP = 20_000


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    return _t


@pytest.fixture(scope="module")
def ctx(torch):
    c = T.Context(0.1, None)
    yield c
    c.close()


def _interior(bins, n=32):
    iz = bins % n
    iy = (bins // n) % n
    ix = bins // (n * n)
    return (ix > 0) & (ix < n - 1) & (iy > 0) & (iy < n - 1) & (iz > 0) & (iz < n - 1)


def test_candidate_cell_pairs_cover_exact_pairs(ctx):
    """Every cell pair with an exact yield is a candidate when both cells are interior
    (edge cells also hold the photons outside the grid); the yield of the uncovered edge
    pairs is a negligible part of the total."""
    inst = surrogate.Instance(beams.st_headon(N_MP))
    tab, tot = inst.exact(ctx)
    keys, ys = tab.items()
    x, y0, key = inst.features(ctx)
    k = key.cpu().numpy()
    assert tot > 0 and len(keys) > 100
    nb = inst.gb.n_bins
    inner = _interior(keys // nb) & _interior(keys % nb)
    covered = np.isin(keys, k)
    assert np.all(covered[inner]), "an interior cell pair with a yield has no candidate row"
    assert ys[~covered].sum() <= 1e-4 * tot
    assert np.all(y0.cpu().numpy() > 0)
    assert np.all(np.isfinite(x.cpu().numpy()))
    t, y = T.tril_st_targets(key, y0, tab, 1e-3)
    yv = y.cpu().numpy()
    idx = {kk: i for i, kk in enumerate(k)}
    ck = keys[covered]
    assert np.array_equal(yv[[idx[kk] for kk in ck]], ys[covered])
    assert abs(yv.sum() - ys[covered].sum()) <= 1e-9 * tot


def test_trained_ensemble_beats_bin_level_estimate_and_per_pair_gate(torch, ctx):
    """Trained on six instances from the batched workload's parameter ranges, tested on
    the head-on shape (held out). The method without the network is the bin-level yield
    Y0 with one global scale fitted on the training rows. The network recovers the
    distribution of the yield over cell pairs far better (L1 distance to the exact
    distribution). The per-pair gate does what it states: every bin pair whose ensemble
    spread exceeds 1% goes to the exact path and every other keeps its prediction, and
    with this off-shape training that removes most of the network's bias. The spread of
    single pairs bounds no bias the members share, so the per-pair gate fixes no bound on
    the total; the audit gate does (test below)."""
    eps = 1e-3
    train_insts = [surrogate.Instance(beams.st_train_instance(m, N_MP)) for m in range(6)]
    x, t, y0, y = surrogate.training_rows(ctx, train_insts, eps=eps)
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    keep = (y > 0) | (torch.rand(y.shape[0], device="cuda", generator=g) < 0.25)
    net = T.Mlp(4, seed=11)
    try:
        surrogate.train(net, x[keep].contiguous(), t[keep].contiguous(), n_steps=1500, batch=8192,
                        lr=1e-3)
        inst = surrogate.Instance(beams.st_headon(N_MP))
        tab, exact_total = inst.exact(ctx)
        kappa = float(y.sum() / y0.sum())
        xe, y0e, ke = inst.features(ctx, T.sur_params(eps=eps))
        _, ye = T.tril_st_targets(ke, y0e, tab, eps)
        mean, sd = net.predict(xe)
        pred = (y0e * (torch.exp(mean.double()) - eps)).clamp(min=0)
        res = inst.surrogate(ctx, net, T.sur_params(eps=eps, gate=0.01, per_pair=True))
        never = inst.surrogate(ctx, net, T.sur_params(eps=eps, gate=1e30, per_pair=True))
    finally:
        net.close()
    l1_base = float((kappa * y0e - ye).abs().sum() / ye.sum())
    l1_net = float((pred - ye).abs().sum() / ye.sum())
    err_gated = abs(res["total"] - exact_total) / exact_total
    err_never = abs(never["total"] - exact_total) / exact_total
    unsure = sd > 0.01
    print(f"\nexact {exact_total:.6g}  L1 bin-level {l1_base:.3f}  L1 network {l1_net:.3f}  "
          f"ungated error {err_never:.5f}  gated error {err_gated:.5f} "
          f"({res['n_gated']} of {res['n_bin_pairs']} pairs exact)")
    assert abs(never["total"] - float(pred.sum())) <= 1e-4 * float(pred.sum())
    assert never["n_gated"] == 0 and res["n_gated"] > 0
    # the gate's own guarantee: exactly the pairs above the spread threshold are exact, and
    # the confident pairs contribute their predictions
    assert res["n_gated"] == int(unsure.sum())
    assert res["surrogate_part"] == pytest.approx(float(pred[~unsure].sum()), rel=1e-4)
    assert l1_net < 0.5 * l1_base
    assert err_gated <= 0.25 * err_never


@pytest.fixture(scope="module")
def same_shape_net(torch, ctx):
    """Ensemble trained on head-on instances of the benchmark's shape (seeds 2000 + m),
    with its calibration factor."""
    eps = 1e-3
    insts = [surrogate.Instance(beams.st_headon(N_MP, seed=2000 + m)) for m in range(4)]
    x, t, y0, y = surrogate.training_rows(ctx, insts, eps=eps)
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    keep = (y > 0) | (torch.rand(y.shape[0], device="cuda", generator=g) < 0.25)
    net = T.Mlp(4, seed=12)
    surrogate.train(net, x[keep].contiguous(), t[keep].contiguous(), n_steps=1500, batch=8192,
                    lr=1e-3)
    scale = surrogate.yield_scale(net, x, y0, y, eps)
    yield net, scale
    net.close()


def test_budget_gate_with_same_shape_training(torch, ctx, same_shape_net):
    """Trained on head-on instances of the same shape, the ensemble's spread is a fair error
    estimate: the budget gate (largest uncertainty contributions exact until the spread of
    the rest is within 1% of the total) holds the total within 1% while most bin pairs stay
    with the network."""
    net, scale = same_shape_net
    inst = surrogate.Instance(beams.st_headon(N_MP))
    _, exact_total = inst.exact(ctx)
    res = inst.surrogate(ctx, net, T.sur_params(eps=1e-3, gate=0.01, scale=scale))
    err = abs(res["total"] - exact_total) / exact_total
    print(f"\nbudget gate: error {err:.5f}, {res['n_gated']} of {res['n_bin_pairs']} pairs exact, "
          f"predicted spread {res['predicted_spread']:.4f}")
    assert res["predicted_spread"] <= 0.01
    assert err <= 0.01
    assert res["n_gated"] < 0.2 * res["n_bin_pairs"]


def test_calibration_factor_is_reproducible(torch, same_shape_net):
    """tril_st_calibrate reduces in a fixed order: the same rows give the same factor."""
    net, scale = same_shape_net
    insts = [surrogate.Instance(beams.st_headon(N_MP, seed=2000 + m)) for m in range(2)]
    c = T.Context(0.1, None)
    try:
        x, _, y0, y = surrogate.training_rows(c, insts)
        x2, _, _, _ = surrogate.training_rows(c, insts)
    finally:
        c.close()
    # rows come in ascending key order: the same rows in the same order on every call (an
    # FP32 feature may differ in its last bit where its FP64 sum was rounded in another order)
    assert x.shape == x2.shape
    assert float((x - x2).abs().max()) <= 1e-5 * float(x.abs().max())
    f1 = T.tril_st_calibrate(net, x, y0, y)
    f2 = T.tril_st_calibrate(net, x, y0, y)
    assert f1 == f2
    mean, _ = net.predict(x)
    pred = (y0 * (torch.exp(mean.double()) - 1e-3)).clamp(min=0)
    assert f1 == pytest.approx(float(y.sum() / pred.sum()), rel=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_audit_gate_holds_total_within_1pct_on_held_out_seeds(torch, ctx, same_shape_net, seed):
    """Held-out instances (seeds not used in training): the audit gate (a sampled exact
    estimate with the network's predictions as control, pilot-scaled) gives a total within
    1% of the exact total of the hierarchy path, inside twice its own 95% half-width, with
    its macro-particle sample a small part of the beams."""
    net, scale = same_shape_net
    inst = surrogate.Instance(beams.st_headon(N_MP, seed=seed))
    _, exact_total = inst.exact(ctx)
    res = inst.surrogate(ctx, net, T.sur_params(eps=1e-3, scale=scale, audit=True,
                                                audit_sample=2000, audit_reps=8,
                                                audit_seed=100 + seed))
    err = abs(res["total"] - exact_total) / exact_total
    print(f"\naudit gate seed {seed}: error {err:.5f}, half-width "
          f"{res['audit_half_width'] / exact_total:.5f}, network alone "
          f"{res['surrogate_part'] / exact_total - 1:+.5f}")
    assert err <= 0.01
    assert abs(res["total"] - exact_total) <= 2.0 * res["audit_half_width"]
    assert res["audit_half_width"] <= 0.005 * exact_total
    assert res["audit_sampled"] <= 0.5 * 9 * 2 * N_MP
