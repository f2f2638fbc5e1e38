"""The sampled estimate of the exact statistical-regime total (tril_st_audit, through the C
ABI): its thinning and Horvitz-Thompson sum against the CPU oracle replicate by replicate,
its identity with the exact total when every macro-particle is kept, its confidence
interval against the exact total of the hierarchy path, and the variance a control
removes."""
import numpy as np
import pytest

from oracle import audit_oracle as AO
from paper_1608_01125_amd import beams, surrogate
from paper_1608_01125_amd import tril as T

pytestmark = pytest.mark.gpu


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


@pytest.fixture(scope="module")
def inst20k(ctx):
    inst = surrogate.Instance(beams.st_headon(20_000))
    _, exact = inst.exact(ctx)
    return inst, exact


def test_replicate_matches_oracle_thinning_and_sum(ctx):
    """No control: each replicate's thinned beams (rows and inclusion probabilities) are the
    oracle's Philox draws, and its estimate is the oracle's exact sum over the thinned
    beams' cloud pairs (the same pair yields in another summation order)."""
    wl = beams.st_headon(3000)
    A, B = beams.draw_pair(wl)
    inst = surrogate.Instance(wl, A, B)
    lam, seed = 700, 91
    res = inst.audit(ctx, None, T.AUDIT_NONE, n_sample=lam, n_rep=2, seed=seed)
    rows_q, pi_q = T.tril_dbg_st_audit_sample(ctx, 0, 5000)
    rows_t, pi_t = T.tril_dbg_st_audit_sample(ctx, 1, 5000)
    pa = AO.inclusion_no_control(A["w"], lam)
    pb = AO.inclusion_no_control(B["w"], lam)
    est, ka, kb = AO.ht_total(A, B, pa, pb, seed, 1, wl.dt, 0, wl.n_steps, inst.ga.cell)
    o = np.argsort(rows_q)
    assert np.array_equal(rows_q[o], ka)
    np.testing.assert_allclose(pi_q[o], pa[ka], rtol=1e-15, atol=0)
    o = np.argsort(rows_t)
    assert np.array_equal(rows_t[o], kb)
    np.testing.assert_allclose(pi_t[o], pb[kb], rtol=1e-15, atol=0)
    assert est > 0
    assert res["rep"][1] == pytest.approx(est, rel=1e-9)
    assert res["control_total"] == 0.0
    assert res["n_sampled"][0] > 0.8 * 2 * lam


def test_keeping_every_macro_particle_gives_the_exact_total(ctx, inst20k):
    """With an expected sample far above the beam size every inclusion probability is 1:
    each replicate is the exact total, and the control total cancels its thinned estimate."""
    inst, exact = inst20k
    for control, passes in ((T.AUDIT_BIN_LEVEL, 3), (T.AUDIT_NONE, 2)):  # with a pilot: 3
        res = inst.audit(ctx, None, control, n_sample=10_000_000, n_rep=2, seed=5)
        for r in res["rep"]:
            assert r == pytest.approx(exact, rel=1e-9)
        assert res["n_sampled"] == (passes * 20_000, passes * 20_000)
        if control == T.AUDIT_BIN_LEVEL:
            # the pilot of a full sample measures the control's scale exactly
            assert res["control_total"] == pytest.approx(exact, rel=1e-9)


def test_confidence_interval_covers_exact_total_and_control_shrinks_it(ctx, inst20k):
    """Bin-level control: the 95% interval holds the exact total of the hierarchy path
    (three seeds) and is several times narrower than with no control at the same sample
    size; the mean over many replicates converges to the exact total (unbiased)."""
    inst, exact = inst20k
    hw = {}
    for control in (T.AUDIT_BIN_LEVEL, T.AUDIT_NONE):
        for seed in (1, 2, 3):
            res = inst.audit(ctx, None, control, n_sample=3000, n_rep=8, seed=seed)
            assert abs(res["estimate"] - exact) <= 2.0 * res["half_width"], (control, seed, res)
            hw.setdefault(control, []).append(res["half_width"] / exact)
    print(f"\nrelative half-widths: bin-level control {np.round(hw[T.AUDIT_BIN_LEVEL], 4)}, "
          f"none {np.round(hw[T.AUDIT_NONE], 4)}")
    assert max(hw[T.AUDIT_BIN_LEVEL]) < 0.5 * min(hw[T.AUDIT_NONE])
    res = inst.audit(ctx, None, T.AUDIT_BIN_LEVEL, n_sample=3000, n_rep=64, seed=17)
    reps = np.array(res["rep"])
    se = reps.std(ddof=1) / np.sqrt(len(reps))
    assert abs(reps.mean() - exact) <= 4 * se
    # the half-width is Student's t (63 degrees of freedom) times the standard error
    assert res["half_width"] == pytest.approx(1.9983 * se, rel=2e-3)


def test_audit_argument_checks(ctx, inst20k):
    inst, _ = inst20k
    with pytest.raises(T.TrilError):
        inst.audit(ctx, None, T.AUDIT_NETWORK)  # the network control needs a model
    with pytest.raises(T.TrilError):
        inst.audit(ctx, None, T.AUDIT_NONE, n_rep=1)
    with pytest.raises(T.TrilError):
        inst.audit(ctx, None, T.AUDIT_NONE, n_rep=65)
