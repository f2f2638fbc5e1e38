"""Pins of the sampled-estimate oracle (CPU): the thinning draws keep each row with its
inclusion probability, keeping every row reproduces the exact total, and the Horvitz-
Thompson estimate is unbiased (its mean over independent replicates converges to the
exact total of the cloud-pair yields)."""
import numpy as np
import pytest

from oracle import audit_oracle as AO
from oracle import oracle as O


def _beam(n, sgn, rng, E=2.0, w0=1e5):
    d = np.c_[rng.normal(0, 0.01, n), rng.normal(0, 0.01, n), np.full(n, sgn)]
    d /= np.linalg.norm(d, axis=1)[:, None]
    return {"x": rng.normal(0, 0.3, n), "y": rng.normal(0, 0.3, n),
            "z": -sgn * 1.0 + rng.normal(0, 0.3, n),
            "px": E * d[:, 0], "py": E * d[:, 1], "pz": E * d[:, 2], "E": np.full(n, E),
            "w": w0 * rng.uniform(0.5, 1.5, n)}


def test_inclusion_probability_formula():
    w = np.array([1.0, 2.0, 3.0, 0.0, 4.0])
    p = AO.inclusion_no_control(w, 2.0)
    np.testing.assert_allclose(p, [0.2, 0.4, 0.6, 0.0, 0.8], rtol=0, atol=1e-15)
    assert np.all(AO.inclusion_no_control(w, 100.0)[w > 0] == 1.0)


def test_draws_keep_each_row_with_its_probability():
    n, reps = 50, 400
    pi = np.linspace(0.02, 0.98, n)
    kept = np.zeros(n)
    for r in range(reps):
        kept += AO.uniforms(n, 7, r, 0) < pi
    freq = kept / reps
    # binomial standard error per row; 5 sigma over 50 rows
    assert np.all(np.abs(freq - pi) <= 5 * np.sqrt(pi * (1 - pi) / reps) + 1e-12)
    # the two beam sides and two replicates draw different numbers
    assert not np.array_equal(AO.uniforms(n, 7, 0, 0), AO.uniforms(n, 7, 0, 1))
    assert not np.array_equal(AO.uniforms(n, 7, 0, 0), AO.uniforms(n, 7, 1, 0))


def test_full_sample_is_the_exact_total():
    rng = np.random.default_rng(3)
    A, B = _beam(30, 1.0, rng), _beam(30, -1.0, rng)
    cell = (0.3, 0.3, 0.4)
    exact = O.st_pairs(A, B, 0.1, 0, 40, cell).sum()
    assert exact > 0
    est, ka, kb = AO.ht_total(A, B, np.ones(30), np.ones(30), 1, 0, 0.1, 0, 40, cell)
    assert len(ka) == 30 and len(kb) == 30
    assert est == pytest.approx(exact, rel=1e-13)


def test_horvitz_thompson_mean_converges_to_exact():
    rng = np.random.default_rng(5)
    A, B = _beam(40, 1.0, rng), _beam(40, -1.0, rng)
    cell = (0.3, 0.3, 0.4)
    Y = O.st_pairs(A, B, 0.1, 0, 40, cell)
    exact = Y.sum()
    pa = AO.inclusion_no_control(A["w"], 15.0)
    pb = AO.inclusion_no_control(B["w"], 15.0)
    reps = 300
    est = np.array([AO.ht_total(A, B, pa, pb, 11, r, 0.1, 0, 40, cell)[0] for r in range(reps)])
    # variance of the two-sided Horvitz-Thompson estimator with independent Poisson draws
    ya, yb = Y.sum(1), Y.sum(0)
    var = (np.sum((1 / pa - 1) * ya ** 2) + np.sum((1 / pb - 1) * yb ** 2)
           + np.sum(np.outer(1 / pa - 1, 1 / pb - 1) * Y ** 2))
    se = np.sqrt(var / reps)
    assert abs(est.mean() - exact) <= 4 * se
    # the sample variance agrees with the closed form
    assert 0.7 * var <= est.var(ddof=1) <= 1.4 * var
