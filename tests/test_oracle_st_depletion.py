"""Pins of the depletion picture of the statistical regime (CPU): the closed forms n_1/2 and
n_alpha against a numerical integration of the rate equation they solve, their limits (no
depletion at small exposure, the smaller cloud used up at large exposure), the equality of
one closed form at the summed exposure with a step-by-step depletion, the per-pair exposure
against the pinned linear yield, and a hand-built co-located pair."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import oracle as O
from oracle import st_oracle as SO

ME = 0.51099895


def _ode(a, b, k_tau):
    """dn/dt = (a - n)(b - n) integrated to t = k tau (k = 1), tight tolerances."""
    sol = solve_ivp(lambda t, n: (a - n) * (b - n), (0.0, k_tau), [0.0], method="DOP853",
                    rtol=1e-12, atol=1e-14 * min(a, b))
    return float(sol.y[0, -1])


@pytest.mark.parametrize("alpha", [0.5, 0.3, 0.05, 0.4999, 0.9])
@pytest.mark.parametrize("n0k_tau", [1e-3, 0.3, 2.0, 15.0])
def test_closed_forms_solve_the_rate_equation(alpha, n0k_tau):
    n0 = 4.0
    a, b = alpha * n0, (1.0 - alpha) * n0
    k_tau = n0k_tau / n0
    expect = _ode(a, b, k_tau)
    got = SO.depleted_density(a, b, k_tau)
    assert got == pytest.approx(expect, rel=1e-9)
    if alpha == 0.5:
        assert SO.n_half(n0, k_tau) == pytest.approx(expect, rel=1e-9)
    else:
        assert SO.n_alpha(n0, min(alpha, 1 - alpha), k_tau) == pytest.approx(expect, rel=1e-9)


def test_limits():
    a, b = 3.0, 7.0
    for S in (1e-12, 1e-9, 1e-6):  # no depletion: the linear yield a b S
        assert SO.depleted_density(a, b, S) == pytest.approx(a * b * S, rel=10 * b * S + 1e-14)
    assert SO.depleted_density(a, b, 50.0) == pytest.approx(a, rel=1e-12)  # smaller cloud used up
    assert SO.depleted_density(5.0, 5.0, 1e6) == pytest.approx(5.0, rel=1e-5)
    assert SO.depleted_density(a, b, 0.0) == 0.0
    # alpha -> 1/2 joins n_1/2 continuously
    for eps in (1e-6, 1e-9, 1e-12):
        assert SO.depleted_density(5.0 * (1 - eps), 5.0, 0.2) == pytest.approx(
            SO.depleted_density(5.0, 5.0, 0.2), rel=5 * eps + 1e-13)


@pytest.mark.parametrize("a,b", [(3.0, 7.0), (5.0, 5.0), (0.01, 9.0)])
def test_summed_exposure_equals_step_by_step_depletion(a, b):
    """Densities depleted after every step by that step's creations, each step taken with the
    closed form at its own exposure: the total equals one closed form at the summed exposure
    (the equation is autonomous in n)."""
    rng = np.random.default_rng(0)
    S = rng.uniform(0.0, 0.08, 40)
    n, aa, bb = 0.0, a, b
    for s in S:
        d = SO.depleted_density(aa, bb, s)
        n += d
        aa -= d
        bb -= d
    assert n == pytest.approx(SO.depleted_density(a, b, S.sum()), rel=1e-11)


def _beams(seed, n=30):
    rng = np.random.default_rng(seed)
    A = {"x": rng.normal(0, 0.3, n), "y": rng.normal(0, 0.3, n), "z": rng.normal(-2, 0.5, n),
         "px": rng.normal(0, 0.05, n), "py": rng.normal(0, 0.05, n), "pz": np.full(n, 2.0),
         "w": rng.uniform(0.5, 2.0, n) * 1e8}
    B = {"x": rng.normal(0, 0.3, n), "y": rng.normal(0, 0.3, n), "z": rng.normal(2, 0.5, n),
         "px": rng.normal(0, 0.05, n), "py": rng.normal(0, 0.05, n), "pz": np.full(n, -1.5),
         "w": rng.uniform(0.5, 2.0, n) * 1e8}
    for X in (A, B):
        X["E"] = np.sqrt(X["px"] ** 2 + X["py"] ** 2 + X["pz"] ** 2)
    return A, B


def test_exposure_against_linear_yield_and_bounds():
    """Per pair, S (w_i / V)(w_j / V) V is the pinned linear yield; the depleted yield never
    exceeds it nor the smaller cloud's weight."""
    A, B = _beams(1)
    cell = (0.5, 0.5, 0.5)
    V = 0.125
    S = O.st_exposure(A, B, 0.1, 0, 40, cell)
    Ylin = O.st_pairs(A, B, 0.1, 0, 40, cell)
    assert (S > 0).sum() > 30
    lin = S * (A["w"][:, None] / V) * (B["w"][None, :] / V) * V
    np.testing.assert_allclose(lin, Ylin, rtol=1e-12, atol=0)
    for boost in (1.0, 1e12):
        Ab, Bb = dict(A), dict(B)
        Ab["w"], Bb["w"] = A["w"] * boost, B["w"] * boost
        Y, S2 = SO.st_depleted_pairs(Ab, Bb, 0.1, 0, 40, cell)
        assert np.array_equal(S, S2)
        Yl = O.st_pairs(Ab, Bb, 0.1, 0, 40, cell)
        assert np.all(Y <= Yl * (1 + 1e-12))
        assert np.all(Y <= np.minimum(Ab["w"][:, None], Bb["w"][None, :]) * (1 + 1e-12))
        if boost == 1.0:  # (a + b) S ~ 1e-8: first-order depletion only
            ab = (Ab["w"][:, None] + Bb["w"][None, :]) / V * S
            assert ab.max() < 1e-6
            assert np.all(Yl - Y <= Yl * ab + 1e-14 * Yl)
            assert np.all(Yl - Y >= Yl * ab / 4 - 1e-14 * Yl)
        else:             # strongly depleted pairs exist
            r = Y[S > 0] / Yl[S > 0]
            assert r.min() < 0.5


def test_co_located_pair_by_hand():
    """Head-on clouds shorter along z than one step's closing distance meet fully overlapping
    in one step: S = sigma (1 - cos pi) dt = 2 sigma dt; with equal weights w the depleted
    yield is V (w/V)^2 S / (1 + (w/V) S)."""
    dt, k, E, w = 0.1, 7, 2.0, 3.0e17
    t_star = k * dt + 0.5 * dt
    cell = (1.0, 1.0, 0.15)
    V = 0.15
    A = {"x": np.zeros(1), "y": np.zeros(1), "z": np.array([-t_star]), "px": np.zeros(1),
         "py": np.zeros(1), "pz": np.array([E]), "E": np.array([E]), "w": np.array([w])}
    B = {"x": np.zeros(1), "y": np.zeros(1), "z": np.array([t_star]), "px": np.zeros(1),
         "py": np.zeros(1), "pz": np.array([-E]), "E": np.array([E]), "w": np.array([w])}
    s = E * E * 2.0 / (2.0 * ME * ME)
    S = 2.0 * O.sigma(s) * dt
    Y, S2 = SO.st_depleted_pairs(A, B, dt, 0, 20, cell)
    assert S2[0, 0] == pytest.approx(S, rel=1e-13)
    n = w / V
    assert Y[0, 0] == pytest.approx(V * n * n * S / (1.0 + n * S), rel=1e-12)
    assert n * S > 0.5  # the case is depleted
