"""Pins of the pair-kinematics oracle (CPU): the counter-based generator against numpy's
independent Philox4x64-10, and the lepton momenta against what relativity fixes whatever the
draw: four-momentum conservation, the mass shell, a textbook boost of the centre-of-mass
four-momenta (an independent route to the velocity-addition law of Eq. Lorentz), the equal
head-on case (gamma = E / m_e), the threshold case (both leptons at the CoM velocity), the
uniform lab Lorentz factor between closed-form bounds for 7/3 beams and the isotropy of the
direction draw."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import kinematics_oracle as K

ME = K.ME
MASK = (1 << 64) - 1


def _numpy_block(counter, key):
    """numpy's Philox4x64 block at `counter`: numpy adds one to its 256-bit counter before
    each block, so it is started one below."""
    c = sum(int(v) << (64 * a) for a, v in enumerate(counter)) - 1
    start = [(c >> (64 * a)) & MASK for a in range(4)]
    g = np.random.Philox(counter=np.array(start, dtype=np.uint64),
                         key=np.array(key, dtype=np.uint64))
    return [int(v) for v in g.random_raw(4)]


@pytest.mark.parametrize("counter,key", [
    ((1, 0, 0, 0), (5, 0)), ((3, 17, 29, 0), (12345, 0)), ((0, 1, 0, 0), (0, 0)),
    ((399, 999_999, 123_456, 0), (0xDEADBEEFCAFEF00D, 0)),
    ((MASK, MASK, MASK, 0), (MASK, 0)), ((7, 2, 3, 11), (1, 99))])
def test_philox_matches_numpy(counter, key):
    assert K.philox4x64(counter, key) == _numpy_block(counter, key)


def _photon(E, theta, phi=0.0):
    return E, (E * math.sin(theta) * math.cos(phi), E * math.sin(theta) * math.sin(phi),
               E * math.cos(theta))


def _random_pairs(n, seed, e_lo=0.6, e_hi=10.0):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        E1, E2 = np.exp(rng.uniform(math.log(e_lo), math.log(e_hi), 2))
        t1, t2 = np.arccos(rng.uniform(-1, 1, 2))
        p1, p2 = rng.uniform(0, 2 * math.pi, 2)
        a, pa = _photon(E1, t1, p1)
        b, pb = _photon(E2, t2, p2)
        s = (a * b - (pa[0] * pb[0] + pa[1] * pb[1] + pa[2] * pb[2])) / (2 * ME * ME)
        if s > 1.0:
            out.append((a, pa, b, pb))
    return out


def _boost(E, p, beta):
    """Textbook pure boost of four-momentum (E, p) by velocity beta (CoM -> lab)."""
    b2 = sum(x * x for x in beta)
    if b2 == 0.0:
        return E, tuple(p)
    g = 1.0 / math.sqrt(1.0 - b2)
    bp = sum(beta[a] * p[a] for a in range(3))
    coef = (g - 1.0) * bp / b2 + g * E
    return g * (E + bp), tuple(p[a] + coef * beta[a] for a in range(3))


def test_conservation_mass_shell_and_boost_equivalence():
    for h, (Ea, pa, Eb, pb) in enumerate(_random_pairs(300, 1)):
        pos, ele, n = K.pair_leptons(Ea, pa, Eb, pb, seed=7, k=h, i=2 * h, j=3 * h + 1)
        scale = Ea + Eb
        # four-momentum conservation
        assert abs(pos[0] + ele[0] - (Ea + Eb)) <= 1e-12 * scale
        for a in range(3):
            assert abs(pos[1 + a] + ele[1 + a] - (pa[a] + pb[a])) <= 1e-12 * scale
        # mass shell
        for lep in (pos, ele):
            m2 = lep[0] ** 2 - (lep[1] ** 2 + lep[2] ** 2 + lep[3] ** 2)
            assert abs(m2 - ME * ME) <= 1e-11 * lep[0] ** 2
        # the boost matrix applied to the CoM four-momenta (E', +-p' n)
        Et = Ea + Eb
        pt = [pa[a] + pb[a] for a in range(3)]
        s4 = Et * Et - sum(x * x for x in pt)
        pc = math.sqrt(s4 / 4.0 - ME * ME)
        ec = math.sqrt(s4) / 2.0
        beta = [x / Et for x in pt]
        for sgn, lep in ((1.0, pos), (-1.0, ele)):
            E_b, p_b = _boost(ec, [sgn * pc * x for x in n], beta)
            assert abs(E_b - lep[0]) <= 1e-11 * scale
            for a in range(3):
                assert abs(p_b[a] - lep[1 + a]) <= 1e-11 * scale


@pytest.mark.parametrize("gamma", [1.5, 5.0, 19.0])
def test_equal_head_on_energies_give_gamma_E_over_me(gamma):
    E = gamma * ME
    for h in range(50):
        pos, ele, n = K.pair_leptons(E, (0.0, 0.0, E), E, (0.0, 0.0, -E), 3, h, h + 1, 2 * h)
        assert abs(pos[0] / ME - gamma) <= 1e-12 * gamma
        assert abs(ele[0] / ME - gamma) <= 1e-12 * gamma
        p = math.sqrt(gamma * gamma - 1.0) * ME
        for a in range(3):  # CoM frame = lab frame: directions are the drawn ones
            assert abs(pos[1 + a] - p * n[a]) <= 1e-12 * E
            assert abs(ele[1 + a] + p * n[a]) <= 1e-12 * E


def test_threshold_leptons_move_with_the_centre_of_mass():
    # 90 degree crossing at threshold: E1 E2 (1 - cos 90) / 2 = m_e^2
    E1 = 3.0 * ME
    E2 = 2.0 * ME * ME / E1
    pos, ele, _ = K.pair_leptons(E1, (E1, 0.0, 0.0), E2, (0.0, E2, 0.0), 1, 2, 3, 4)
    for lep in (pos, ele):
        assert abs(lep[0] - (E1 + E2) / 2) <= 1e-6 * E1
        assert abs(lep[1] - E1 / 2) <= 1e-6 * E1  # p' ~ sqrt(rounding) at threshold
        assert abs(lep[2] - E2 / 2) <= 1e-6 * E1
        assert abs(lep[3]) <= 1e-6 * E1


def test_seven_three_beams_give_uniform_gamma_between_closed_form_bounds():
    """Head-on 7 m_e and 3 m_e photons: the lab gamma is linear in the CoM polar cosine,
    gamma = 5 (1 + 0.4 sqrt(20/21) cos theta*), so an isotropic draw spreads it uniformly
    over 5 -+ 2 sqrt(20/21) (the 3 <= gamma <= 7 spread of the 7/3 beams)."""
    E1, E2 = 7.0 * ME, 3.0 * ME
    half = 2.0 * math.sqrt(20.0 / 21.0)
    g = []
    for h in range(3000):
        pos, ele, n = K.pair_leptons(E1, (0.0, 0.0, E1), E2, (0.0, 0.0, -E2), 11, h % 7, h, h // 3)
        gp = pos[0] / ME
        assert abs(gp - 5.0 * (1.0 + 0.4 * math.sqrt(20.0 / 21.0) * n[2])) <= 1e-11
        assert abs(ele[0] / ME - 5.0 * (1.0 - 0.4 * math.sqrt(20.0 / 21.0) * n[2])) <= 1e-11
        g.append(gp)
    g = np.array(g)
    assert g.min() >= 5.0 - half - 1e-12 and g.max() <= 5.0 + half + 1e-12
    assert stats.kstest(g, stats.uniform(loc=5.0 - half, scale=2 * half).cdf).pvalue > 1e-3


def test_direction_draw_is_isotropic():
    d = np.array([K.cm_direction(5, k, i, 0) for k in range(40) for i in range(100)])
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    assert stats.kstest(d[:, 2], stats.uniform(loc=-1, scale=2).cdf).pvalue > 1e-3
    phi = np.mod(np.arctan2(d[:, 1], d[:, 0]), 2 * math.pi)
    assert stats.kstest(phi, stats.uniform(loc=0, scale=2 * math.pi).cdf).pvalue > 1e-3
    # distinct keys give distinct draws
    assert len({tuple(x) for x in d}) == len(d)


def test_histograms_by_hand():
    """Two pairs of known Lorentz factor (equal head-on energies, gamma = E / m_e) and
    weights: each lands in its bin with weight sqrt(w_i w_j); a factor outside the edges is
    dropped from the gamma histogram but kept in the angle histogram."""
    g = np.array([2.5, 4.5, 9.0])
    E = g * ME
    A = {"E": E, "px": np.zeros(3), "py": np.zeros(3), "pz": E, "w": np.array([1.0, 4.0, 9.0])}
    B = {"E": E, "px": np.zeros(3), "py": np.zeros(3), "pz": -E, "w": np.array([4.0, 9.0, 1.0])}
    i = np.array([0, 1, 2])
    j = np.array([0, 1, 2])
    k = np.array([0, 5, 9])
    pos, ele = K.kinematics(A, B, i, j, k, seed=1)
    edges = np.array([1.0, 3.0, 5.0, 8.0])
    gh, th = K.histograms(A, B, i, j, pos, edges, 4)
    assert np.allclose(gh, [2.0, 6.0, 0.0], rtol=0, atol=1e-12)
    assert abs(th.sum() - 11.0) <= 1e-12
    # polar angle bins from the drawn CoM directions (the lab frame here)
    expect = np.zeros(4)
    for h in range(3):
        n = K.cm_direction(1, int(k[h]), int(i[h]), int(j[h]))
        b = min(int(math.acos(n[2]) / math.pi * 4), 3)
        expect[b] += math.sqrt(A["w"][h] * B["w"][h])
    assert np.allclose(th, expect, rtol=0, atol=1e-12)
