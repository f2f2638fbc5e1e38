"""Pins of the IP-regime swarm oracle (CPU): placement of the real photons (a full lattice
when n = 8^L, one per octant and balanced at every level otherwise), single-photon swarms
against closed-form impact parameters, aligned head-on lattices whose collisions can be
counted by hand, threshold and symmetry."""
import math

import numpy as np
import pytest

from oracle import oracle as O

ME = 0.51099895


def test_full_lattice_when_n_is_a_power_of_eight():
    cell = (0.5, 0.8, 1.25)
    for L in (1, 2, 3):
        n = 8 ** L
        o = O.swarm_offsets(n, cell)
        m = 2 ** L
        expect = set()
        for ix in range(m):
            for iy in range(m):
                for iz in range(m):
                    expect.add(tuple(round(((c + 0.5) * cell[a] / m - 0.5 * cell[a]), 12)
                                     for a, c in enumerate((ix, iy, iz))))
        got = {tuple(round(v, 12) for v in row) for row in o}
        assert got == expect


@pytest.mark.parametrize("n", [2, 9, 27, 100, 333, 511, 700])
def test_balanced_over_octants_at_every_level(n):
    """Real photons spread evenly: per octant of level 1 and per sub-octant of level 2 the
    counts differ by at most one."""
    cell = (1.0, 1.0, 1.0)
    o = O.swarm_offsets(n, cell) + 0.5  # [0, 1)^3
    for level in (1, 2):
        m = 2 ** level
        idx = np.floor(o * m).astype(int)
        key = (idx[:, 0] * m + idx[:, 1]) * m + idx[:, 2]
        counts = np.bincount(key, minlength=m ** 3)
        if n >= m ** 3:
            assert counts.max() - counts.min() <= 1
        else:  # fewer photons than sub-octants: at most one each, spread over level-1 octants
            assert counts.max() == 1
            top = np.bincount((np.floor(o * 2).astype(int) @ np.array([4, 2, 1])), minlength=8)
            assert top.max() - top.min() <= 1
    # distinct positions inside the box
    assert len({tuple(r) for r in o}) == n
    assert o.min() > 0.0 and o.max() < 1.0


def _pair(b, E=2.0, t_star=1.0, w=1.0, dx_dir=0.0):
    """Photon a along +z at (b, 0, -t*), photon b along -z at (0, 0, t*): they pass at
    distance b at time t*."""
    A = {"x": np.array([b]), "y": np.zeros(1), "z": np.array([-t_star]),
         "px": np.array([dx_dir]), "py": np.zeros(1), "pz": np.array([E]), "E": np.array([E]),
         "w": np.array([w])}
    A["E"] = np.sqrt(A["px"] ** 2 + A["pz"] ** 2)
    B = {"x": np.zeros(1), "y": np.zeros(1), "z": np.array([t_star]), "px": np.zeros(1),
         "py": np.zeros(1), "pz": np.array([-E]), "E": np.array([E]), "w": np.array([w])}
    return A, B


def test_single_photon_swarms_against_impact_parameter():
    s = 2.0 * 2.0 * 2.0 / (2 * ME * ME)
    r = math.sqrt(O.sigma(s) / math.pi)
    for f, hit in ((0.0, 1), (0.5, 1), (0.999, 1), (1.001, 0), (3.0, 0)):
        A, B = _pair(f * r)
        cnt, knife = O.swarm_pairs(A, B, 0.1, 0, 20, (0.5, 0.5, 0.5))
        assert knife == 0
        assert cnt[0, 0] == hit
    # the closest approach must fall inside the run window
    A, B = _pair(0.0, t_star=5.0)
    assert O.swarm_pairs(A, B, 0.1, 0, 20, (0.5, 0.5, 0.5))[0][0, 0] == 0
    assert O.swarm_pairs(A, B, 0.1, 40, 20, (0.5, 0.5, 0.5))[0][0, 0] == 1
    # the window is [k0 dt, (k0 + n_steps) dt]: a crossing in its last or first step counts
    A, B = _pair(0.0, t_star=1.95)
    assert O.swarm_pairs(A, B, 0.1, 0, 20, (0.5, 0.5, 0.5))[0][0, 0] == 1
    assert O.swarm_pairs(A, B, 0.1, 0, 19, (0.5, 0.5, 0.5))[0][0, 0] == 0
    A, B = _pair(0.0, t_star=0.05)
    assert O.swarm_pairs(A, B, 0.1, 0, 1, (0.5, 0.5, 0.5))[0][0, 0] == 1
    assert O.swarm_pairs(A, B, 0.1, 1, 5, (0.5, 0.5, 0.5))[0][0, 0] == 0


@pytest.mark.parametrize("L", [1, 2])
def test_aligned_head_on_lattices(L):
    """Equal cells and n = 8^L photons per swarm, head-on along z, same transverse centre:
    photons of equal (x, y) lattice columns pass through each other (distance 0), all others
    stay a lattice spacing apart; so 4^L columns x (2^L)^2 pairs collide. Shifted by half a
    spacing transversely, none."""
    n = 8 ** L
    cell = (0.5, 0.5, 0.5)
    A, B = _pair(0.0, t_star=1.0, w=float(n))
    cnt, knife = O.swarm_pairs(A, B, 0.1, 0, 20, cell)
    assert knife == 0
    assert cnt[0, 0] == 16 ** L
    A, B = _pair(0.5 * cell[0] / 2 ** L, t_star=1.0, w=float(n))
    assert O.swarm_pairs(A, B, 0.1, 0, 20, cell)[0][0, 0] == 0


def test_threshold_rounding_and_symmetry():
    rng = np.random.default_rng(3)
    n = 12

    def beam(zc, sgn, E):
        # collimated, transverse spread and cloud size of the order of the radius (~2e-9 um)
        return {"x": rng.normal(0, 2e-9, n), "y": rng.normal(0, 2e-9, n),
                "z": rng.normal(zc, 0.05, n), "px": np.zeros(n), "py": np.zeros(n),
                "pz": np.full(n, sgn * E), "E": np.full(n, E),
                "w": rng.integers(1, 60, n).astype(float) + 0.4}
    A, B = beam(-0.5, 1.0, 2.0), beam(0.5, -1.0, 2.0)
    cell = (4e-9, 4e-9, 4e-9)
    c1, k1 = O.swarm_pairs(A, B, 0.1, 0, 20, cell)
    c2, k2 = O.swarm_pairs(B, A, 0.1, 0, 20, cell)
    assert k1 == 0 and k2 == 0
    assert c1.sum() > 0
    assert np.array_equal(c1, c2.T)
    # weights round to floor(w + 1/2): k + 0.4 -> k photons, k + 0.6 -> k + 1
    Ak = dict(A)
    Ak["w"] = A["w"] - 0.4
    assert np.array_equal(O.swarm_pairs(Ak, B, 0.1, 0, 20, cell)[0], c1)
    A6, A7 = dict(A), dict(A)
    A6["w"] = A["w"] + 0.2
    A7["w"] = A["w"] + 0.6
    assert np.array_equal(O.swarm_pairs(A6, B, 0.1, 0, 20, cell)[0],
                          O.swarm_pairs(A7, B, 0.1, 0, 20, cell)[0])
    # below threshold: nothing
    for X in (A, B):
        X["E"] = X["E"] * 0.1
        X["px"], X["py"], X["pz"] = X["px"] * 0.1, X["py"] * 0.1, X["pz"] * 0.1
    c4, _ = O.swarm_pairs(A, B, 0.1, 0, 20, cell)
    assert c4.sum() == 0
