"""Pins of the statistical-regime oracle (CPU): closed forms of the cloud yield, the
time integral of the overlap of two cubes, symmetries, and hand-computed bin indices."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import st_oracle as SO

ME = 0.51099895


def _beam(x, p, E, w):
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    p = np.atleast_2d(np.asarray(p, dtype=np.float64))
    return {"x": x[:, 0].copy(), "y": x[:, 1].copy(), "z": x[:, 2].copy(),
            "px": p[:, 0].copy(), "py": p[:, 1].copy(), "pz": p[:, 2].copy(),
            "E": np.asarray(E, dtype=np.float64).reshape(-1), "w": np.asarray(w, dtype=np.float64).reshape(-1)}


def _headon(t_star, E=2.0, wa=3.0e5, wb=7.0e5, dx=0.0):
    """Photon a along +z and photon b along -z, at the same point (up to an offset dx
    along x) at time t_star."""
    A = _beam([[dx, 0.0, -t_star]], [[0.0, 0.0, E]], [E], [wa])
    B = _beam([[0.0, 0.0, t_star]], [[0.0, 0.0, -E]], [E], [wb])
    s = E * E * 2.0 / (2.0 * ME * ME)
    return A, B, s


def test_single_step_co_location():
    """Clouds shorter along z than the 2 dt the pair closes in per step meet in one step
    only, fully overlapping: Y = w_a w_b sigma(s) (1 - cos pi) dt / V."""
    dt, k = 0.1, 7
    t_star = k * dt + 0.5 * dt
    cell = (1.0, 1.0, 0.15)
    A, B, s = _headon(t_star)
    Y = O.st_pairs(A, B, dt, 0, 20, cell)[0, 0]
    V = cell[0] * cell[1] * cell[2]
    expect = 3.0e5 * 7.0e5 * O.sigma(s) * 2.0 * dt / V
    assert Y == pytest.approx(expect, rel=1e-13)
    # one step shorter on either side misses it
    assert O.st_pairs(A, B, dt, 0, k, cell)[0, 0] == 0.0
    assert O.st_pairs(A, B, dt, k + 1, 10, cell)[0, 0] == 0.0


@pytest.mark.parametrize("dx", [0.0, 0.3, -0.45])
def test_overlap_integral_of_crossing_cubes(dx):
    """Head-on clouds with c_z = 10 dt that coincide (up to dx) at a step boundary: the
    overlap along z, c_z - 2|t - t*|, has its kinks on step boundaries, so the midpoint
    sum over steps equals its integral c_z^2 / 2; the transverse overlap is (c_x - |dx|) c_y.
    Y = n_a n_b sigma (1 - cos pi) (c_x - |dx|) c_y c_z^2 / 2."""
    dt = 0.1
    cell = (1.0, 0.8, 1.0)
    t_star = 1.0
    A, B, s = _headon(t_star, dx=dx)
    Y = O.st_pairs(A, B, dt, 0, 40, cell)[0, 0]
    V = cell[0] * cell[1] * cell[2]
    expect = (3.0e5 * 7.0e5 / V ** 2) * O.sigma(s) * 2.0 * (cell[0] - abs(dx)) * cell[1] * cell[2] ** 2 / 2.0
    assert Y == pytest.approx(expect, rel=1e-12)


def test_below_threshold_and_co_moving_give_nothing():
    dt = 0.1
    cell = (1.0, 1.0, 1.0)
    A, B, s = _headon(1.0, E=0.3)
    assert s < 1.0
    assert O.st_pairs(A, B, dt, 0, 40, cell)[0, 0] == 0.0
    # same direction: s = 0
    A = _beam([[0.0, 0.0, 0.0]], [[0.0, 0.0, 5.0]], [5.0], [1e6])
    B = _beam([[0.1, 0.0, 0.0]], [[0.0, 0.0, 5.0]], [5.0], [1e6])
    assert O.st_pairs(A, B, dt, 0, 40, cell)[0, 0] == 0.0


def _random_pair(n, seed):
    rng = np.random.default_rng(seed)
    def one(sign):
        u = rng.normal(size=(n, 3)) * 0.05
        u[:, 2] = sign
        u /= np.linalg.norm(u, axis=1)[:, None]
        E = rng.uniform(1.0, 4.0, n)
        x = rng.normal(size=(n, 3)) * [0.5, 0.5, 1.0]
        x[:, 2] -= sign * 2.0
        return _beam(x, u * E[:, None], E, rng.uniform(1e4, 1e6, n))
    return one(1.0), one(-1.0)


def test_swapping_the_beams_transposes_the_yields():
    A, B = _random_pair(40, 3)
    cell = (0.7, 0.7, 0.9)
    Yab = O.st_pairs(A, B, 0.1, 0, 40, cell)
    Yba = O.st_pairs(B, A, 0.1, 0, 40, cell)
    assert (Yab > 0).sum() > 20
    assert np.array_equal(Yab, Yba.T)


def test_yield_scales_with_weights():
    A, B = _random_pair(30, 4)
    cell = (0.7, 0.7, 0.9)
    Y1 = O.st_pairs(A, B, 0.1, 0, 40, cell)
    A2 = dict(A, w=A["w"] * 2.0)
    assert np.array_equal(O.st_pairs(A2, B, 0.1, 0, 40, cell), 2.0 * Y1)


GRID = SO.Grid(lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0), n_pos=(4, 4, 4), n_e=4, e_lo=1.0,
               e_hi=16.0, n_th=2, th_max=0.2, axis=(0.0, 0.0, 1.0), t_bin=0.0)


def _dir(theta):
    return np.array([math.sin(theta), 0.0, math.cos(theta)])


def test_bin_indices_by_hand():
    # photon 0: x (-0.9, 0.1, 0.6): cells (0, 2, 3); E = 3: log(3)/log(16) * 4 = 1.58 -> 1;
    # angle 0.15 rad of 0.2 over 2 bins -> 1. bin = (((0*4 + 2)*4 + 3)*4 + 1)*2 + 1 = 91
    # photon 1: x (5, -5, 0) clamps to cells (3, 0, 2); E = 100 -> 3; angle 1 rad -> 1.
    #   bin = (((3*4 + 0)*4 + 2)*4 + 3)*2 + 1 = 407
    # photon 2: x (0.2, -0.2, -0.2), E = 1.5 -> 0, angle 0.05 -> 0: cells (2, 1, 1):
    #   bin = (((2*4 + 1)*4 + 1)*4 + 0)*2 + 0 = 296
    x = [[-0.9, 0.1, 0.6], [5.0, -5.0, 0.0], [0.2, -0.2, -0.2]]
    E = np.array([3.0, 100.0, 1.5])
    d = np.stack([_dir(0.15), _dir(1.0), _dir(0.05)])
    b, sums = SO.bin_beam(_beam(x, d * E[:, None], E, [2.0, 3.0, 4.0]), GRID)
    assert list(b) == [91, 407, 296]
    assert sums[407][0] == 3.0 and sums[407][1] == 300.0


def test_bin_uses_position_at_grid_time():
    # a photon along +z from z = -0.6 reaches z = -0.1 at t_bin = 0.5: cell 1 instead of 0
    g = SO.Grid(**{**GRID.__dict__, "t_bin": 0.5})
    B = _beam([[0.0, 0.0, -0.6]], [[0.0, 0.0, 2.0]], [2.0], [1.0])
    b0, _ = SO.bin_beam(B, GRID)
    b1, _ = SO.bin_beam(B, g)
    # cells (2, 2, 0) vs (2, 2, 1); E = 2 -> 1; angle 0 -> 0
    assert b0[0] == (((2 * 4 + 2) * 4 + 0) * 4 + 1) * 2
    assert b1[0] == (((2 * 4 + 2) * 4 + 1) * 4 + 1) * 2


def test_table_adds_up_to_total():
    A, B = _random_pair(50, 5)
    cell = (0.7, 0.7, 0.9)
    ga = SO.Grid(**{**GRID.__dict__, "lo": (-2, -2, -4), "hi": (2, 2, 4)})
    ba, _ = SO.bin_beam(A, ga)
    bb, _ = SO.bin_beam(B, ga)
    tab, tot = SO.st_table(A, ba, B, bb, ga.n_bins, 0.1, 0, 40, cell)
    assert len(tab) > 5
    assert sum(tab.values()) == pytest.approx(tot, rel=1e-12)


def test_table_keys_two_by_two_bins_closed_form():
    """Hand-built keying of the bin-pair table: query photons of bins 3 and 7, target
    photons of bins 1 and 5, with 11 target bins, so the keys are 3*11+1 = 34, 38, 78 and
    82 (a swapped key b*n + a, or a stride other than the target's bin count, gives other
    numbers). All four clouds meet head-on in one step, fully overlapping, so each pair's
    yield is the single-step closed form w_i w_j sigma(s_ij) (1 - cos pi) dt / V with
    s_ij = 2 E_i E_j / (2 m_e^2); the four yields differ, so a key mapped to the wrong pair
    of photons fails too."""
    dt, k = 0.1, 7
    t_star = k * dt + 0.5 * dt
    cell = (1.0, 1.0, 0.15)
    Ea, wa = [2.0, 3.0], [3.0e5, 5.0e5]
    Eb, wb = [2.0, 4.0], [7.0e5, 2.0e5]
    A = _beam([[0.0, 0.0, -t_star]] * 2, [[0.0, 0.0, e] for e in Ea], Ea, wa)
    B = _beam([[0.0, 0.0, t_star]] * 2, [[0.0, 0.0, -e] for e in Eb], Eb, wb)
    bins_a, bins_b = np.array([3, 7]), np.array([1, 5])
    tab, tot = SO.st_table(A, bins_a, B, bins_b, 11, dt, 0, 20, cell)
    V = cell[0] * cell[1] * cell[2]
    expect = {}
    for i in range(2):
        for j in range(2):
            s = Ea[i] * Eb[j] * 2.0 / (2.0 * ME * ME)
            expect[int(bins_a[i]) * 11 + int(bins_b[j])] = wa[i] * wb[j] * O.sigma(s) * 2.0 * dt / V
    assert sorted(tab) == [34, 38, 78, 82]
    for key, y in expect.items():
        assert tab[key] == pytest.approx(y, rel=1e-13), key
    assert len(set(round(v / max(expect.values()), 12) for v in expect.values())) == 4
    assert tot == pytest.approx(sum(expect.values()), rel=1e-13)
