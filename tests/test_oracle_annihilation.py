"""Pins of the oracle's annihilation mode (CPU): photons that collide are consumed, and the
collisions of a step are taken in chronological order (time of closest approach inside the
step, then i, then j). Hand-built crossings with known times, the matching and maximality
invariants of the chronological greedy, and its equality with a literal step-by-step
simulation that removes consumed photons before the next step."""
import math

import numpy as np
import pytest

from oracle import oracle as O

ME = 0.51099895


def _axis_beams(a_z, b_z, E=2.0, r=0.005, b_x=None):
    """A photons on the z axis at a_z moving +z, B photons at b_z moving -z (optionally
    shifted to x = b_x), weights giving collision radius r for the head-on invariant.
    A pair on the axis meets at t* = (b_z - a_z) / 2 and is within r of each other for
    |t - t*| <= r / 2."""
    s = E * E / (ME * ME)
    w = math.pi * r * r / O.sigma(s)
    na, nb = len(a_z), len(b_z)
    bx = np.zeros(nb) if b_x is None else np.asarray(b_x, float)
    A = {"x": np.zeros(na), "y": np.zeros(na), "z": np.asarray(a_z, float),
         "px": np.zeros(na), "py": np.zeros(na), "pz": np.full(na, E),
         "E": np.full(na, E), "w": np.full(na, w)}
    B = {"x": bx, "y": np.zeros(nb), "z": np.asarray(b_z, float),
         "px": np.zeros(nb), "py": np.zeros(nb), "pz": np.full(nb, -E),
         "E": np.full(nb, E), "w": np.full(nb, w)}
    return A, B


def _kept(A, B, dt, n_steps):
    raw = O.collide(A, B, dt, n_steps, strict=True)
    kept = O.annihilate(raw, A, B, dt)
    return raw, {(int(i), int(j), int(k)) for i, j, k in zip(kept.i, kept.j, kept.k)}


def test_earliest_collision_in_a_step_wins():
    """Crossing times 0.44 (A0 B0), 0.41 (A0 B1), 0.46 (A1 B0), 0.43 (A1 B1), all in step 4
    of dt = 0.1: A0-B1 comes first and consumes A0 and B1, so A1-B1 (0.43) and A0-B0 (0.44)
    are dropped and A1-B0 (0.46), the latest, is kept."""
    A, B = _axis_beams([0.0, -0.04], [0.88, 0.82])
    raw, kept = _kept(A, B, 0.1, 10)
    assert sorted(zip(raw.i.tolist(), raw.j.tolist(), raw.k.tolist())) == \
        [(0, 0, 4), (0, 1, 4), (1, 0, 4), (1, 1, 4)]
    tau = O.hit_tau(raw, A, B, 0.1)
    order = {(int(i), int(j)): t for i, j, t in zip(raw.i, raw.j, tau)}
    assert order[(0, 1)] == pytest.approx(0.01, abs=1e-12)
    assert order[(1, 0)] == pytest.approx(0.06, abs=1e-12)
    assert kept == {(0, 1, 4), (1, 0, 4)}


def test_photon_consumed_in_an_earlier_step_is_gone():
    """A0 meets B0 in step 2 (t = 0.25) and B1 in step 6 (0.65); A1 meets B0 in step 7 (0.75)
    and B1 in step 11 (1.15). A0-B0 consumes both, so the step-6 and step-7 hits are dropped
    and A1-B1 is kept."""
    A, B = _axis_beams([0.0, -1.0], [0.5, 1.3])
    raw, kept = _kept(A, B, 0.1, 14)
    assert sorted(zip(raw.i.tolist(), raw.j.tolist(), raw.k.tolist())) == \
        [(0, 0, 2), (0, 1, 6), (1, 0, 7), (1, 1, 11)]
    assert kept == {(0, 0, 2), (1, 1, 11)}


def test_simultaneous_collisions_ordered_by_index():
    """Two target photons at the same place meet A0 at the same instant: equal tau*, so the
    lower target index is taken."""
    A, B = _axis_beams([0.0], [0.5, 0.5])
    raw, kept = _kept(A, B, 0.1, 6)
    tau = O.hit_tau(raw, A, B, 0.1)
    assert len(raw.i) == 2 and tau[0] == tau[1]
    assert kept == {(0, 0, 2)}


def _dense(seed, n=40, steps=24):
    """Head-on bunches of n photons in a 0.2 um wide, 0.6 um long region with radii of
    tens of nm: every photon has several partners over the run."""
    rng = np.random.default_rng(seed)
    E = rng.uniform(1.5, 3.0, size=(2, n))
    def beam(sign, E):
        d = rng.normal(size=(n, 3)) * 0.02
        d[:, 2] = sign
        d /= np.linalg.norm(d, axis=1)[:, None]
        x = rng.uniform(-0.1, 0.1, size=(n, 3))
        x[:, 2] = rng.uniform(-0.3, 0.3, n) - sign * 0.6
        return {"x": x[:, 0].copy(), "y": x[:, 1].copy(), "z": x[:, 2].copy(),
                "px": d[:, 0] * E, "py": d[:, 1] * E, "pz": d[:, 2] * E, "E": E.copy(),
                "w": rng.uniform(0.5, 2.0, n) * 1e15}
    return beam(1.0, E[0]), beam(-1.0, E[1]), 0.05, steps


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_kept_hits_are_a_maximal_chronological_matching(seed):
    A, B, dt, steps = _dense(seed)
    raw = O.collide(A, B, dt, steps, strict=True)
    kept = O.annihilate(raw, A, B, dt)
    assert len(raw.i) > 2 * len(kept.i) > 0  # many conflicts
    # a matching: every photon at most once
    assert len(set(kept.i.tolist())) == len(kept.i)
    assert len(set(kept.j.tolist())) == len(kept.j)
    # every dropped hit meets a kept hit of one of its photons that comes no later
    tau = O.hit_tau(raw, A, B, dt)
    key = {(int(i), int(j), int(k)): (int(k), float(t), int(i), int(j))
           for i, j, k, t in zip(raw.i, raw.j, raw.k, tau)}
    kset = set(zip(kept.i.tolist(), kept.j.tolist(), kept.k.tolist()))
    by_a = {i: key[(i, j, k)] for i, j, k in kset}
    by_b = {j: key[(i, j, k)] for i, j, k in kset}
    for h, kh in key.items():
        if h in kset:
            continue
        i, j, _ = h
        assert (i in by_a and by_a[i] < kh) or (j in by_b and by_b[j] < kh)


@pytest.mark.parametrize("seed", [4, 5])
def test_equal_to_step_by_step_removal(seed):
    """The same process run literally: each step collides only the photons not yet
    consumed, resolves that step's hits in order of (tau*, i, j), and removes the photons
    of the kept hits before the next step."""
    A, B, dt, steps = _dense(seed)
    raw = O.collide(A, B, dt, steps, strict=True)
    kept = O.annihilate(raw, A, B, dt)
    alive_a = np.ones(len(A["E"]), bool)
    alive_b = np.ones(len(B["E"]), bool)
    lit = set()
    for k in range(steps):
        ra, rb = np.nonzero(alive_a)[0], np.nonzero(alive_b)[0]
        Bs = {c: v[rb] for c, v in B.items()}
        hk = O.collide(A, Bs, dt, 1, rows=ra, k0=k, strict=True)
        hk.j = rb[hk.j]  # back to rows of B
        tk = O.hit_tau(hk, A, B, dt)
        for h in sorted(range(len(hk.i)), key=lambda h: (tk[h], int(hk.i[h]), int(hk.j[h]))):
            i, j = int(hk.i[h]), int(hk.j[h])
            if alive_a[i] and alive_b[j]:
                alive_a[i] = alive_b[j] = False
                lit.add((i, j, k))
    assert lit == set(zip(kept.i.tolist(), kept.j.tolist(), kept.k.tolist()))
    assert len(lit) > 5
