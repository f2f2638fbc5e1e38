"""Builds the hand-derived two-photon scenarios of golden/two_photon_cases.json.

The collision radius is computed here from the paper's literal cross-section
formula (Sec. 1, Eq. 1) in 50-digit arithmetic, with no code shared with either
the oracle or the GPU library.
"""
from __future__ import annotations

import json
import os

import mpmath as mp
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ME = "0.51099895000"      # MeV, CODATA 2018
RE = "2.8179403262e-9"    # um, CODATA 2018


def sigma_literal(s) -> mp.mpf:
    """Eq. 1 exactly as printed: (pi/2) r_e^2 (1-b^2) [-2b(2-b^2) + (3-b^4) ln((1+b)/(1-b))]."""
    with mp.workdps(max(50, mp.mp.dps)):
        s = mp.mpf(s)
        if s <= 1:
            return mp.mpf(0)
        re = mp.mpf(RE)
        b = mp.sqrt(1 - 1 / s)
        return mp.pi / 2 * re ** 2 * (1 - b ** 2) * (
            -2 * b * (2 - b ** 2) + (3 - b ** 4) * mp.log((1 + b) / (1 - b)))


def invariant_exact(Ea, Eb, cos_phi) -> mp.mpf:
    with mp.workdps(50):
        me = mp.mpf(ME)
        return mp.mpf(Ea) * mp.mpf(Eb) * (1 - mp.mpf(cos_phi)) / (2 * me ** 2)


def _energy(v):
    if v == "m_e":
        return float(ME)
    if isinstance(v, str):
        assert v == "m_e*sqrt(1+1e-6)"
        with mp.workdps(50):
            return float(mp.mpf(ME) * mp.sqrt(1 + mp.mpf("1e-6")))
    return float(v)


def load_cases():
    with open(os.path.join(HERE, "golden", "two_photon_cases.json")) as f:
        return json.load(f)["cases"]


def build_case(c):
    """Return (A, B, dt, n_steps, expected_steps) as one-photon beams."""
    Ea, Eb = _energy(c["E_A"]), _energy(c["E_B"])
    geo = c["geometry"]
    cos_phi = {"head_on": -1.0, "ninety": 0.0, "separating": -1.0, "co_moving": 1.0}[geo]
    s = invariant_exact(Ea, Eb, cos_phi)
    with mp.workdps(50):
        r = mp.sqrt(mp.sqrt(mp.mpf(c["w_A"]) * mp.mpf(c["w_B"])) * sigma_literal(s) / mp.pi)
    b = float(c["b_over_r"] * r)
    z = float(c["z_start"])
    if geo == "head_on":
        pa, ua = (0.0, 0.0, -z), (0.0, 0.0, 1.0)
        pb, ub = (b, 0.0, z), (0.0, 0.0, -1.0)
    elif geo == "ninety":
        pa, ua = (0.0, 0.0, -z), (0.0, 0.0, 1.0)
        pb, ub = (-z, b, 0.0), (1.0, 0.0, 0.0)
    elif geo == "separating":
        pa, ua = (0.0, 0.0, z), (0.0, 0.0, 1.0)
        pb, ub = (b, 0.0, -z), (0.0, 0.0, -1.0)
    elif geo == "co_moving":
        pa, ua = (0.0, 0.0, 0.0), (0.0, 0.0, 1.0)
        pb, ub = (b, 0.0, 0.0), (0.0, 0.0, 1.0)
    else:
        raise ValueError(geo)

    def beam(p, u, E, w):
        return {"x": np.array([p[0]]), "y": np.array([p[1]]), "z": np.array([p[2]]),
                "px": np.array([E * u[0]]), "py": np.array([E * u[1]]),
                "pz": np.array([E * u[2]]), "E": np.array([E]), "w": np.array([float(w)])}

    A = beam(pa, ua, Ea, c["w_A"])
    B = beam(pb, ub, Eb, c["w_B"])
    return A, B, float(c["dt"]), int(c["n_steps"]), list(c["expect_steps"])
