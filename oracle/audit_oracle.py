"""Sampled estimate of the exact statistical-regime total: the thinning draws and the
Horvitz-Thompson sum written out plainly (numpy, Python integers for the generator).

TEST INFRASTRUCTURE ONLY: used by the test suite, never by the product library.

The exact total of the statistical regime (Sec. 2.2 rate picture) is the sum over query
macro-particles i and target macro-particles j of the cloud-pair yield Y_ij over the steps;
Y_ij is linear in w_i and in w_j. Thinning: macro-particle i of a beam is kept with
probability pi_i; with no control, pi_i = min(1, lambda w_i / W), W the beam's total
weight. A kept macro-particle carries weight w_i / pi_i, so the yield of a kept pair is
Y_ij / (pi_i pi_j), and the sum over kept pairs has expectation sum_ij Y_ij when the two
beams are thinned independently (Horvitz & Thompson 1952).

Draws: Philox4x64-10 (Salmon et al., SC'11) with counter (row, side, 0, 0) and key (seed,
replicate); u = (first output word >> 11) 2^-53; row kept iff u < pi. side 0 is the query
beam, 1 the target.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

from . import kinematics_oracle as K
from . import oracle as O


def inclusion_no_control(w: np.ndarray, lam: float) -> np.ndarray:
    """pi_i = min(1, lambda w_i / W) (0 for w_i <= 0)."""
    W = float(np.sum(w[w > 0.0]))
    p = np.minimum(1.0, lam * (w / W))
    return np.where(w > 0.0, p, 0.0)


def uniforms(n: int, seed: int, rep: int, side: int) -> np.ndarray:
    """u of rows 0 .. n-1 for one replicate and beam side."""
    out = np.empty(n)
    for i in range(n):
        r = K.philox4x64((i, side, 0, 0), (seed, rep))
        out[i] = (r[0] >> 11) * 2.0 ** -53
    return out


def thin(beam: Dict[str, np.ndarray], pi: np.ndarray, u: np.ndarray) -> Tuple[np.ndarray, Dict[str, np.ndarray]]:
    """Kept rows (u < pi) and the thinned beam with weights w / pi."""
    keep = np.nonzero(u < pi)[0]
    out = {k: np.ascontiguousarray(v[keep]) for k, v in beam.items()}
    out["w"] = beam["w"][keep] / pi[keep]
    return keep, out


def ht_total(A, B, pi_a, pi_b, seed: int, rep: int, dt: float, k0: int, n_steps: int, cell):
    """One replicate's estimate with no control: exact cloud-pair yields of the two thinned
    beams (orc_st_pairs) summed. Returns (estimate, kept query rows, kept target rows)."""
    ka, As = thin(A, pi_a, uniforms(len(A["w"]), seed, rep, 0))
    kb, Bs = thin(B, pi_b, uniforms(len(B["w"]), seed, rep, 1))
    if len(ka) == 0 or len(kb) == 0:
        return 0.0, ka, kb
    Y = O.st_pairs(As, Bs, dt, k0, n_steps, cell)
    return float(Y.sum()), ka, kb
