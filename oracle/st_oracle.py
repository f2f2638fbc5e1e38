"""Statistical (cloud) regime oracle: binning and bin-pair yields, plain numpy + the C
oracle's per-pair yields (oracle/tril_oracle.c, orc_st_pairs).

TEST INFRASTRUCTURE ONLY: used by the test suite and the benchmark's CPU baseline,
never by the product library.

Binning (one beam, grid g): position cell of X(t_bin) = x0 + t_bin p/E in the box
[lo, hi] with n_pos cells per axis; energy bin log-spaced on [e_lo, e_hi] (n_e bins);
polar-angle bin of the direction about the unit axis on [0, th_max] (n_th bins);
out-of-range values fall in the edge bin; bin = (((ix ny + iy) nz + iz) n_e + ie) n_th + ith.
Each index is floor(fraction of the range x number of bins), evaluated in FP64 in that
order: ((X - lo) / (hi - lo)) n, (log(E / e_lo) / log(e_hi / e_lo)) n_e,
(acos(u.axis / |u|) / th_max) n_th.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, Optional, Tuple

import numpy as np

from . import oracle as O


@dataclass
class Grid:
    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]
    n_pos: Tuple[int, int, int]
    n_e: int
    e_lo: float
    e_hi: float
    n_th: int
    th_max: float
    axis: Tuple[float, float, float]
    t_bin: float

    @property
    def n_bins(self) -> int:
        return int(np.prod(self.n_pos)) * self.n_e * self.n_th

    @property
    def cell(self) -> np.ndarray:
        return (np.asarray(self.hi) - np.asarray(self.lo)) / np.asarray(self.n_pos)


def _cell(v: np.ndarray, n: int) -> np.ndarray:
    f = np.floor(v)
    f = np.where(np.isnan(f), 0.0, f)
    return np.clip(f, 0, n - 1).astype(np.int64)


def bin_beam(beam: Dict[str, np.ndarray], g: Grid) -> Tuple[np.ndarray, np.ndarray]:
    """Bin index per photon and per-bin sums (w, w E, w ux, w uy, w uz, w X, w Y, w Z
    with X the position at t_bin) as a dict {bin: 8-vector} over occupied bins."""
    E = beam["E"]
    u = np.stack([beam["px"] / E, beam["py"] / E, beam["pz"] / E], axis=1)
    X = np.stack([beam["x"], beam["y"], beam["z"]], axis=1) + g.t_bin * u
    ip = [_cell(((X[:, a] - g.lo[a]) / (g.hi[a] - g.lo[a])) * g.n_pos[a], g.n_pos[a]) for a in range(3)]
    ie = _cell((np.log(E / g.e_lo) / np.log(g.e_hi / g.e_lo)) * g.n_e, g.n_e)
    uu = (u[:, 0] * u[:, 0] + u[:, 1] * u[:, 1]) + u[:, 2] * u[:, 2]
    cth = ((u[:, 0] * g.axis[0] + u[:, 1] * g.axis[1]) + u[:, 2] * g.axis[2]) / np.sqrt(uu)
    cth = np.clip(cth, -1.0, 1.0)
    ith = _cell((np.arccos(cth) / g.th_max) * g.n_th, g.n_th)
    b = (((ip[0] * g.n_pos[1] + ip[1]) * g.n_pos[2] + ip[2]) * g.n_e + ie) * g.n_th + ith
    w = beam["w"]
    vals = np.stack([w, w * E, w * u[:, 0], w * u[:, 1], w * u[:, 2],
                     w * X[:, 0], w * X[:, 1], w * X[:, 2]], axis=1)
    occ, inv = np.unique(b, return_inverse=True)
    sums = np.zeros((len(occ), 8))
    np.add.at(sums, inv, vals)
    return b.astype(np.int64), dict(zip(occ.tolist(), sums))


def bin_margin(beam: Dict[str, np.ndarray], g: Grid) -> np.ndarray:
    """Distance of each photon's bin coordinates from the nearest bin edge (in units of
    one bin): photons closer than ~1e-12 are knife-edge cases where rounding of log and
    acos on two platforms may pick different bins."""
    E = beam["E"]
    u = np.stack([beam["px"] / E, beam["py"] / E, beam["pz"] / E], axis=1)
    X = np.stack([beam["x"], beam["y"], beam["z"]], axis=1) + g.t_bin * u
    parts = [((X[:, a] - g.lo[a]) / (g.hi[a] - g.lo[a])) * g.n_pos[a] for a in range(3)]
    parts.append((np.log(E / g.e_lo) / np.log(g.e_hi / g.e_lo)) * g.n_e)
    uu = (u[:, 0] * u[:, 0] + u[:, 1] * u[:, 1]) + u[:, 2] * u[:, 2]
    cth = np.clip(((u[:, 0] * g.axis[0] + u[:, 1] * g.axis[1]) + u[:, 2] * g.axis[2]) / np.sqrt(uu), -1, 1)
    parts.append((np.arccos(cth) / g.th_max) * g.n_th)
    return np.min([np.abs(p - np.round(p)) for p in parts], axis=0)


def st_table(A, bins_a, B, bins_b, n_bins_b: int, dt: float, k0: int, n_steps: int, cell,
             rows: Optional[np.ndarray] = None) -> Tuple[Dict[int, float], float]:
    """Bin-pair yields {bin_a * n_bins_b + bin_b: Y} and the total, from the per-pair
    yields of the C oracle (query beam A, target beam B)."""
    Y = O.st_pairs(A, B, dt, k0, n_steps, cell, rows=rows)
    ra = bins_a if rows is None else bins_a[rows]
    keys = ra[:, None] * n_bins_b + bins_b[None, :]
    nz = Y > 0.0
    k = keys[nz]
    v = Y[nz]
    uk, inv = np.unique(k, return_inverse=True)
    tot = np.zeros(len(uk))
    np.add.at(tot, inv, v)
    return dict(zip(uk.tolist(), tot.tolist())), float(Y.sum())


# --------------------------------------------------------------------------------------
# Depletion (Sec. 2.2, the rate equation with the loss of collision partners). Two clouds of
# densities n_I(0), n_II(0) create pairs at the rate dn/dt = k (n_I(0) - n)(n_II(0) - n), with
# n0 = n_I(0) + n_II(0) and alpha = n_I(0) / n0. The printed reactivity 2 pi sigma c is read as
# k = sigma c (1 - cos phi), the factor the closed form n_alpha carries (the two printed
# closed forms use different constants; both solve the same equation).
#
# Per cloud pair the overlap changes from step to step. With the densities of the shared
# volume depleted only by the pair's own creations, the equation is autonomous in n with the
# rate scaled by V_ov(t) / V, so its solution is the closed form at the pair's exposure
#   k tau -> S = sum_k sigma (1 - cos phi) dt V_ov(t_k) / V      (orc_st_exposure),
# and the pair's depleted yield (physical pairs) is V n(S).
# --------------------------------------------------------------------------------------


def n_half(n0: float, k_tau: float) -> float:
    """Closed form for equal densities (alpha = 1/2): (n0/2)^2 k tau / (1 + (n0/2) k tau)."""
    h = n0 / 2.0
    return (h * h * k_tau) / (1.0 + h * k_tau)


def n_alpha(n0: float, alpha: float, k_tau: float) -> float:
    """Closed form for alpha != 1/2: (alpha - 1) alpha n0 (1 - e^X) / (alpha e^X + alpha - 1),
    X = n0 (2 alpha - 1) k tau, with e^X written as 1 + expm1(X) (the same expression; it
    keeps the small-X regime, where 1 - e^X cancels, at full precision)."""
    X = n0 * (2.0 * alpha - 1.0) * k_tau
    E = np.expm1(X)
    return ((alpha - 1.0) * alpha * n0 * (-E)) / (alpha * E + (2.0 * alpha - 1.0))


def depleted_density(a: float, b: float, k_tau: float) -> float:
    """Pair density created by two clouds of densities a and b at exposure k tau. The equation
    is symmetric in a and b; alpha is taken as the smaller share so that X <= 0 (e^X never
    overflows)."""
    if a <= 0.0 or b <= 0.0 or k_tau <= 0.0:
        return 0.0
    n0 = a + b
    if a == b:
        return n_half(n0, k_tau)
    return n_alpha(n0, min(a, b) / n0, k_tau)


def st_depleted_pairs(A, B, dt: float, k0: int, n_steps: int, cell,
                      rows: Optional[np.ndarray] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Depleted yield and exposure of every (query row, target photon) cloud pair: (Y, S),
    shape (rows, n_B); Y = V n(w_i / V, w_j / V, S)."""
    S = O.st_exposure(A, B, dt, k0, n_steps, cell, rows=rows)
    V = (cell[0] * cell[1]) * cell[2]
    wa = A["w"] if rows is None else A["w"][rows]
    Y = np.zeros_like(S)
    for a, b in zip(*np.nonzero(S > 0.0)):
        Y[a, b] = V * depleted_density(wa[a] / V, B["w"][b] / V, S[a, b])
    return Y, S


def st_depleted_table(A, bins_a, B, bins_b, n_bins_b: int, dt: float, k0: int, n_steps: int,
                      cell) -> Tuple[Dict[int, float], float, Dict[int, float]]:
    """Bin-pair depleted yields {bin_a * n_bins_b + bin_b: Y}, their total, and the per-pair
    yields {i * n_B + j: Y} (pairs with a positive exposure whose rows both have a bin)."""
    Y, S = st_depleted_pairs(A, B, dt, k0, n_steps, cell)
    keys = bins_a[:, None].astype(np.int64) * n_bins_b + bins_b[None, :]
    ok = (S > 0.0) & (bins_a[:, None] >= 0) & (bins_b[None, :] >= 0)
    tab: Dict[int, float] = {}
    for k, v in zip(keys[ok].tolist(), Y[ok].tolist()):
        tab[k] = tab.get(k, 0.0) + v
    ia, jb = np.nonzero(ok)
    pairs = {int(i) * len(B["E"]) + int(j): float(Y[i, j]) for i, j in zip(ia, jb)}
    return tab, float(sum(pairs.values())), pairs
