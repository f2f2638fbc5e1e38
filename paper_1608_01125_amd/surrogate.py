"""Surrogate workflow of the statistical regime: training rows from the exact path,
training of the network ensemble, and the surrogate path with its exact fallback.

Every computation runs in libtril's kernels (tril_st_bin, tril_st_exact,
tril_st_features, tril_st_targets, tril_mlp_*, tril_st_calibrate, tril_st_audit,
tril_st_surrogate); this module only sequences the calls and holds device buffers.

The surrogate works on pairs of position cells of the 32^3 grid: the grids given to it
have one energy and one angle bin, and energy and direction enter as each cell's
weighted means (the features E_a, E_b and the angle). With 16 x 8 energy x angle bins
per cell the bin pairs would outnumber the macro-particle pairs they stand for."""
from __future__ import annotations

from dataclasses import replace
from typing import List, Tuple

from . import beams
from . import tril as T


def cell_grid(wl: beams.Workload, which: str, beam) -> beams.StGridSpec:
    """Position-cell grid of one beam (32^3 cells, one energy and one angle bin)."""
    return replace(beams.st_grid(wl, which, beam), n_e=1, n_th=1)


def bin_device(beam: T.Beam, grid) -> Tuple["object", "object"]:
    import torch
    bins = torch.empty(max(beam.n, 1), dtype=torch.int32, device="cuda")
    sums = torch.zeros((grid.n_bins, 8), dtype=torch.float64, device="cuda")
    T.tril_st_bin(beam, grid, bins, sums)
    return bins, sums


class Instance:
    """One collision in the statistical regime, resident on the device."""

    def __init__(self, wl: beams.Workload, A=None, B=None):
        if A is None:
            A, B = beams.draw_pair(wl)
        self.wl = wl
        self.qa, self.tb = T.Beam(A), T.Beam(B)
        self.ga, self.gb = cell_grid(wl, "a", A), cell_grid(wl, "b", B)
        self.qbins, self.qsums = bin_device(self.qa, self.ga)
        self.tbins, self.tsums = bin_device(self.tb, self.gb)

    def exact(self, ctx: T.Context, cap_log2: int = 0):
        """Exact cell-pair yields (table) and their total. cap_log2 = 0: a table size that
        grows with the instance (2^22 slots up to 2.5e5 macro-particles per beam, 2^24
        above)."""
        if cap_log2 <= 0:
            cap_log2 = 22 if self.wl.a.n <= 250_000 else 24
        tab = T.StTable(cap_log2)
        tot = T.tril_st_exact(ctx, self.tb, self.tbins, self.gb.n_bins, self.qa, self.qbins,
                              self.ga.cell, 0, self.wl.n_steps, tab)
        return tab, tot

    def exact_depleted(self, ctx: T.Context, cap_log2: int = 22, pair_log2: int = 24):
        """Depleted cell-pair yields (table), per-cloud-pair yields (pair table), total."""
        tab, pt = T.StTable(cap_log2), T.StTable(pair_log2)
        tot = T.tril_st_exact_depleted(ctx, self.tb, self.tbins, self.gb.n_bins, self.qa,
                                       self.qbins, self.ga.cell, 0, self.wl.n_steps, pt, tab)
        return tab, pt, tot

    def features(self, ctx: T.Context, params=None):
        return T.tril_st_features(ctx, self.qsums, self.ga, self.tsums, self.gb, 0,
                                  self.wl.n_steps, params)

    def audit(self, ctx: T.Context, net, control: int, n_sample: int = 0, n_rep: int = 0,
              seed: int = 0, mix: float = 0.0, sur=None) -> dict:
        """Sampled estimate of the exact total (tril_st_audit) with the given control."""
        return T.tril_st_audit(ctx, net, self.tb, self.tbins, self.tsums, self.gb, self.qa,
                               self.qbins, self.qsums, self.ga, 0, self.wl.n_steps, control,
                               n_sample, n_rep, seed, mix, sur)

    def surrogate(self, ctx: T.Context, net: T.Mlp, params=None) -> dict:
        return T.tril_st_surrogate(ctx, net, self.tb, self.tbins, self.tsums, self.gb, self.qa,
                                   self.qbins, self.qsums, self.ga, 0, self.wl.n_steps, params)


def training_rows(ctx: T.Context, insts: List[Instance], eps: float = 1e-3, log=None):
    """Features and targets log((Y + eps Y0) / Y0) of every candidate cell pair of the
    instances, concatenated on the device, with their Y0 and exact Y."""
    import torch
    xs, ts, y0s, ys = [], [], [], []
    for n, inst in enumerate(insts):
        tab, _ = inst.exact(ctx)
        if log is not None:
            log(f"training instance {n + 1}/{len(insts)}: exact yields done")
        x, y0, key = inst.features(ctx, T.sur_params(eps=eps))
        t, y = T.tril_st_targets(key, y0, tab, eps)
        xs.append(x), ts.append(t), y0s.append(y0), ys.append(y)
    return torch.cat(xs), torch.cat(ts), torch.cat(y0s), torch.cat(ys)


def train(net: T.Mlp, x, t, n_steps: int = 3000, batch: int = 4096, lr: float = 1e-3,
          seed: int = 0):
    net.fit_norm(x, t)
    return net.train(x, t, n_steps, batch, lr, seed)


def yield_scale(net: T.Mlp, x, y0, y, eps: float = 1e-3) -> float:
    """Exact over predicted total yield on training rows (tril_st_calibrate): the network
    fits the mean of log((Y + eps Y0) / Y0), whose exponential falls short of the mean
    ratio."""
    return T.tril_st_calibrate(net, x, y0, y, eps)
