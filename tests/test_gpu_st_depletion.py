"""Depletion of cloud pairs in the statistical regime on the GPU against the oracle: per
cloud pair (exposure -> closed-form yield) and per bin pair, at a physical photon number where
nothing is depleted and at one where most pairs saturate, with equal and unequal weights,
several step batches, ragged instances, and table overflow."""
import numpy as np
import pytest

from oracle import st_oracle as SO
from paper_1608_01125_amd import beams
from paper_1608_01125_amd import tril as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    return _t


def _bins(torch, beam_np, grid, offs=None):
    b = T.Beam(beam_np, offs)
    bins = torch.empty(max(b.n, 1), dtype=torch.int32, device="cuda")
    T.tril_st_bin(b, grid, bins, None)
    torch.cuda.synchronize()
    return b, bins


def _grids(wl, A, B):
    return beams.st_grid(wl, "a", A), beams.st_grid(wl, "b", B)


def _gpu(torch, A, B, wl, k0, n_steps, grids, offA=None, offB=None, cap_log2=20, pair_log2=22,
         linear=False, **kw):
    ga, gb = grids
    qa, qbins = _bins(torch, A, ga, offA)
    tb, tbins = _bins(torch, B, gb, offB)
    ctx = T.Context(wl.dt, None, **kw)
    tab, pt = T.StTable(cap_log2), T.StTable(pair_log2)
    try:
        tot = T.tril_st_exact_depleted(ctx, tb, tbins, gb.n_bins, qa, qbins, ga.cell, k0, n_steps,
                                       pt, tab)
        lin = None
        if linear:
            lt = T.StTable(cap_log2)
            ltot = T.tril_st_exact(ctx, tb, tbins, gb.n_bins, qa, qbins, ga.cell, k0, n_steps, lt)
            lin = (lt.items(), ltot)
    finally:
        ctx.close()
    return tab.items(), pt.items(), tot, lin


def _oracle(A, B, wl, k0, n_steps, grids, offA=None, offB=None):
    ga, gb = grids
    ba, _ = SO.bin_beam(A, ga)
    bb, _ = SO.bin_beam(B, gb)
    if offA is None:
        return SO.st_depleted_table(A, ba, B, bb, gb.n_bins, wl.dt, k0, n_steps, ga.cell)
    tab, tot, pairs = {}, 0.0, {}
    nB = len(B["E"])
    for m in range(len(offA) - 1):
        Am = {k: v[offA[m]:offA[m + 1]] for k, v in A.items()}
        Bm = {k: v[offB[m]:offB[m + 1]] for k, v in B.items()}
        if len(Am["E"]) == 0 or len(Bm["E"]) == 0:
            continue
        t, s, p = SO.st_depleted_table(Am, ba[offA[m]:offA[m + 1]], Bm, bb[offB[m]:offB[m + 1]],
                                       gb.n_bins, wl.dt, k0, n_steps, ga.cell)
        for k, v in t.items():
            tab[k] = tab.get(k, 0.0) + v
        nBm = len(Bm["E"])
        for k, v in p.items():
            i, j = divmod(k, nBm)
            pairs[(offA[m] + i) * nB + offB[m] + j] = v
        tot += s
    return tab, tot, pairs


def _assert_table(items, ref, rel=1e-9):
    keys, ys = items
    rk = np.array(sorted(ref), dtype=np.int64)
    assert np.array_equal(keys, rk)
    np.testing.assert_allclose(ys, np.array([ref[k] for k in rk]), rtol=rel, atol=0)


def _draw(physical, unequal, n=2000, seed=0):
    wl = beams.st_headon(n, physical=physical, seed=seed)
    A, B = beams.draw_pair(wl)
    if unequal:
        rng = np.random.default_rng(11)
        A["w"] = A["w"] * rng.uniform(0.5, 2.0, len(A["w"]))
        B["w"] = B["w"] * rng.uniform(0.5, 2.0, len(B["w"]))
    return wl, A, B


@pytest.mark.parametrize("physical,unequal,step_batch", [
    (1e9, False, 0), (1e20, False, 0), (1e20, True, 7), (1e22, True, 0), (3e18, True, 1)])
def test_depleted_matches_oracle(torch, physical, unequal, step_batch):
    """2000 macro-particles per beam, the 100 steps around the crossing. At 1e9 photons per
    beam nothing is visibly depleted (1e-11 of the linear yield); 3e18 removes 2%, 1e20 about
    a third, 1e22 saturates most overlapping pairs."""
    wl, A, B = _draw(physical, unequal)
    grids = _grids(wl, A, B)
    ref, ref_tot, ref_pairs = _oracle(A, B, wl, 150, 100, grids)
    items, pitems, tot, lin = _gpu(torch, A, B, wl, 150, 100, grids, step_batch=step_batch,
                                   linear=True)
    assert len(ref) > 200 and len(ref_pairs) > 1000
    _assert_table(items, ref)
    _assert_table(pitems, ref_pairs)
    assert abs(tot - ref_tot) <= 1e-9 * ref_tot
    # never above the linear yield; equal to it when nothing is depleted
    (lk, ly), ltot = lin
    assert np.array_equal(lk, items[0])
    assert np.all(items[1] <= ly * (1 + 1e-12))
    ratio = tot / ltot
    if physical == 1e9:
        assert ratio > 1 - 1e-6
    elif physical == 3e18:
        assert 0.95 < ratio < 0.995
    else:
        assert ratio < 0.75


def test_depleted_instances(torch):
    parts_a, parts_b = [], []
    for m, (na, nb) in enumerate([(800, 600), (0, 300), (500, 1), (700, 900)]):
        wl = beams.st_headon(1000, physical=1e20, seed=m)
        A, B = beams.draw_pair(wl)
        parts_a.append(beams.head(A, na))
        parts_b.append(beams.head(B, nb))
    A, offA = beams.concat(parts_a)
    B, offB = beams.concat(parts_b)
    wl = beams.st_headon(1000, physical=1e20)
    grids = _grids(wl, A, B)
    ref, ref_tot, ref_pairs = _oracle(A, B, wl, 170, 60, grids, offA, offB)
    items, pitems, tot, _ = _gpu(torch, A, B, wl, 170, 60, grids, offA, offB)
    assert len(ref) > 50
    _assert_table(items, ref)
    _assert_table(pitems, ref_pairs)
    assert abs(tot - ref_tot) <= 1e-9 * ref_tot


def test_pair_table_overflow_reported(torch):
    wl, A, B = _draw(1e20, False)
    with pytest.raises(T.TrilError) as e:
        _gpu(torch, A, B, wl, 150, 100, _grids(wl, A, B), pair_log2=4)
    assert e.value.code == T.TRIL_E_OVERFLOW


def test_depleted_benchmark_size_sampled_rows(torch):
    """The benchmark's depletion configuration (2e4 macro-particles per beam, 1e20 photons,
    all 400 steps): the per-cloud-pair yields of 40 sampled query rows against the oracle."""
    wl = beams.st_headon(20_000, physical=1e20)
    A, B = beams.draw_pair(wl)
    grids = _grids(wl, A, B)
    items, pitems, tot, _ = _gpu(torch, A, B, wl, 0, wl.n_steps, grids, cap_log2=23, pair_log2=25)
    keys, ys = pitems
    nB = len(B["E"])
    rows = np.sort(np.random.default_rng(2).choice(len(A["E"]), 40, replace=False))
    ga, _ = grids
    Y, S = SO.st_depleted_pairs(A, B, wl.dt, 0, wl.n_steps, ga.cell, rows=rows)
    ba, _ = SO.bin_beam(A, grids[0])
    bb, _ = SO.bin_beam(B, grids[1])
    ref = {}
    for a, r in enumerate(rows):
        for j in np.nonzero((S[a] > 0) & (bb >= 0))[0]:
            if ba[r] >= 0:
                ref[int(r) * nB + int(j)] = float(Y[a, j])
    sel = np.isin(keys // nB, rows)
    got = dict(zip(keys[sel].tolist(), ys[sel].tolist()))
    assert len(ref) > 100 and set(got) == set(ref)
    for k, v in ref.items():
        assert abs(got[k] - v) <= 1e-9 * v
