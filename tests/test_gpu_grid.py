"""The uniform-grid broad phase (TRIL_GRID) against the oracle: the same pair sets, first
steps, per-step counts, yields and spectra as the hierarchy, on the workloads of the main
parity tests, at full size on sampled rows, with annihilation, and its limits (one
instance)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1608_01125_amd import beams
from paper_1608_01125_amd import tril as T
from tests.gpu_common import assert_parity, gpu_run, oracle_run

pytestmark = pytest.mark.gpu

EDGES = beams.spectrum_edges()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    return _t


@pytest.mark.parametrize("run", [False, True])
def test_mono_headon_2k(torch, run):
    wl = beams.mono_headon_2k()
    A, B = beams.draw_pair(wl)
    raw, S = oracle_run(A, B, wl.dt, wl.n_steps, EDGES)
    gpu = gpu_run(A, B, wl.dt, wl.n_steps, EDGES, graph=run, flags=T.TRIL_GRID)
    assert S.n_pairs > 20
    assert_parity(gpu, raw, S, wl.n_steps)


@pytest.mark.parametrize("flags", [0, T.TRIL_SORT_QUERIES_ONCE | T.TRIL_TIMING])
def test_gauss_headon_reduced(torch, flags):
    full = beams.gauss_headon_1m()
    wl = beams.gauss_headon_1m(n=20_000, w=full.a.w * 2500.0)
    A, B = beams.draw_pair(wl)
    raw, S = oracle_run(A, B, wl.dt, wl.n_steps, EDGES)
    gpu = gpu_run(A, B, wl.dt, wl.n_steps, EDGES, graph=True, flags=T.TRIL_GRID | flags)
    assert S.n_pairs > 200
    assert_parity(gpu, raw, S, wl.n_steps)


def test_broadband_subsample(torch):
    full = beams.broadband_16m(n=10)
    wl = beams.broadband_16m(n=5000, w=full.a.w * 2e4)
    A, B = beams.draw_pair(wl)
    raw, S = oracle_run(A, B, wl.dt, wl.n_steps, EDGES)
    gpu = gpu_run(A, B, wl.dt, wl.n_steps, EDGES, graph=True, flags=T.TRIL_GRID)
    assert S.n_pairs > 50
    assert_parity(gpu, raw, S, wl.n_steps)


@pytest.mark.parametrize("na,nb", [(0, 10), (10, 0), (0, 0), (1, 1), (1, 500), (500, 1), (2, 2)])
def test_degenerate_sizes(torch, na, nb):
    wl = beams.mono_headon_2k()
    wl = beams.mono_headon_2k(w=wl.a.w * 1e4)
    A, B = beams.draw_pair(wl)
    A, B = beams.head(A, na), beams.head(B, nb)
    raw, S = oracle_run(A, B, wl.dt, wl.n_steps, EDGES)
    gpu = gpu_run(A, B, wl.dt, wl.n_steps, EDGES, graph=True, flags=T.TRIL_GRID)
    assert_parity(gpu, raw, S, wl.n_steps)


def test_full_size_sampled_rows(torch):
    wl = beams.gauss_headon_1m()
    A, B = beams.draw_pair(wl)
    i, j, k, st = gpu_run(A, B, wl.dt, wl.n_steps, EDGES, graph=True, cap=1 << 21,
                          flags=T.TRIL_GRID)
    assert 10_000 < st["n_pairs"] < 40_000
    rng = np.random.default_rng(1)
    rows = np.unique(np.concatenate([rng.choice(np.unique(i), 150, replace=False),
                                     rng.choice(len(A["E"]), 150, replace=False)]))
    raw = O.collide(A, B, wl.dt, wl.n_steps, rows=rows)
    S = O.summarize(raw, A, B, wl.n_steps, EDGES)
    assert raw.knife_margin == 0 and raw.knife_s == 0
    keep = np.isin(i, rows)
    assert np.array_equal(i[keep], S.i) and np.array_equal(j[keep], S.j)
    assert np.array_equal(k[keep], S.first_step)


def test_annihilation_with_grid(torch):
    full = beams.gauss_headon_1m()
    wl = beams.gauss_headon_1m(n=20_000, w=full.a.w * 2500.0)
    A, B = beams.draw_pair(wl)
    raw = O.collide(A, B, wl.dt, wl.n_steps)
    kept = O.annihilate(raw, A, B, wl.dt)
    ctx = T.Context(wl.dt, EDGES, flags=T.TRIL_GRID | T.TRIL_ANNIHILATE)
    try:
        pairs = T.Pairs(1 << 20)
        T.run_steps(ctx, T.Beam(B), T.Beam(A), wl.n_steps, pairs, graph=True)
        st = ctx.stats(pairs)
        gi, gj, gk = pairs.numpy()
    finally:
        ctx.close()
    ko = set(zip(kept.i.tolist(), kept.j.tolist(), kept.k.tolist()))
    assert st["n_hits"] == len(ko) > 100
    assert set(zip(gi.tolist(), gj.tolist(), gk.tolist())) == {(i, j, k) for i, j, k in ko}


def test_instances_not_supported(torch):
    parts_a, parts_b = [], []
    for m in range(2):
        wl = beams.batch64_instance(m)
        A, B = beams.draw_pair(wl)
        parts_a.append(beams.head(A, 100))
        parts_b.append(beams.head(B, 100))
    A, offA = beams.concat(parts_a)
    B, offB = beams.concat(parts_b)
    ctx = T.Context(0.1, EDGES, flags=T.TRIL_GRID)
    try:
        with pytest.raises(T.TrilError) as e:
            T.run_steps(ctx, T.Beam(B, offB), T.Beam(A, offA), 3, T.Pairs(64), graph=True)
        assert e.value.code == T.TRIL_E_NOTIMPL
    finally:
        ctx.close()
