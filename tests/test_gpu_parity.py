"""End-to-end parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

The colliding-pair set, each pair's first step and the per-step hit counts must be
identical; yield and spectrum sums agree to far better than 1e-6 relative (they
add identical per-pair terms in a different order)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1608_01125_amd import beams
from paper_1608_01125_amd import tril as T
from tests.golden_cases import build_case, load_cases
from tests.gpu_common import assert_parity, gpu_run, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    return _t


EDGES = beams.spectrum_edges()


@pytest.mark.parametrize("case", load_cases(), ids=lambda c: c["name"])
def test_golden_two_photon(torch, case):
    A, B, dt, n_steps, expect = build_case(case)
    i, j, k, st = gpu_run(A, B, dt, n_steps, EDGES)
    assert st["n_hits"] == len(expect)
    assert list(st["step_counts"].nonzero()[0]) == expect


@pytest.mark.parametrize("graph", [False, True])
def test_mono_headon_2k_full(torch, graph):
    wl = beams.mono_headon_2k()
    A, B = beams.draw_pair(wl)
    raw, S = oracle_run(A, B, wl.dt, wl.n_steps, EDGES)
    gpu = gpu_run(A, B, wl.dt, wl.n_steps, EDGES, graph=graph)
    assert S.n_pairs > 20
    assert_parity(gpu, raw, S, wl.n_steps)


def _gauss_small(n, boost, seed=0):
    full = beams.gauss_headon_1m(seed=seed)
    wl = beams.gauss_headon_1m(seed=seed, n=n, w=full.a.w * boost)
    A, B = beams.draw_pair(wl)
    return wl, A, B


@pytest.mark.parametrize("graph,flags", [(False, 0), (True, 0), (True, T.TRIL_SORT_QUERIES_ONCE)])
def test_gauss_headon_reduced_all_steps(torch, graph, flags):
    """20k photons per beam, weight raised 2500x so that the reduced beams collide about
    as often per photon as the full 1e6 beams; all 400 steps."""
    wl, A, B = _gauss_small(20_000, 2500.0)
    raw, S = oracle_run(A, B, wl.dt, wl.n_steps, EDGES)
    gpu = gpu_run(A, B, wl.dt, wl.n_steps, EDGES, graph=graph, flags=flags)
    assert S.n_pairs > 200
    assert_parity(gpu, raw, S, wl.n_steps)


@pytest.mark.parametrize("step_batch,flags,morton", [
    (1, 0, 0), (7, 0, 0), (64, T.TRIL_TIMING, 0), (0, T.TRIL_SORT_QUERIES_ONCE, 0),
    (13, T.TRIL_SORT_QUERIES_ONCE | T.TRIL_TIMING, 0), (400, 0, 0), (16, 0, 12),
    (9, T.TRIL_SORT_QUERIES_ONCE, 3), (64, T.TRIL_TIMING, 20)])
def test_step_batches(torch, step_batch, flags, morton):
    """tril_run with several time steps per launch (each step its own subtree) equals the
    oracle for any batch size, including a shorter last batch, and for any number of
    Morton bits in the sort keys."""
    wl, A, B = _gauss_small(8000, 1.5e4, seed=4)
    raw, S = oracle_run(A, B, wl.dt, wl.n_steps, EDGES)
    gpu = gpu_run(A, B, wl.dt, wl.n_steps, EDGES, graph=True, flags=flags, step_batch=step_batch,
                  morton_bits=morton)
    assert S.n_pairs > 100
    assert_parity(gpu, raw, S, wl.n_steps)


def test_step_batches_with_instances(torch):
    """Step batches combined with ragged instances: combined (step, instance) subtrees."""
    parts_a, parts_b = [], []
    for m, (na, nb) in enumerate([(1200, 900), (0, 50), (1, 1), (900, 1500), (3, 700)]):
        wl = beams.batch64_instance(m)
        wl = beams.batch64_instance(m, w=wl.a.w * 800.0)
        A, B = beams.draw_pair(wl)
        parts_a.append(beams.head(A, na))
        parts_b.append(beams.head(B, nb))
    A, offA = beams.concat(parts_a)
    B, offB = beams.concat(parts_b)
    raw, S = oracle_run(A, B, 0.1, 400, EDGES, offA=offA, offB=offB)
    for sb, flags, mb in [(9, 0, 0), (50, T.TRIL_SORT_QUERIES_ONCE, 0), (0, T.TRIL_TIMING, 0),
                          (16, 0, 12)]:
        gpu = gpu_run(A, B, 0.1, 400, EDGES, graph=True, offA=offA, offB=offB, step_batch=sb,
                      flags=flags, morton_bits=mb)
        assert_parity(gpu, raw, S, 400)
    assert S.n_pairs > 20


def test_gauss_headon_1m_sampled_rows(torch):
    """Full size (1e6 per beam, calibrated weight, 400 steps, graph replay, the launch
    configuration of the benchmark): every pair of 300 sampled query rows, 150 of them
    drawn from the rows that collided, checked against the oracle."""
    wl = beams.gauss_headon_1m()
    A, B = beams.draw_pair(wl)
    i, j, k, st = gpu_run(A, B, wl.dt, wl.n_steps, EDGES, graph=True, cap=1 << 21)
    assert 10_000 < st["n_pairs"] < 40_000
    rng = np.random.default_rng(0)
    hit_rows = np.unique(i)
    rows = np.unique(np.concatenate([rng.choice(hit_rows, 150, replace=False),
                                     rng.choice(len(A["E"]), 150, replace=False)]))
    raw = O.collide(A, B, wl.dt, wl.n_steps, rows=rows)
    S = O.summarize(raw, A, B, wl.n_steps, EDGES)
    assert raw.knife_margin == 0 and raw.knife_s == 0
    keep = np.isin(i, rows)
    assert np.array_equal(i[keep], S.i)
    assert np.array_equal(j[keep], S.j)
    assert np.array_equal(k[keep], S.first_step)


def test_broadband_subsample_all_steps(torch):
    """Power-law spectrum, 150 deg crossing, 30 mrad: first 5000 photons of each
    1.6e7 beam prefix drawn at reduced size (i.i.d. photons), weight raised so the
    subsample collides; all 1000 steps."""
    full = beams.broadband_16m(n=10)
    wl = beams.broadband_16m(n=5000, w=full.a.w * 2e4)
    A, B = beams.draw_pair(wl)
    raw, S = oracle_run(A, B, wl.dt, wl.n_steps, EDGES)
    gpu = gpu_run(A, B, wl.dt, wl.n_steps, EDGES, graph=True)
    assert S.n_pairs > 50
    assert_parity(gpu, raw, S, wl.n_steps)


@pytest.mark.timeout(900)
def test_broadband_1e5_subsample_all_steps_with_spectrum(torch):
    """The large broadband workload's parity subsample: the first 1e5 photons of each
    1.6e7-photon beam (photons are drawn independently, so the prefix is a uniform sample),
    each carrying the weight of the 160 photons it stands for (so that the subsample holds
    the beam's physical photons and collides like it), all 1000 steps: pair set, first
    steps, per-step counts, yield and pair-energy spectrum against the oracle."""
    wl = beams.broadband_16m()
    A, B = beams.draw_pair(wl)
    A, B = beams.head(A, 100_000), beams.head(B, 100_000)
    for X in (A, B):
        X["w"] = X["w"] * (wl.a.n / 100_000)
    raw, S = oracle_run(A, B, wl.dt, wl.n_steps, EDGES)
    gpu = gpu_run(A, B, wl.dt, wl.n_steps, EDGES, graph=True, cap=1 << 22)
    assert S.n_pairs > 1000
    assert np.count_nonzero(S.spectrum) > 10
    assert_parity(gpu, raw, S, wl.n_steps)


def test_batched_instances_ragged(torch):
    """Several independent collisions in one launch, including empty and one-photon
    instances; photons only collide within their own instance."""
    parts_a, parts_b = [], []
    sizes = [(3000, 2500), (0, 100), (1, 1), (700, 0), (1500, 4000), (2, 3000)]
    for m, (na, nb) in enumerate(sizes):
        wl = beams.batch64_instance(m)
        wl = beams.batch64_instance(m, w=wl.a.w * 300.0)
        A, B = beams.draw_pair(wl)
        parts_a.append(beams.head(A, na))
        parts_b.append(beams.head(B, nb))
    A, offA = beams.concat(parts_a)
    B, offB = beams.concat(parts_b)
    raw, S = oracle_run(A, B, 0.1, 400, EDGES, offA=offA, offB=offB)
    for graph in (False, True):
        gpu = gpu_run(A, B, 0.1, 400, EDGES, graph=graph, offA=offA, offB=offB)
        assert_parity(gpu, raw, S, 400)
    assert S.n_pairs > 20


def test_below_threshold_beams_give_nothing(torch):
    wl = beams.mono_headon_2k(n=500)
    A, B = beams.draw_pair(wl)
    for b in (A, B):
        b["E"] = b["E"] * 0.25
        b["pz"] = b["pz"] * 0.25
        b["w"] = b["w"] * 1e6
    i, j, k, st = gpu_run(A, B, wl.dt, wl.n_steps, EDGES)
    assert st["n_pairs"] == 0 and st["n_hits"] == 0 and st["yield"] == 0.0


@pytest.mark.parametrize("na,nb", [(0, 10), (10, 0), (0, 0), (1, 1), (1, 500), (500, 1), (2, 2)])
def test_degenerate_sizes(torch, na, nb):
    wl = beams.mono_headon_2k()
    wl = beams.mono_headon_2k(w=wl.a.w * 1e4)
    A, B = beams.draw_pair(wl)
    A, B = beams.head(A, na), beams.head(B, nb)
    raw, S = oracle_run(A, B, wl.dt, wl.n_steps, EDGES)
    for graph in (False, True):
        gpu = gpu_run(A, B, wl.dt, wl.n_steps, EDGES, graph=graph)
        assert_parity(gpu, raw, S, wl.n_steps)


def test_overflow_then_rerun_is_identical(torch):
    wl, A, B = _gauss_small(5000, 2e4, seed=3)
    ctx = T.Context(wl.dt, EDGES)
    tb, qb = T.Beam(B), T.Beam(A)
    small = T.Pairs(8)
    T.run_steps(ctx, tb, qb, wl.n_steps, small)
    st = ctx.stats(small, check=False)
    assert st["code"] == T.TRIL_E_OVERFLOW
    need = st["n_hits"]
    assert need > 8
    ctx.close()
    runs = []
    for _ in range(2):
        ctx = T.Context(wl.dt, EDGES)
        big = T.Pairs(need)
        T.run_steps(ctx, tb, qb, wl.n_steps, big)
        st2 = ctx.stats(big)
        assert st2["n_hits"] == need
        runs.append(big.numpy())
        ctx.close()
    for a, b in zip(runs[0], runs[1]):
        assert np.array_equal(a, b)


def test_invalid_photon_data_reported(torch):
    wl = beams.mono_headon_2k(n=100)
    A, B = beams.draw_pair(wl)
    B["E"][17] = np.nan
    ctx = T.Context(wl.dt, EDGES)
    pairs = T.Pairs(1024)
    T.run_steps(ctx, T.Beam(B), T.Beam(A), 3, pairs)
    st = ctx.stats(pairs, check=False)
    ctx.close()
    assert st["code"] == T.TRIL_E_DATA


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("rel,rejected", [(1e-9, True), (-3e-12, True), (1e-13, False),
                                          (-1e-13, False)])
def test_momentum_off_shell_reported(torch, graph, rel, rejected):
    """A photon's momentum magnitude must equal its energy (c = 1) to 1e-12 relative:
    one photon of either beam scaled off the light cone by rel is rejected as bad data,
    one within the bound is accepted."""
    wl = beams.mono_headon_2k(n=100)
    A, B = beams.draw_pair(wl)
    for X, row in ((B, 17), (A, 53)):
        for f in ("px", "py", "pz"):
            X[f][row] *= 1.0 + rel
        ctx = T.Context(wl.dt, EDGES)
        pairs = T.Pairs(1024)
        T.run_steps(ctx, T.Beam(B), T.Beam(A), 3, pairs, graph=graph)
        st = ctx.stats(pairs, check=False)
        ctx.close()
        assert (st["code"] == T.TRIL_E_DATA) == rejected, (rel, st["code"])
        for f in ("px", "py", "pz"):
            X[f][row] /= 1.0 + rel


def test_counters_and_threshold_prune(torch):
    wl, A, B = _gauss_small(4000, 1e3, seed=5)
    ctx = T.Context(wl.dt, EDGES)
    pairs = T.Pairs(1 << 16)
    T.run_steps(ctx, T.Beam(B), T.Beam(A), 50, pairs, k0=180)
    st = ctx.stats(pairs)
    ctx.close()
    assert st["n_builds"] == 50 and st["n_collides"] == 50
    assert st["n_queries"] == 50 * 4000
    # every query loads its root at least once per descent (8 steps in a context's first run)
    assert st["n_node_visits"] * 8 >= st["n_queries"]
    assert st["n_candidates"] >= st["n_hits"]


def test_broadband_full_size_sampled_rows(torch):
    """Full size of the broadband workload (1.6e7 photons per beam, calibrated weight, 1000
    steps, graph replay, the benchmark's launch configuration of 32 steps per launch): every
    pair of 120 sampled query rows, 60 of them among the rows that collided, against the
    oracle."""
    wl = beams.broadband_16m()
    A, B = beams.draw_pair(wl)
    i, j, k, st = gpu_run(A, B, wl.dt, wl.n_steps, EDGES, graph=True, cap=1 << 22)
    assert 200_000 < st["n_pairs"] < 500_000
    rng = np.random.default_rng(3)
    rows = np.unique(np.concatenate([rng.choice(np.unique(i), 60, replace=False),
                                     rng.choice(len(A["E"]), 60, replace=False)]))
    raw = O.collide(A, B, wl.dt, wl.n_steps, rows=rows)
    S = O.summarize(raw, A, B, wl.n_steps, EDGES)
    assert raw.knife_margin == 0 and raw.knife_s == 0
    keep = np.isin(i, rows)
    assert np.array_equal(i[keep], S.i)
    assert np.array_equal(j[keep], S.j)
    assert np.array_equal(k[keep], S.first_step)
