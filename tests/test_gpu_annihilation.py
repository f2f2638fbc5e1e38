"""Annihilation mode on the GPU (TRIL_ANNIHILATE) against the oracle's chronological
greedy: hand-built crossings, dense conflicting bunches, a reduced head-on beam with
boosted weights and ragged batched instances give the oracle's kept hits exactly (yield
and spectrum to rounding of the sums); at full size the kept hits form a maximal matching
inside the raw hits."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1608_01125_amd import beams
from paper_1608_01125_amd import tril as T
from tests.gpu_common import assert_parity, gpu_run
from tests.test_oracle_annihilation import _axis_beams, _dense

pytestmark = pytest.mark.gpu

EDGES = beams.spectrum_edges()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    return _t


_CACHE = {}


def _oracle(A, B, dt, n_steps, offA=None, offB=None, key=None):
    if key is not None and key in _CACHE:
        return _CACHE[key]
    out = _oracle_run(A, B, dt, n_steps, offA, offB)
    if key is not None:
        _CACHE[key] = out
    return out


def _oracle_run(A, B, dt, n_steps, offA, offB):
    if offA is None:
        raw = O.collide(A, B, dt, n_steps)
    else:
        raw, _ = O.run_instances(A, offA, B, offB, dt, n_steps, EDGES)
    kept = O.annihilate(raw, A, B, dt)
    return raw, kept, O.summarize(kept, A, B, n_steps, EDGES)


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("case", ["order", "steps", "tie"])
def test_hand_built_crossings(torch, case, graph):
    if case == "order":
        (A, B), n = _axis_beams([0.0, -0.04], [0.88, 0.82]), 10
        want = {(0, 1, 4), (1, 0, 4)}
    elif case == "steps":
        (A, B), n = _axis_beams([0.0, -1.0], [0.5, 1.3]), 14
        want = {(0, 0, 2), (1, 1, 11)}
    else:
        (A, B), n = _axis_beams([0.0], [0.5, 0.5]), 6
        want = {(0, 0, 2)}
    raw, kept, S = _oracle(A, B, 0.1, n)
    gpu = gpu_run(A, B, 0.1, n, EDGES, graph=graph, flags=T.TRIL_ANNIHILATE)
    assert set(zip(*[x.tolist() for x in gpu[:3]])) == want
    assert_parity(gpu, kept, S, n)


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_dense_bunches(torch, seed):
    A, B, dt, n = _dense(seed)
    raw, kept, S = _oracle(A, B, dt, n)
    assert len(raw.i) > 2 * len(kept.i) > 0
    gpu = gpu_run(A, B, dt, n, EDGES, graph=True, flags=T.TRIL_ANNIHILATE)
    assert_parity(gpu, kept, S, n)
    # the same run without the flag keeps every raw hit's pair
    plain = gpu_run(A, B, dt, n, EDGES, graph=True)
    assert plain[3]["n_hits"] == len(raw.i)


@pytest.mark.parametrize("graph,step_batch,flags", [(True, 0, 0), (False, 0, 0), (True, 7, 0),
                                                    (True, 0, T.TRIL_FP64_NARROW)])
def test_gauss_headon_reduced_boosted(torch, graph, step_batch, flags):
    """20000 photons per beam, weights x 2500: about twice as many raw hits as kept."""
    wl = beams.gauss_headon_1m(seed=2)
    wl = beams.gauss_headon_1m(seed=2, n=20_000, w=wl.a.w * 2500.0)
    A, B = beams.draw_pair(wl)
    raw, kept, S = _oracle(A, B, wl.dt, wl.n_steps, key="gauss_reduced")
    assert len(raw.i) > 1.3 * len(kept.i) > 100
    gpu = gpu_run(A, B, wl.dt, wl.n_steps, EDGES, graph=graph, step_batch=step_batch,
                  flags=flags | T.TRIL_ANNIHILATE)
    assert_parity(gpu, kept, S, wl.n_steps)


@pytest.mark.parametrize("step_batch", [50, 7, 1])
def test_consumed_photons_drop_out_of_later_batches(torch, step_batch):
    """tril_run resolves every batch of steps as it finishes and leaves the photons it consumed
    out of the later batches' hierarchies and queries: the kept hits are still the oracle's,
    and the broad phase finds fewer candidates than the same run without annihilation (photons
    consumed early meet nobody later)."""
    wl = beams.gauss_headon_1m(seed=2)
    wl = beams.gauss_headon_1m(seed=2, n=20_000, w=wl.a.w * 2500.0)
    A, B = beams.draw_pair(wl)
    raw, kept, S = _oracle(A, B, wl.dt, wl.n_steps, key="gauss_reduced")
    plain = gpu_run(A, B, wl.dt, wl.n_steps, EDGES, graph=True, step_batch=step_batch)
    gpu = gpu_run(A, B, wl.dt, wl.n_steps, EDGES, graph=True, step_batch=step_batch,
                  flags=T.TRIL_ANNIHILATE)
    assert_parity(gpu, kept, S, wl.n_steps)
    assert gpu[3]["n_candidates"] < plain[3]["n_candidates"]
    assert plain[3]["n_hits"] == len(raw.i)


def test_batched_instances_ragged(torch):
    parts_a, parts_b = [], []
    for m, (na, nb) in enumerate([(3000, 2000), (0, 500), (1, 1), (2500, 4000), (700, 0)]):
        wl = beams.gauss_headon_1m(seed=40 + m)
        wl = beams.gauss_headon_1m(seed=40 + m, n=max(na, nb, 1), w=wl.a.w * 3e4)
        A, B = beams.draw_pair(wl)
        parts_a.append(beams.head(A, na))
        parts_b.append(beams.head(B, nb))
    A, offA = beams.concat(parts_a)
    B, offB = beams.concat(parts_b)
    wl = beams.gauss_headon_1m()
    raw, kept, S = _oracle(A, B, wl.dt, wl.n_steps, offA, offB)
    assert len(raw.i) > len(kept.i) > 50
    gpu = gpu_run(A, B, wl.dt, wl.n_steps, EDGES, graph=True, offA=offA, offB=offB,
                  flags=T.TRIL_ANNIHILATE)
    assert_parity(gpu, kept, S, wl.n_steps)


def test_full_size_kept_hits_are_a_maximal_matching(torch):
    """1e6 per beam, calibrated weight x 30, 400 steps (the benchmark's launch
    configuration): every kept hit is a raw hit, no photon is kept twice, and every photon
    with a raw hit keeps one or meets a partner consumed by a kept hit."""
    wl = beams.gauss_headon_1m()
    wl = beams.gauss_headon_1m(w=wl.a.w * 30.0)
    A, B = beams.draw_pair(wl)
    cap = 1 << 22
    ctx = T.Context(wl.dt, EDGES)
    try:
        tb, qb = T.Beam(B), T.Beam(A)
        pairs = T.Pairs(cap)
        T.run_steps(ctx, tb, qb, wl.n_steps, pairs)
        # raw hits before the union (the union rewrites the buffer)
        torch.cuda.synchronize()
        n_raw = int(pairs.count.item())
        ri = pairs.i[:n_raw].cpu().numpy().copy()
        rj = pairs.j[:n_raw].cpu().numpy().copy()
    finally:
        ctx.close()
    i, j, k, st = gpu_run(A, B, wl.dt, wl.n_steps, EDGES, graph=True, cap=cap,
                          flags=T.TRIL_ANNIHILATE)
    assert n_raw > len(i) > 1000
    assert len(np.unique(i)) == len(i) and len(np.unique(j)) == len(j)
    raw_pairs = set(zip(ri.tolist(), rj.tolist()))
    assert set(zip(i.tolist(), j.tolist())) <= raw_pairs
    used_a, used_b = set(i.tolist()), set(j.tolist())
    assert all(a in used_a or b in used_b for a, b in raw_pairs)
    assert st["n_hits"] == len(i)
