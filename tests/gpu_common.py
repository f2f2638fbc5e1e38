"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
compare with the CPU oracle."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_1608_01125_amd import tril as T


def gpu_run(A, B, dt, n_steps, edges, graph=False, flags=0, cap=1 << 20, k0=0,
            offA=None, offB=None, block=0, step_batch=0, morton_bits=0):
    """Tree over B (target), queries from A. Returns unique pairs + stats dict.
    graph=True goes through tril_run (step batches), else one build/collide per step."""
    ctx = T.Context(dt, edges, flags=flags, block_traverse=block, step_batch=step_batch,
                    morton_bits=morton_bits)
    try:
        tb = T.Beam(B, offB)
        qb = T.Beam(A, offA)
        pairs = T.Pairs(cap)
        T.run_steps(ctx, tb, qb, n_steps, pairs, k0=k0, graph=graph)
        st = ctx.stats(pairs, n_step_counts=k0 + n_steps)
        i, j, k = pairs.numpy()
    finally:
        ctx.close()
    return i, j, k, st


def oracle_run(A, B, dt, n_steps, edges, offA=None, offB=None, rows=None):
    if offA is None:
        raw, S = O.run(A, B, dt, n_steps, edges, rows=rows)
    else:
        raw, S = O.run_instances(A, offA, B, offB, dt, n_steps, edges, rows_per_inst=rows)
    return raw, S


def assert_parity(gpu, raw, S, n_steps, rel=1e-9):
    i, j, k, st = gpu
    assert raw.knife_margin == 0 and raw.knife_s == 0, "knife-edge pairs present"
    assert st["n_pairs"] == S.n_pairs, (st["n_pairs"], S.n_pairs)
    assert np.array_equal(i, S.i), "pair i differs"
    assert np.array_equal(j, S.j), "pair j differs"
    assert np.array_equal(k, S.first_step), "first step differs"
    assert np.array_equal(st["step_counts"][:n_steps], S.step_counts[:n_steps])
    assert st["n_hits"] == len(raw.i)
    if S.n_pairs:
        assert abs(st["yield"] - S.yield_) <= rel * abs(S.yield_)
        np.testing.assert_allclose(st["spectrum"], S.spectrum, rtol=rel, atol=0)
    else:
        assert st["yield"] == 0.0
