"""Window copies of the target hierarchy (GPU, through the C ABI): one copy of a batch's
tree shape serves W consecutive steps. The copies must hold exactly the boxes of their
window's middle step, every step's leaf box of the window must lie inside the copy's box
widened as the traversal widens it (the proof obligation of the slack, checked on every
leaf and step), and the candidates, hits and pairs must be those of one copy per step."""
import numpy as np
import pytest

from paper_1608_01125_amd import beams
from paper_1608_01125_amd import tril as T
from tests.gpu_common import assert_parity, oracle_run

pytestmark = pytest.mark.gpu

EDGES = beams.spectrum_edges()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    return _t


def _beams(n=3000, seed=2, boost=3e3, shift=None):
    wl = beams.gauss_headon_1m(n=n, seed=seed)
    wl = beams.gauss_headon_1m(n=n, seed=seed, w=wl.a.w * boost)
    A, B = beams.draw_pair(wl)
    if shift is not None:
        for X in (A, B):
            for a, f in enumerate(("x", "y", "z")):
                X[f] = X[f] + shift[a]
    return wl, A, B


def _ref_step(cp, win, m):
    a = cp * win
    return a + (min(win, m - a) - 1) // 2


def _run(wl, A, B, k0, n_steps, m, win, offA=None, offB=None, dwin=0):
    ctx = T.Context(wl.dt, EDGES, step_batch=m, kinetic_window=win, descent_window=dwin)
    try:
        pairs = T.Pairs(1 << 18)
        ctx.run(T.Beam(B, offB), T.Beam(A, offA), k0, n_steps, pairs)
        ci, cj, _ = T.tril_dbg_candidates(ctx)
        st = ctx.stats(pairs, n_step_counts=k0 + n_steps)
        i, j, k = pairs.numpy()
    finally:
        ctx.close()
    cand = np.sort(ci.astype(np.int64) << 32 | cj.astype(np.int64))
    return (i, j, k, st), cand


@pytest.mark.parametrize("m,wins", [
    (40, ((2, 0), (5, 0), (16, 0), (16, 1), (16, 3), (16, 16), (32, 0), (32, 32), (40, 7),
          (40, 32))),
    (7, ((2, 0), (3, 2), (7, 0), (7, 7))),
    (64, ((2, 0),))])
def test_candidates_and_pairs_equal_per_step_copies(torch, m, wins):
    """Same candidates (the last launch's, as a multiset, and the count over the run),
    hits and pairs as one copy per step, for windows (steps per copy, steps per descent: 0
    the default) that divide the batch, leave a short last window, and span the whole
    batch, with descents that divide the window or leave a shorter last one in each copy.
    (64 steps in copies of 2: 32 copies over 3000 rows, whose levels above the refit's
    chunks are merged level by level, with the binary nodes below the chunk tops unstored.)
    Every candidate comes from a leaf record read: at most one per step of its descent."""
    wl, A, B = _beams(n=3000, boost=3e3)
    k0, n_steps = 150, 3 * m + m // 2 + 1  # full batches (graphs) and a shorter last one
    base, cand1 = _run(wl, A, B, k0, n_steps, m, 1)
    assert base[3]["n_leaf_checks"] == 0
    assert base[3]["n_pairs"] > 5 and base[3]["n_candidates"] > 20
    for win, dwin in wins:
        got, cand = _run(wl, A, B, k0, n_steps, m, win, dwin=dwin)
        st, st1 = got[3], base[3]
        assert np.array_equal(cand, cand1), (win, dwin)
        assert st["n_candidates"] == st1["n_candidates"], (win, dwin)
        assert st["n_hits"] == st1["n_hits"] and st["n_pairs"] == st1["n_pairs"]
        for a, b in zip(got[:3], base[:3]):
            assert np.array_equal(a, b), (win, dwin)
        # the same pairs; the yield's FP64 sum runs in no fixed order
        assert st["yield"] == pytest.approx(st1["yield"], rel=1e-12)
        assert st["n_leaf_checks"] * min(win, m) >= st["n_candidates"]
        assert st["n_queries"] == st1["n_queries"]


def test_window_copies_match_oracle(torch):
    """Default windows (32 steps per copy, 8 per descent) over a whole 400-step run against
    the oracle."""
    wl, A, B = _beams(n=3000, boost=3e3, seed=5)
    raw, S = oracle_run(A, B, wl.dt, 400, EDGES)
    got, _ = _run(wl, A, B, 0, 400, 0, 0)
    assert S.n_pairs > 5
    assert_parity(got, raw, S, 400)


def test_far_from_origin_candidates_equal(torch):
    """Far from the origin (|x| ~ 1e3 um, one FP32 ulp ~ 6e-5 um) the rounding slack of
    the widened boxes grows with the magnitude: the candidates still equal those of one copy
    per step."""
    wl, A, B = _beams(n=2000, boost=3e4, shift=np.array([1000.0, -700.0, 900.0]))
    base, cand1 = _run(wl, A, B, 176, 48, 48, 1)
    got, cand = _run(wl, A, B, 176, 48, 48, 16)
    assert base[3]["n_candidates"] > 0
    assert np.array_equal(cand, cand1)
    assert got[3]["n_candidates"] == base[3]["n_candidates"]
    for a, b in zip(got[:3], base[:3]):
        assert np.array_equal(a, b)


def _walk(link, root):
    leaves, stack = [], [root] if root >= 0 else []
    if root <= -2:
        return [-2 - root]
    while stack:
        p = stack.pop()
        for c in link[p]:
            if c >= 0:
                stack.append(int(c))
            else:
                leaves.append(-2 - int(c))
    return leaves


@pytest.mark.parametrize("m,win", [(40, 16), (40, 4), (5, 2), (9, 9)])
def test_copies_hold_middle_step_boxes_and_contain_every_step(torch, m, win):
    """Several instances (one of a single row, one empty): ceil(m / W) copies of one shape;
    each (copy, instance) root reaches exactly that instance's sorted positions; a leaf's box
    in copy k is the photon's box at the window's middle step r (bit for bit); every step s
    of the window has every leaf's box inside the copy's box at r widened by the instance's
    motion bounds over s - r and the slack the traversal adds, with at least a factor two to
    spare."""
    parts = []
    for k, n_k in enumerate([1700, 1, 0, 900, 2]):
        wl = beams.gauss_headon_1m(n=max(n_k, 1), seed=20 + k)
        parts.append(beams.head(beams.draw_pair(wl)[1], n_k))
    Bc, off = beams.concat(parts)
    n, n_inst = len(Bc["E"]), len(off) - 1
    wl = beams.gauss_headon_1m(n=1000)
    k0 = 180
    ctx = T.Context(wl.dt, step_batch=m, kinetic_window=win)
    T.tril_dbg_keep_nodes(ctx)  # the whole binary tree, for the dump below
    try:
        tb = T.Beam(Bc, off)
        pairs = T.Pairs(1 << 12)
        ctx.run(tb, tb, k0, m, pairs)
        tree = T.tril_dbg_tree(ctx, n, n_inst, m)
        w_got, rec = T.tril_dbg_target_records(ctx, n)
        boxes = T.tril_dbg_boxes(ctx, 0, m * n)
    finally:
        ctx.close()
    eff = min(win, m)
    assert w_got == eff
    copies = -(-m // eff)
    assert tree["copies"] == copies
    n_int = n - 1
    link = tree["link"]
    assert link.shape == (copies * n_int, 2)
    base = link[:n_int]
    for cp in range(1, copies):  # the same shape: internal links offset, leaves the same
        lc = link[cp * n_int:(cp + 1) * n_int]
        assert np.array_equal(lc, np.where(base >= 0, base + cp * n_int, base))
    roots = tree["roots"].reshape(copies, n_inst)
    for cp in range(copies):
        for mi in range(n_inst):
            pos = np.arange(off[mi], off[mi + 1])
            r = int(roots[cp, mi])
            if len(pos) == 0:
                assert r == -1
                continue
            assert np.array_equal(np.sort(_walk(link, r)), pos)
    row = rec["row"]
    assert np.array_equal(np.sort(row), np.arange(n))
    blo = boxes["lo"].astype(np.float64)
    bhi = boxes["hi"].astype(np.float64)
    leaf = link < 0
    dt = wl.dt
    reach = np.float32((m + eff + 8) * dt + 1e-6)
    worst = 0.0
    for cp in range(copies):
        lk = link[cp * n_int:(cp + 1) * n_int]
        lo_c = tree["lo"][cp * n_int:(cp + 1) * n_int]
        hi_c = tree["hi"][cp * n_int:(cp + 1) * n_int]
        r = _ref_step(cp, eff, m)
        lf = lk < 0
        pos = -2 - lk[lf]
        e = r * n + row[pos]
        assert np.array_equal(lo_c[lf], boxes["lo"][e])
        assert np.array_equal(hi_c[lf], boxes["hi"][e])
        c = lk[~lf] - cp * n_int
        assert np.array_equal(lo_c[~lf], lo_c[c].min(axis=1))
        assert np.array_equal(hi_c[~lf], hi_c[c].max(axis=1))
        # every step of the window: leaf boxes inside the widened reference boxes
        d = rec["d"].astype(np.float64)
        for mi in range(n_inst):
            p = np.arange(off[mi], off[mi + 1])
            if len(p) == 0:
                continue
            dlo, dhi = d[p].min(axis=0), d[p].max(axis=0)
            er = r * n + row[p]
            for s in range(cp * eff, min((cp + 1) * eff, m)):
                es = s * n + row[p]
                delta = s - r
                emin = np.minimum(delta * dlo, delta * dhi)
                emax = np.maximum(delta * dlo, delta * dhi)
                mag = np.maximum(np.abs(blo[es]), np.abs(bhi[es]))
                sl = (mag + reach) * 2.0 ** -18
                need_lo = (blo[er] + emin) - blo[es]   # must be <= sl
                need_hi = bhi[es] - (bhi[er] + emax)   # must be <= sl
                worst = max(worst, float(np.max(need_lo / sl)), float(np.max(need_hi / sl)))
    assert leaf.any()
    print(f"\nlargest rounding excess over the slack: {worst:.3f}")
    assert worst <= 0.5


def test_repeated_runs_identical(torch):
    """Identical runs give identical candidate counts, hits and pairs, with window copies
    and with per-step copies in short batches (both merge the levels above the refit's
    chunks by climbing with arrival flags, whose halves must be visible device-wide before
    the flag counts them)."""
    wl = beams.gauss_headon_1m()
    A, B = beams.draw_pair(wl)
    tb, qb = T.Beam(B), T.Beam(A)
    for win, sb in ((16, 0), (1, 16)):
        ctx = T.Context(wl.dt, kinetic_window=win, step_batch=sb)
        try:
            pairs = T.Pairs(1 << 16)
            seen = set()
            for _ in range(4):
                pairs.reset()
                ctx.reset_counters()
                T.run_steps(ctx, tb, qb, 120, pairs, k0=140)
                st = ctx.stats(pairs)
                seen.add((st["n_candidates"], st["n_hits"], st["n_pairs"]))
        finally:
            ctx.close()
        assert len(seen) == 1, (win, sb, seen)
        assert next(iter(seen))[2] > 1000


def _unpack_slots(w):
    """Cell boxes (lo, hi: (k, 4, 3)), first-child ids (k, 4), leaf flags and energies of the
    four-child forms (words as tril_dbg_quad_nodes gives them)."""
    w = w.astype(np.int64)
    lo = np.zeros((len(w), 4, 3), np.int64)
    hi = np.zeros((len(w), 4, 3), np.int64)
    for k in range(4):
        a0, a1, a2 = w[:, 3 * k], w[:, 3 * k + 1], w[:, 3 * k + 2]
        lo[:, k] = np.stack([a0 & 0xFFFF, a0 >> 16, a1 & 0xFFFF], axis=1)
        hi[:, k] = np.stack([a1 >> 16, a2 & 0xFFFF, a2 >> 16], axis=1)
    ids = np.stack([w[:, 12], w[:, 12] + 1, w[:, 13], w[:, 13] + 1], axis=1)
    eh = np.stack([w[:, 14] & 0xFFFF, w[:, 14] >> 16, w[:, 15] & 0xFFFF, w[:, 15] >> 16], axis=1)
    leaf = (eh >> 15) & 1
    e = ((eh & 0x7FFF) << 16).astype(np.uint32).view(np.float32)
    return lo, hi, ids, leaf, e


@pytest.mark.parametrize("m,win", [(40, 16), (5, 2), (40, 40)])
def test_four_child_forms_hold_the_copies(torch, m, win):
    """The four-child forms the traversal descends: each node's slots are its grandchildren
    in the FP32 tree (or a leaf child and an empty slot), each slot's 16-bit cell box holds the
    grandchild's FP32 box in its copy's frame with no coordinate cut by the frame, and the
    15-bit energy bounds are not below the FP32 ones."""
    parts = []
    for k, n_k in enumerate([1700, 1, 0, 900, 2]):
        wl = beams.gauss_headon_1m(n=max(n_k, 1), seed=60 + k)
        parts.append(beams.head(beams.draw_pair(wl)[1], n_k))
    Bc, off = beams.concat(parts)
    n, n_inst = len(Bc["E"]), len(off) - 1
    wl = beams.gauss_headon_1m(n=1000)
    ctx = T.Context(wl.dt, step_batch=m, kinetic_window=win)
    try:
        tb = T.Beam(Bc, off)
        # by default the refit leaves the binary nodes below its chunks' tops unstored: the
        # dump refuses, and a run that stores them all gives the same forms and pairs
        pairs0 = T.Pairs(1 << 12)
        ctx.run(tb, tb, 170, m, pairs0)
        q0, _ = T.tril_dbg_quad_nodes(ctx, n, m)
        with pytest.raises(T.TrilError) as ei:
            T.tril_dbg_tree(ctx, n, n_inst, m)
        assert ei.value.code == T.TRIL_E_STATE
        T.tril_dbg_keep_nodes(ctx)
        pairs = T.Pairs(1 << 12)
        ctx.run(tb, tb, 170, m, pairs)
        tree = T.tril_dbg_tree(ctx, n, n_inst, m)
        q, frames = T.tril_dbg_quad_nodes(ctx, n, m)
    finally:
        ctx.close()
    assert np.array_equal(q0, q)
    got0 = sorted(zip(*(a.tolist() for a in pairs0.numpy())))
    got = sorted(zip(*(a.tolist() for a in pairs.numpy())))
    assert got0 == got
    copies = tree["copies"]
    n_int = n - 1
    assert q.shape == (copies * n_int, 16) and frames.shape == (copies, 8)
    lo, hi, ids, leaf, e = _unpack_slots(q)
    link = tree["link"].astype(np.int64)
    cp = np.repeat(np.arange(copies), n_int)
    cbase = cp * n_int
    # expected slots from the FP32 tree: grandchildren, or a leaf child and an empty slot
    for side in (0, 1):
        ch = link[:, side]
        internal = ch >= 0
        s0, s1 = 2 * side, 2 * side + 1
        gi = np.where(internal, ch, 0)
        want_link0 = np.where(internal, link[gi, 0], ch)
        want_link1 = np.where(internal, link[gi, 1], 0)
        for s, want, valid in ((s0, want_link0, np.ones(len(ch), bool)), (s1, want_link1, internal)):
            got = np.where(leaf[:, s] == 1, -2 - ids[:, s], cbase + ids[:, s])
            assert np.array_equal(got[valid], want[valid]), (side, s)
            flo = np.where(internal[:, None], tree["lo"][gi, s - 2 * side], tree["lo"][:, side])
            fhi = np.where(internal[:, None], tree["hi"][gi, s - 2 * side], tree["hi"][:, side])
            fe = np.where(internal, tree["e"][gi, s - 2 * side], tree["e"][:, side])
            if s == s1:  # a leaf child leaves its second slot empty
                assert np.all(lo[~internal, s] > hi[~internal, s])
                assert np.all(e[~internal, s] == 0)
            fb = frames[cp, 0:3].astype(np.float64)
            fi = frames[cp, 4:7].astype(np.float64)
            full = valid & (flo <= fhi).all(axis=1)
            a = (flo.astype(np.float64) - fb) * fi
            b = (fhi.astype(np.float64) - fb) * fi
            assert np.all(lo[full, s] <= a[full]) and np.all(hi[full, s] >= b[full])
            assert np.all(a[full] >= -1.0) and np.all(b[full] <= 65536.0)
            assert np.all(e[valid, s] >= fe[valid])


def test_automatic_descent_length_follows_the_leaf_tests_and_keeps_the_pairs(torch):
    """Automatic descent length: 8 steps in a context's first run; after each tril_stats it
    halves when the run tested more than 0.45 leaves per descent (that length is then not
    taken again) and doubles below 0.13. Every run finds the same pairs."""
    for boost, n in ((3e3, 3000), (3e3, 20000)):
        wl, A, B = _beams(n=n, boost=boost, seed=9)
        ctx = T.Context(wl.dt, EDGES)
        try:
            got, rejected, expect = [], set(), 8
            for _ in range(5):
                ctx.reset_counters()
                pairs = T.Pairs(1 << 18)
                ctx.run(T.Beam(B), T.Beam(A), 0, 200, pairs)
                st = ctx.stats(pairs)
                d = st["descent_window"]
                assert d == expect
                got.append(pairs.numpy())
                L = st["n_leaf_checks"] * d / st["n_queries"]
                if L > 0.45 and d > 1:
                    rejected.add(d)
                    expect = d // 2
                elif L < 0.13 and 2 * d <= 32 and 2 * d not in rejected:
                    expect = 2 * d
        finally:
            ctx.close()
        assert len(got[0][0]) > 0
        for g in got[1:]:
            for a, b in zip(g, got[0]):
                assert np.array_equal(a, b)
