"""Bounds of a descent over several steps of a window copy (host check, no GPU).

A descent serves steps s0 .. s1 of one copy of the target hierarchy, whose boxes are those
of the copy's step r. Two bounds make its candidates those of one descent per step:

* the hull: internal nodes are tested with the hull of the query's widened boxes at s0
  and s1 (its box at the step, shifted by the target instance's motion bounds over s - r,
  widened by the slack taken with the larger coordinates of the two boxes). Any leaf whose
  box at a step s of the descent meets the query's box at s has its box at r inside the hull.
* the step range: a leaf that passes is tested exactly at the steps of a range formed from
  the two records' relative motion; every step at which the exact test accepts lies in it.

The device's FP32 steps are emulated with numpy float32 (a fused multiply-add as an exact
FP64 product plus the FP64 sum, rounded once). Inputs are adversarial: coordinates from
1e-6 to 1e3 um, motion per step down to 1e-9 um, nearly co-moving pairs, boxes that touch
at some step, descents up to 32 steps, up to 4096 steps into a batch. Each check also runs
a broken form (the motion shift's sign reversed; the step range without its margins) that
must fail somewhere, so that it has teeth.
"""
import numpy as np

F = np.float32


def fma32(s, d, lo):
    return (s.astype(np.float64) * d.astype(np.float64) + lo.astype(np.float64)).astype(F)


def moved_axis(lo0, d, w, s):
    """One axis of a record's box at step offset s, as the device forms it."""
    l = fma32(s, d, lo0)
    h = (l + w).astype(F)
    e = (((np.abs(l) + np.abs(h)).astype(F) + (s * np.abs(d)).astype(F)).astype(F)
         * F(2.0 ** -21)).astype(F)
    return (l - e).astype(F), (h + e).astype(F)


def wslack(ql, qh, reach):
    return ((np.maximum(np.abs(ql), np.abs(qh)) + reach).astype(F) * F(2.0 ** -18)).astype(F)


def _records(rng, n, near=None):
    """Records (lo, d, w) per axis, shape (n, 3); near: lo of another record to sit close to."""
    mag = 10.0 ** rng.uniform(-6, 3, size=(n, 3)) * rng.choice([-1.0, 1.0], size=(n, 3))
    lo = mag.astype(F) if near is None else near
    d = (10.0 ** rng.uniform(-9, -1, size=(n, 3)) * rng.choice([-1.0, 1.0], size=(n, 3))).astype(F)
    w = (10.0 ** rng.uniform(-7, -1, size=(n, 3))).astype(F)
    return lo, d, w


def _pairs(n, seed):
    """Query and target records that meet at a chosen step of a descent, or nearly."""
    rng = np.random.default_rng(seed)
    ql, qd, qw = _records(rng, n)
    tl, td, tw = _records(rng, n, near=ql)
    co = rng.random((n, 1)) < 0.3  # nearly co-moving pairs
    td = np.where(co, (qd * (1 + rng.uniform(-1e-6, 1e-6, size=(n, 3)))).astype(F), td)
    s0 = rng.integers(0, 4064, size=(n, 1))
    ln = rng.integers(1, 33, size=(n, 1))
    meet = s0 + rng.integers(0, 32, size=(n, 1)) % ln
    # place the target so that its box touches or overlaps the query's at step `meet`
    mf = meet.astype(F)
    q_lo, q_hi = moved_axis(ql, qd, qw, mf)
    frac = rng.choice([-1.0, 0.0, 0.5, 1.0, 1.0 + 1e-7], size=(n, 3))
    anchor = np.where(frac < 0, q_lo - tw, q_lo + (q_hi - q_lo) * frac.astype(F)).astype(F)
    tl = (anchor.astype(np.float64) - mf.astype(np.float64) * td.astype(np.float64)).astype(F)
    return (ql, qd, qw), (tl, td, tw), s0, ln


def step_range(q, t, s0, ln, margin=True):
    """The device's step range of a leaf (before clamping to the descent, then clamped)."""
    (ql, qd, qw), (tl, td, tw) = q, t
    s1 = (s0 + ln - 1).astype(F)
    g = (((np.abs(ql) + np.abs(tl)).astype(F) + (qw + tw).astype(F)).astype(F)
         + (s1 * (np.abs(qd) + np.abs(td)).astype(F)).astype(F)).astype(F) * F(2.0 ** -17)
    if not margin:
        g = g * F(0.0)
    dd = (tl - ql).astype(F)
    lo = ((dd - qw).astype(F) - g).astype(F)
    hi = ((dd + tw).astype(F) + g).astype(F)
    rel = (qd - td).astype(F)
    tlo = np.broadcast_to(s0.astype(F), ql.shape).copy()
    thi = np.broadcast_to(s1, ql.shape).copy()
    nz = rel != 0
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        a1 = np.where(nz, lo / np.where(nz, rel, F(1)), F(0)).astype(F)
        a2 = np.where(nz, hi / np.where(nz, rel, F(1)), F(0)).astype(F)
    one = F(1.0) if margin else F(0.0)
    tlo = np.where(nz, np.fmax(tlo, np.floor(np.fmin(a1, a2)) - one), tlo)
    thi = np.where(nz, np.fmin(thi, np.ceil(np.fmax(a1, a2)) + one), thi)
    thi = np.where(~nz & ~((lo <= 0) & (hi >= 0)), F(-1.0), thi)
    return tlo.max(axis=1), thi.min(axis=1)


def exact_hits(q, t, s0, ln):
    """Steps (offset from s0) at which the exact closed test accepts, as an (n, 32) mask."""
    (ql, qd, qw), (tl, td, tw) = q, t
    n = ql.shape[0]
    hits = np.zeros((n, 32), dtype=bool)
    for k in range(32):
        s = (s0 + k).astype(F)
        a, b = moved_axis(ql, qd, qw, s)
        c, e = moved_axis(tl, td, tw, s)
        ok = ((a <= e) & (b >= c)).all(axis=1)
        hits[:, k] = ok & (k < ln[:, 0])
    return hits


def _range_escapes(margin, n=60_000, seed=11):
    q, t, s0, ln = _pairs(n, seed)
    hits = exact_hits(q, t, s0, ln)
    tlo, thi = step_range(q, t, s0, ln, margin)
    k = np.arange(32)[None, :] + s0
    inside = (k >= tlo[:, None]) & (k <= thi[:, None])
    return hits, (hits & ~inside)


def test_step_range_holds_every_exact_hit():
    hits, esc = _range_escapes(True)
    assert hits.sum() > 20_000  # the pairs do meet, at many steps
    assert not esc.any(), f"{esc.sum()} accepted steps outside the step range"


def test_step_range_without_margins_loses_hits():
    _, esc = _range_escapes(False)
    assert esc.any()


def _hull_misses(sign, n=60_000, seed=23):
    """Leaves meeting the query at a step of the descent whose box at r misses the hull
    (sign: +1 as the device shifts the boxes by the motion, -1 a sign error)."""
    rng = np.random.default_rng(seed)
    q, t, s0, ln = _pairs(n, seed)
    (ql, qd, qw), (tl, td, tw) = q, t
    # the target instance's motion bounds hold the leaf's motion (for half the pairs one
    # FP32 step around it, as tight as an instance of one photon); r anywhere in the copy
    spread = np.where(rng.random((n, 1)) < 0.5, 0.0, rng.uniform(0, 0.5, size=(n, 1))).astype(F)
    vlo = np.nextafter((td - np.abs(td) * spread).astype(F), F(-np.inf))
    vhi = np.nextafter((td + np.abs(td) * spread).astype(F), F(np.inf))
    r = s0 + rng.integers(-16, 48, size=(n, 1)) % np.maximum(ln + 16, 1)
    m, win = 4096 + 32, 32
    dt = 1.0
    reach = F((m + win + 8) * dt + 1e-6)
    sa, sz = s0.astype(F), (s0 + ln - 1).astype(F)
    qa_lo, qa_hi = moved_axis(ql, qd, qw, sa)
    qz_lo, qz_hi = moved_axis(ql, qd, qw, sz)
    sl = wslack(np.fmin(qa_lo, qz_lo), np.fmax(qa_hi, qz_hi), reach)
    da, dz = F(sign) * (s0 - r).astype(F), F(sign) * (s0 + ln - 1 - r).astype(F)
    wl = np.fmin(((qa_lo - np.fmax(da * vlo, da * vhi)).astype(F) - sl).astype(F),
                 ((qz_lo - np.fmax(dz * vlo, dz * vhi)).astype(F) - sl).astype(F))
    wh = np.fmax(((qa_hi - np.fmin(da * vlo, da * vhi)).astype(F) + sl).astype(F),
                 ((qz_hi - np.fmin(dz * vlo, dz * vhi)).astype(F) + sl).astype(F))
    c_lo, c_hi = moved_axis(tl, td, tw, r.astype(F))
    reached = ((c_lo <= wh) & (c_hi >= wl)).all(axis=1)
    hits = exact_hits(q, t, s0, ln).any(axis=1)
    return hits, hits & ~reached


def test_hull_reaches_every_leaf_that_meets_the_query():
    hits, miss = _hull_misses(1)
    assert hits.sum() > 20_000
    assert not miss.any(), f"{miss.sum()} meeting leaves outside the hull"


def test_hull_with_the_motion_reversed_misses_leaves():
    _, miss = _hull_misses(-1)
    assert miss.any()
