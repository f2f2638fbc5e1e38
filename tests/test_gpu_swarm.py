"""IP-regime swarms on the GPU against the oracle: the number of colliding real-photon pairs
of every macro-particle pair is exact (an integer decided in FP64 on both sides in the same
operation order). Tiny clouds (cells of a few 1e-9 um, the size of the collision radius) make
the real photons of two swarms meet at the test sizes; head-on and 90 degree crossings,
directions with small angles, swarm sizes from 1 to 4096 real photons, bins aggregated; a
realistic-size case where nothing collides; an oversized swarm reported."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1608_01125_amd import tril as T

pytestmark = pytest.mark.gpu

ME = 0.51099895


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    return _t


def _tiny(seed, n, phi_deg=180.0, w_lo=1, w_hi=600, spread=2e-9, ang=0.0, E=2.0, along=0.05):
    rng = np.random.default_rng(seed)

    def beam(axis, other):
        b = {}
        pos = -0.5 * axis
        tr = rng.normal(0.0, spread, (n, 3))
        tr -= np.outer(tr @ axis, axis)
        along = rng.normal(0.0, along_sd, n)
        X = pos + tr + np.outer(along, axis)
        d = axis + rng.normal(0.0, ang, (n, 3)) if ang > 0 else np.repeat(axis[None], n, 0)
        d /= np.linalg.norm(d, axis=1)[:, None]
        b["x"], b["y"], b["z"] = X[:, 0].copy(), X[:, 1].copy(), X[:, 2].copy()
        b["px"], b["py"], b["pz"] = (E * d[:, 0]).copy(), (E * d[:, 1]).copy(), (E * d[:, 2]).copy()
        b["E"] = np.full(n, E)
        b["w"] = rng.integers(w_lo, w_hi + 1, n).astype(float)
        return b
    along_sd = along
    ph = np.radians(phi_deg)
    A = beam(np.array([0.0, 0.0, 1.0]), None)
    B = beam(np.array([np.sin(ph), 0.0, np.cos(ph)]), None)
    return A, B


def _run(torch, A, B, cell, k0=0, n_steps=10, dt=0.1, n_bins=3, pair_log2=16):
    nA, nB = len(A["E"]), len(B["E"])
    qa, tb = T.Beam(A), T.Beam(B)
    qbins = torch.tensor(np.arange(nA) % n_bins, dtype=torch.int32, device="cuda")
    tbins = torch.tensor(np.arange(nB) % n_bins, dtype=torch.int32, device="cuda")
    ctx = T.Context(dt, None)
    pt, tab = T.StTable(pair_log2), T.StTable(12)
    try:
        tot = T.tril_ip_swarm(ctx, tb, tbins, n_bins, qa, qbins, cell, k0, n_steps, pt, tab)
    finally:
        ctx.close()
    pk, pv = pt.items()
    bk, bv = tab.items()
    return tot, pk, pv, bk, bv


def _check(torch, A, B, cell, k0=0, n_steps=10, dt=0.1, min_total=1, **kw):
    cnt, knife = O.swarm_pairs(A, B, dt, k0, n_steps, cell)
    assert knife == 0
    tot, pk, pv, bk, bv = _run(torch, A, B, cell, k0, n_steps, dt, **kw)
    nB = len(B["E"])
    assert tot == int(cnt.sum()) and tot >= min_total
    # every macro-particle pair with colliding real photons is in the table with its count;
    # the table's other pairs (swept clouds that meet without a real collision) count zero
    got = dict(zip(pk.tolist(), pv.tolist()))
    ii, jj = np.nonzero(cnt)
    for i, j in zip(ii, jj):
        assert got.get(int(i) * nB + int(j)) == float(cnt[i, j])
    assert sum(v > 0 for v in got.values()) == len(ii)
    assert all(v == float(int(v)) for v in pv)
    # bin pairs: key (i % 3) * 3 + (j % 3)
    ref = {}
    for i, j in zip(ii, jj):
        k = (int(i) % 3) * 3 + int(j) % 3
        ref[k] = ref.get(k, 0) + int(cnt[i, j])
    assert dict(zip(bk.tolist(), [int(v) for v in bv])) == ref
    return cnt


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_head_on_tiny_clouds(torch, seed):
    A, B = _tiny(seed, 40)
    cnt = _check(torch, A, B, (4e-9, 4e-9, 4e-9))
    assert (cnt > 0).sum() > 20


def test_small_angles_and_non_cubic_cells(torch):
    A, B = _tiny(4, 40, ang=2e-9)
    _check(torch, A, B, (3e-9, 5e-9, 4e-9))


def test_crossing_at_ninety_degrees(torch):
    A, B = _tiny(5, 40, phi_deg=90.0, along=3e-9)
    _check(torch, A, B, (4e-9, 4e-9, 4e-9))


def test_swarm_sizes_one_to_4096(torch):
    """Single real photons (w = 1), weights rounding at one half, full lattices (4096) and
    counts just above a power of eight (a new octree level)."""
    A, B = _tiny(6, 24, w_lo=1, w_hi=1)
    _check(torch, A, B, (4e-9, 4e-9, 4e-9), min_total=0)
    A, B = _tiny(7, 16)
    A["w"] = np.resize([1.0, 8.0, 9.0, 64.0, 65.0, 512.0, 513.0, 4096.0, 2.5, 3.49], 16)
    B["w"] = np.resize([4096.0, 1.0, 7.5, 100.0, 513.0], 16)
    _check(torch, A, B, (4e-9, 4e-9, 4e-9))


def test_window_edges(torch):
    """The run window [k0 dt, (k0 + n) dt] decides: the crossings happen near t = 0.5."""
    A, B = _tiny(8, 30)
    full = O.swarm_pairs(A, B, 0.1, 0, 10, (4e-9,) * 3)[0].sum()
    part = _check(torch, A, B, (4e-9,) * 3, k0=5, n_steps=1, min_total=0)
    assert part.sum() <= full


def test_realistic_size_nothing_collides(torch):
    """Micrometre clouds and real cross-sections: the macro-particles meet, no real pair comes
    within r (about 2e-9 um)."""
    A, B = _tiny(9, 60, spread=0.2, w_lo=50, w_hi=300)
    tot, pk, pv, _, _ = _run(torch, A, B, (0.3, 0.3, 0.3))
    assert tot == 0 and len(pk) > 100 and not pv.any()
    assert O.swarm_pairs(A, B, 0.1, 0, 10, (0.3, 0.3, 0.3))[0].sum() == 0


def test_oversized_swarm_reported(torch):
    A, B = _tiny(10, 4)
    A["w"][0] = 2.0 ** 31
    with pytest.raises(T.TrilError) as e:
        _run(torch, A, B, (4e-9,) * 3)
    assert e.value.code == T.TRIL_E_DATA


def test_benchmark_configuration_sampled_pairs(torch):
    """The benchmark's swarm configuration (200 macro-particles per beam, 4096 real photons
    each, clouds of 4e-9 um, 10 steps): every macro-particle pair among 6 sampled rows of each
    beam against the brute-force oracle (1.7e7 real pairs per macro-particle pair)."""
    rng = np.random.default_rng(0)
    n, n_real = 200, 4096

    def beam(sgn):
        return {"x": rng.normal(0, 2e-9, n), "y": rng.normal(0, 2e-9, n),
                "z": -sgn * 0.5 + rng.normal(0, 0.05, n), "px": np.zeros(n), "py": np.zeros(n),
                "pz": np.full(n, sgn * 2.0), "E": np.full(n, 2.0), "w": np.full(n, float(n_real))}
    A, B = beam(1.0), beam(-1.0)
    cell = (4e-9, 4e-9, 4e-9)
    tot, pk, pv, _, _ = _run(torch, A, B, cell, pair_log2=20)
    got = dict(zip(pk.tolist(), pv.tolist()))
    ra = np.sort(rng.choice(n, 6, replace=False))
    rb = np.sort(rng.choice(n, 6, replace=False))
    As = {k: v[ra] for k, v in A.items()}
    Bs = {k: v[rb] for k, v in B.items()}
    cnt, knife = O.swarm_pairs(As, Bs, 0.1, 0, 10, cell)
    assert knife == 0 and cnt.sum() > 0
    for a, i in enumerate(ra):
        for b, j in enumerate(rb):
            assert got.get(int(i) * n + int(j), 0.0) == float(cnt[a, b])
