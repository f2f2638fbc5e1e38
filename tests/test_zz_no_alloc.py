"""The no-allocation pair-kinematics entry point (tril_pair_kinematics_noalloc, through the
C ABI) against tril_pair_kinematics on the same pairs: leptons identical, histograms equal
up to summation order (1e-12 relative), status TRIL_OK. Two calls in a row on one device,
the second with fewer pairs and fewer photons (its scratch keeps the first call's contents,
which the call must clear), then a call whose beams are too large for the packed records
(read unpacked, same results), and a call with a pair outside its beam (status
TRIL_E_INVAL, the other pairs still written)."""
import numpy as np
import pytest

from paper_1608_01125_amd import beams
from paper_1608_01125_amd import tril as T

pytestmark = pytest.mark.gpu

G_EDGES = np.linspace(1.05, 10.05, 91)
N_THETA = 36


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    return _t


def _random_pairs(torch, nA, nB, n, seed):
    rng = np.random.default_rng(seed)
    p = T.Pairs(max(n, 1))
    if n:
        p.i[:n].copy_(torch.from_numpy(rng.integers(0, nA, n).astype(np.int32)))
        p.j[:n].copy_(torch.from_numpy(rng.integers(0, nB, n).astype(np.int32)))
        p.step[:n].copy_(torch.from_numpy(rng.integers(0, 400, n).astype(np.int32)))
    p.count.fill_(n)
    return p


def _both(torch, A, B, pairs, n, seed):
    ctx = T.Context(0.1)
    try:
        ref = T.tril_pair_kinematics(ctx, T.Beam(A), T.Beam(B), pairs, n, seed, G_EDGES, N_THETA,
                                     check=False)
    finally:
        ctx.close()
    dev = torch.device("cuda")
    edges = torch.from_numpy(G_EDGES).to(dev)
    gh = torch.full((len(G_EDGES) - 1,), -1.0, dtype=torch.float64, device=dev)
    th = torch.full((N_THETA,), -1.0, dtype=torch.float64, device=dev)
    lep = torch.full((max(n, 1), 8), -1.0, dtype=torch.float64, device=dev)
    status = torch.full((1,), 99, dtype=torch.int32, device=dev)
    rc = T.tril_pair_kinematics_noalloc(T.Beam(A), T.Beam(B), pairs, n, seed, edges, gh, N_THETA,
                                        th, lep, status)
    assert rc == T.TRIL_OK
    torch.cuda.synchronize()
    return ref, {"leptons": lep[:n], "gamma_hist": gh.cpu().numpy(),
                 "theta_hist": th.cpu().numpy(), "status": int(status.item())}


def _assert_same(ref, got):
    assert np.array_equal(ref["leptons"].cpu().numpy(), got["leptons"].cpu().numpy())
    np.testing.assert_allclose(got["gamma_hist"], ref["gamma_hist"], rtol=1e-12, atol=0)
    np.testing.assert_allclose(got["theta_hist"], ref["theta_hist"], rtol=1e-12, atol=0)


def test_noalloc_matches_allocating_entry_twice_then_smaller(torch):
    wl = beams.positron_spectra_1m(5.0, 5.0, n=20_000)
    A, B = beams.draw_pair(wl)
    # first call: 20k photons per beam (packed records), 300k pairs
    pairs = _random_pairs(torch, 20_000, 20_000, 300_000, 1)
    ref, got = _both(torch, A, B, pairs, 300_000, 7)
    assert ref["code"] == T.TRIL_OK and got["status"] == T.TRIL_OK
    assert ref["gamma_hist"].sum() > 0
    _assert_same(ref, got)
    # second call, smaller: 3k photons, 40k pairs; the scratch holds the first call's sums
    A2, B2 = beams.head(A, 3_000), beams.head(B, 3_000)
    pairs2 = _random_pairs(torch, 3_000, 3_000, 40_000, 2)
    ref2, got2 = _both(torch, A2, B2, pairs2, 40_000, 8)
    assert ref2["code"] == T.TRIL_OK and got2["status"] == T.TRIL_OK
    _assert_same(ref2, got2)


def test_noalloc_unpacked_beams_and_bad_pair(torch):
    # 2 x 150k photons: more than the 2^18 packed records the scratch holds
    wl = beams.positron_spectra_1m(7.0, 3.0, n=150_000)
    A, B = beams.draw_pair(wl)
    pairs = _random_pairs(torch, 150_000, 150_000, 400_000, 3)
    ref, got = _both(torch, A, B, pairs, 400_000, 9)
    assert ref["code"] == T.TRIL_OK and got["status"] == T.TRIL_OK
    _assert_same(ref, got)
    # one pair names a row outside the query beam: reported, the others still written
    pairs.i[5].fill_(150_000)
    ref, got = _both(torch, A, B, pairs, 400_000, 9)
    assert ref["code"] == T.TRIL_E_INVAL and got["status"] == T.TRIL_E_INVAL
    keep = np.ones(400_000, dtype=bool)
    keep[5] = False
    assert np.array_equal(ref["leptons"].cpu().numpy()[keep], got["leptons"].cpu().numpy()[keep])
    np.testing.assert_allclose(got["gamma_hist"], ref["gamma_hist"], rtol=1e-12, atol=0)


def test_noalloc_argument_checks(torch):
    wl = beams.positron_spectra_1m(5.0, 5.0, n=100)
    A, B = beams.draw_pair(wl)
    pairs = _random_pairs(torch, 100, 100, 10, 4)
    dev = torch.device("cuda")
    big = torch.zeros(T.TRIL_KIN_MAX_BINS + 2, dtype=torch.float64, device=dev)
    hist = torch.zeros(T.TRIL_KIN_MAX_BINS + 1, dtype=torch.float64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    rc = T.tril_pair_kinematics_noalloc(T.Beam(A), T.Beam(B), pairs, 10, 1, big, hist, 0, None,
                                        None, status)
    assert rc == T.TRIL_E_INVAL
    rc = T.tril_pair_kinematics_noalloc(T.Beam(A), T.Beam(B), pairs, 11, 1, None, None, 4, hist,
                                        None, status)
    assert rc == T.TRIL_E_INVAL  # more pairs than the buffer holds
    # decreasing edges: reported through the device status
    bad = torch.from_numpy(G_EDGES[::-1].copy()).to(dev)
    gh = torch.zeros(len(G_EDGES) - 1, dtype=torch.float64, device=dev)
    rc = T.tril_pair_kinematics_noalloc(T.Beam(A), T.Beam(B), pairs, 10, 1, bad, gh, 0, None,
                                        None, status)
    assert rc == T.TRIL_OK
    torch.cuda.synchronize()
    assert int(status.item()) == T.TRIL_E_INVAL
