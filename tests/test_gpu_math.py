"""The device arithmetic the narrow phase relies on (tril_dbg_math, compiled with the narrow
phase's flags), against the host.

* FP64 division and square root must be correctly rounded: the narrow phase's s and d^2
  carry the same bits as the oracle's only if they are. 1.2e8 argument pairs (random
  exponents over most of the normal range, arguments near 1 where the narrow phase works,
  and the subnormal range), every result bit-identical to numpy's IEEE result.
* The FP32 stage's error bounds assume division and square root within 2 ulp and logf and
  log1pf within 4 ulp; measured against FP64 evaluations on the FP32-rounded arguments over
  2e7 arguments each (including the arguments the cross-section feeds them: s in (1, 1e6],
  b in (0, 1))."""
import numpy as np
import pytest

from paper_1608_01125_amd import tril as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    return _t


def _random_doubles(rng, n, lo_exp, hi_exp):
    m = rng.uniform(1.0, 2.0, n)
    e = rng.integers(lo_exp, hi_exp, n)
    s = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    return s * np.ldexp(m, e)


def _dev(torch, which, a, b=None):
    ta = torch.from_numpy(a).cuda()
    tb = torch.from_numpy(b).cuda() if b is not None else None
    out = torch.empty_like(ta)
    T.tril_dbg_math(which, ta, tb, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_fp64_division_and_sqrt_are_correctly_rounded(torch):
    rng = np.random.default_rng(2024)
    chunk, total = 10_000_000, 0
    kinds = ["wide", "near1", "wide", "near1", "subnormal", "wide"]
    for kind in kinds:
        if kind == "wide":
            a = _random_doubles(rng, chunk, -500, 500)
            b = _random_doubles(rng, chunk, -500, 500)
        elif kind == "near1":
            a = rng.uniform(0.5, 4.0, chunk) * np.where(rng.random(chunk) < 0.5, -1, 1)
            b = rng.uniform(0.5, 4.0, chunk)
        else:
            a = _random_doubles(rng, chunk, -1070, -1000)
            b = _random_doubles(rng, chunk, -30, 30)
        with np.errstate(all="ignore"):
            ref_div = a / b
            ref_sqrt = np.sqrt(np.abs(a))
        got_div = _dev(torch, T.DBG_DIV64, a, b)
        got_sqrt = _dev(torch, T.DBG_SQRT64, np.abs(a))
        assert np.array_equal(got_div.view(np.int64), ref_div.view(np.int64)), kind
        assert np.array_equal(got_sqrt.view(np.int64), ref_sqrt.view(np.int64)), kind
        total += 2 * chunk
    assert total >= 1.2e8


def _ulp32(x):
    """Spacing of FP32 numbers at |x| (subnormal spacing below the normal range)."""
    ax = np.abs(x).astype(np.float32)
    return np.spacing(ax).astype(np.float64)


def _max_ulp(got, ref):
    ok = np.isfinite(ref) & (ref != 0)
    err = np.abs(got[ok] - ref[ok]) / _ulp32(ref[ok])
    return float(err.max()) if err.size else 0.0


def test_fp32_routines_within_the_assumed_bounds(torch):
    rng = np.random.default_rng(7)
    n = 10_000_000
    res = {}
    for rep in range(2):
        a = _random_doubles(rng, n, -60, 60)
        b = _random_doubles(rng, n, -60, 60)
        af, bf = a.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)
        res.setdefault("div", []).append(_max_ulp(_dev(torch, T.DBG_DIV32, a, b), af / bf))
        pos = np.abs(a)
        pf = pos.astype(np.float32).astype(np.float64)
        res.setdefault("sqrt", []).append(_max_ulp(_dev(torch, T.DBG_SQRT32, pos), np.sqrt(pf)))
        # logf on positive arguments and on the cross-section's s in (1, 1e6]
        s = np.where(rng.random(n) < 0.5, pos, 1.0 + 10.0 ** rng.uniform(-7, 6, n))
        sf = s.astype(np.float32).astype(np.float64)
        res.setdefault("log", []).append(_max_ulp(_dev(torch, T.DBG_LOG32, s), np.log(sf)))
        # log1pf on (-1, inf), dense on the cross-section's b in (0, 1)
        x = np.where(rng.random(n) < 0.5, rng.uniform(0.0, 1.0, n),
                     np.expm1(rng.uniform(-20.0, 20.0, n)))
        xf = x.astype(np.float32).astype(np.float64)
        keep = xf > -1.0
        res.setdefault("log1p", []).append(
            _max_ulp(_dev(torch, T.DBG_LOG1P32, x)[keep], np.log1p(xf[keep])))
    worst = {k: max(v) for k, v in res.items()}
    print(f"\nmax ulp: {worst}")
    assert worst["div"] <= 2.0 and worst["sqrt"] <= 2.0
    assert worst["log"] <= 4.0 and worst["log1p"] <= 4.0
