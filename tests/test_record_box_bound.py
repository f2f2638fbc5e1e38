"""Bound of the moved boxes: query records and tree leaves (host check, no GPU).

In a batch of steps a photon's swept box at step offset s, a query's or a leaf's in the
tree, is formed in FP32 from its offset-0 box (rounded outward) moved by s d, where
d = u dt is rounded to FP32 and the box widths are rounded up. It is then widened by
2^-21 (|lo| + |hi| + s |d|). It must contain the box the per-step path forms in FP64 for
that step and rounds outward: the swept segment over [t, t + dt], padded by the radius
bound (none for leaves) and a 1e-12 relative slack.

The traversal's FP32 steps are emulated with numpy float32; the fused multiply-add is
an exact FP64 product plus the FP64 sum, rounded once to FP32. Inputs are adversarial:
positions from 1e-6 to 1e3 um, direction components from 1e-8 to 1, steps up to 4096
into a batch that starts up to 1000 steps into the run. A widening 32 times smaller
must fail somewhere, so that the check has teeth.
"""
import numpy as np


def f32_down(x):
    f = x.astype(np.float32)
    over = f.astype(np.float64) > x
    f[over] = np.nextafter(f[over], np.float32(-np.inf))
    return f


def f32_up(x):
    f = x.astype(np.float32)
    under = f.astype(np.float64) < x
    f[under] = np.nextafter(f[under], np.float32(np.inf))
    return f


def step_box(p, u, t, dt, pad):
    """The per-step box: FP64 swept segment, padded, rounded outward to FP32."""
    a = p + t * u
    b = a + dt * u
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    lo32 = f32_down(lo - (pad + 1e-12 * (1.0 + np.abs(lo))))
    hi32 = f32_up(hi + (pad + 1e-12 * (1.0 + np.abs(hi))))
    return lo32, hi32


def record_box(L0, W, D, s, k):
    """The traversal's box from a record: FP32 arithmetic, widening factor k."""
    sf = s.astype(np.float32)
    lo = (sf.astype(np.float64) * D.astype(np.float64) + L0.astype(np.float64)).astype(np.float32)
    hi = lo + W
    e = ((np.abs(lo) + np.abs(hi)) + sf * np.abs(D)) * np.float32(k)
    return lo - e, hi + e


def _samples(n, seed):
    rng = np.random.default_rng(seed)
    mag = 10.0 ** rng.uniform(-6, 3, size=(n, 3))
    p = mag * rng.choice([-1.0, 1.0], size=(n, 3))
    u = 10.0 ** rng.uniform(-8, 0, size=(n, 3)) * rng.choice([-1.0, 1.0], size=(n, 3))
    u /= np.maximum(1.0, np.linalg.norm(u, axis=1))[:, None]
    dt = rng.choice([0.1, 0.04, 0.05, 0.0137], size=(n, 1))
    step0 = rng.integers(0, 1000, size=(n, 1))
    s = rng.integers(0, 4097, size=(n, 1))
    pad = np.where(rng.random((n, 1)) < 0.2, 0.0, 10.0 ** rng.uniform(-6, -2, size=(n, 1)))
    return p, u, dt, step0, s, pad


def _check(k, n=200_000, seed=5):
    p, u, dt, step0, s, pad = _samples(n, seed)
    t0 = step0 * dt
    L0, H0 = step_box(p, u, t0, dt, pad)
    W = f32_up(H0.astype(np.float64) - L0.astype(np.float64))
    D = (dt * u).astype(np.float32)
    qlo, qhi = record_box(L0, W, D, np.broadcast_to(s, L0.shape), k)
    lo, hi = step_box(p, u, (step0 + s) * dt, dt, pad)
    return (qlo <= lo) & (qhi >= hi)


def test_record_box_contains_the_step_box():
    ok = _check(2.0 ** -21)
    assert ok.all(), f"{(~ok).sum()} of {ok.size} coordinates escape the record box"


def test_a_much_smaller_widening_fails():
    assert not _check(2.0 ** -26).all()
