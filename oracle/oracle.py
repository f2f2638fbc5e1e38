"""Python face of the plain FP64 CPU oracle (tril_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it; the product library never does.  It shares no code
with the GPU path; both are fed from the seeded generators in
``paper_1608_01125_amd.beams``.

Outputs follow the problem statement of the paper (Sec. 1 and Sec. 3): the set
of colliding photon pairs, the number of pairs, the pair yield and the pair
energy spectrum.

  * raw hits: every (i, j, k) with pair (i, j) colliding in step k;
  * pair set: the union over steps, each pair tagged with the first step it
    collides in (with closed intervals a pair can collide in two adjacent steps;
    photons are not removed after colliding);
  * yield: sum over the pair set of sqrt(w_i w_j), the number of physical pairs
    a macro-particle pair stands for (Sec. 2.2);
  * spectrum: the same weights binned by E_i + E_j on caller-given edges, bin b
    holding edges[b] <= E_i + E_j < edges[b+1].
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tril_oracle.c")
LIB = os.path.join(HERE, "libtril_oracle.so")

CFLAGS = ["-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-std=gnu11", "-Wall"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


class _Beam(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [
        (f, ctypes.POINTER(ctypes.c_double)) for f in ("x", "y", "z", "px", "py", "pz", "E", "w")]


class _Out(ctypes.Structure):
    _fields_ = [
        ("cap", ctypes.c_int64), ("count", ctypes.c_int64),
        ("i", ctypes.POINTER(ctypes.c_int32)), ("j", ctypes.POINTER(ctypes.c_int32)),
        ("k", ctypes.POINTER(ctypes.c_int32)), ("margin", ctypes.POINTER(ctypes.c_double)),
        ("knife_margin", ctypes.c_int64), ("knife_s", ctypes.c_int64),
        ("pairs_tested", ctypes.c_int64), ("pairs_full", ctypes.c_int64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        d = ctypes.c_double
        L.orc_sigma.restype = d
        L.orc_sigma.argtypes = [d]
        L.orc_invariant.restype = d
        L.orc_invariant.argtypes = [d] * 8
        L.orc_step_d2.restype = d
        L.orc_step_d2.argtypes = [d] * 14
        L.orc_step_tau.restype = d
        L.orc_step_tau.argtypes = [d] * 14
        L.orc_sigma_max.restype = d
        L.orc_sigma_max.argtypes = []
        L.orc_collide.restype = None
        L.orc_collide.argtypes = [ctypes.POINTER(_Beam), ctypes.POINTER(_Beam),
                                  ctypes.POINTER(ctypes.c_int64), ctypes.c_int64,
                                  d, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.POINTER(_Out)]
        L.orc_st_pairs.restype = None
        L.orc_st_pairs.argtypes = [ctypes.POINTER(_Beam), ctypes.POINTER(_Beam),
                                   ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, d,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(d),
                                   ctypes.POINTER(d)]
        L.orc_st_exposure.restype = None
        L.orc_st_exposure.argtypes = L.orc_st_pairs.argtypes
        L.orc_swarm_pairs.restype = None
        L.orc_swarm_pairs.argtypes = [ctypes.POINTER(_Beam), ctypes.POINTER(_Beam),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, d,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(d),
                                      ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64)]
        L.orc_swarm_offsets.restype = None
        L.orc_swarm_offsets.argtypes = [ctypes.c_int64, ctypes.POINTER(d), ctypes.POINTER(d)]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def sigma(s: float) -> float:
    """Breit-Wheeler total cross-section in um^2 (Eq. 1)."""
    return lib().orc_sigma(float(s))


def sigma_max() -> float:
    return lib().orc_sigma_max()


def invariant(Ei, ui, Ej, uj) -> float:
    return lib().orc_invariant(Ei, *ui, Ej, *uj)


def step_d2(t, dt, xi, ui, xj, uj) -> float:
    return lib().orc_step_d2(t, dt, *xi, *ui, *xj, *uj)


def st_pairs(A, B, dt: float, k0: int, n_steps: int, cell, rows: Optional[np.ndarray] = None) -> np.ndarray:
    """Statistical-regime yield of every (query row, target photon) pair summed over
    steps k0 .. k0+n_steps-1 (cloud picture; see orc_st_pairs). Shape (rows, n_B)."""
    keep: list = []
    a, b = _as_beam(A, keep), _as_beam(B, keep)
    c = np.ascontiguousarray(cell, dtype=np.float64)
    nr = len(A["E"]) if rows is None else len(rows)
    out = np.zeros((nr, len(B["E"])), dtype=np.float64)
    rp = None
    if rows is not None:
        rws = np.ascontiguousarray(rows, dtype=np.int64)
        keep.append(rws)
        rp = rws.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    lib().orc_st_pairs(ctypes.byref(a), ctypes.byref(b), rp, nr, float(dt), int(k0), int(n_steps),
                       c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def st_exposure(A, B, dt: float, k0: int, n_steps: int, cell,
                rows: Optional[np.ndarray] = None) -> np.ndarray:
    """Exposure S of every (query row, target photon) cloud pair summed over steps k0 ..
    k0+n_steps-1 (see orc_st_exposure). Shape (rows, n_B)."""
    keep: list = []
    a, b = _as_beam(A, keep), _as_beam(B, keep)
    c = np.ascontiguousarray(cell, dtype=np.float64)
    nr = len(A["E"]) if rows is None else len(rows)
    out = np.zeros((nr, len(B["E"])), dtype=np.float64)
    rp = None
    if rows is not None:
        rws = np.ascontiguousarray(rows, dtype=np.int64)
        keep.append(rws)
        rp = rws.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    lib().orc_st_exposure(ctypes.byref(a), ctypes.byref(b), rp, nr, float(dt), int(k0),
                          int(n_steps), c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def swarm_offsets(n: int, cell) -> np.ndarray:
    """Offsets (n, 3) of the real photons of a swarm of n from its macro-particle's position
    (see orc_swarm_pairs)."""
    c = np.ascontiguousarray(cell, dtype=np.float64)
    out = np.zeros((max(int(n), 0), 3), dtype=np.float64)
    lib().orc_swarm_offsets(int(n), c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def swarm_pairs(A, B, dt: float, k0: int, n_steps: int, cell,
                rows: Optional[np.ndarray] = None):
    """Colliding real-photon pairs of every (query row, target) macro-particle pair over the
    run window (IP regime swarms; see orc_swarm_pairs): (counts (rows, n_B) int64, knife)."""
    keep: list = []
    a, b = _as_beam(A, keep), _as_beam(B, keep)
    c = np.ascontiguousarray(cell, dtype=np.float64)
    nr = len(A["E"]) if rows is None else len(rows)
    out = np.zeros((nr, len(B["E"])), dtype=np.int64)
    kn = ctypes.c_int64(0)
    rp = None
    if rows is not None:
        rws = np.ascontiguousarray(rows, dtype=np.int64)
        keep.append(rws)
        rp = rws.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    lib().orc_swarm_pairs(ctypes.byref(a), ctypes.byref(b), rp, nr, float(dt), int(k0),
                          int(n_steps), c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(kn))
    return out, int(kn.value)


def num_threads() -> int:
    return lib().orc_num_threads()


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def _as_beam(b: Dict[str, np.ndarray], keep: list) -> _Beam:
    cb = _Beam()
    cb.n = len(b["E"])
    for f in ("x", "y", "z", "px", "py", "pz", "E", "w"):
        a = np.ascontiguousarray(b[f], dtype=np.float64)
        keep.append(a)
        setattr(cb, f, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return cb


@dataclass
class RawHits:
    i: np.ndarray
    j: np.ndarray
    k: np.ndarray
    margin: np.ndarray
    knife_margin: int
    knife_s: int
    pairs_tested: int
    pairs_full: int


def collide(A, B, dt: float, n_steps: int, rows: Optional[np.ndarray] = None,
            k0: int = 0, strict: bool = False, cap: int = 1 << 20) -> RawHits:
    """All (i, j, k) hits for rows of A (all rows by default) against all of B,
    sorted by (i, j, k)."""
    L = lib()
    keep: list = []
    ca, cb = _as_beam(A, keep), _as_beam(B, keep)
    rows_arr = None
    rows_ptr = None
    n_rows = 0
    if rows is not None:
        rows_arr = np.ascontiguousarray(rows, dtype=np.int64)
        rows_ptr = rows_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        n_rows = len(rows_arr)
    while True:
        bi = np.empty(cap, np.int32)
        bj = np.empty(cap, np.int32)
        bk = np.empty(cap, np.int32)
        bm = np.empty(cap, np.float64)
        o = _Out(cap, 0, bi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                 bj.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                 bk.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                 bm.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0, 0, 0, 0)
        L.orc_collide(ctypes.byref(ca), ctypes.byref(cb), rows_ptr, n_rows,
                      float(dt), int(k0), int(n_steps), int(bool(strict)), ctypes.byref(o))
        if o.count <= cap:
            break
        cap = int(o.count) + 16
    n = int(o.count)
    order = np.lexsort((bk[:n], bj[:n], bi[:n]))
    return RawHits(bi[:n][order].copy(), bj[:n][order].copy(), bk[:n][order].copy(),
                   bm[:n][order].copy(), int(o.knife_margin), int(o.knife_s),
                   int(o.pairs_tested), int(o.pairs_full))


@dataclass
class Summary:
    i: np.ndarray           # unique pairs, ascending (i, j)
    j: np.ndarray
    first_step: np.ndarray
    step_counts: np.ndarray  # |H_k| for k in [k0, k0 + n_steps)
    n_pairs: int
    yield_: float
    spectrum: np.ndarray


def summarize(raw: RawHits, A, B, n_steps: int, edges: np.ndarray, k0: int = 0) -> Summary:
    """Union over steps (first step kept), per-step counts, yield and spectrum."""
    key = raw.i.astype(np.int64) * (1 << 32) + raw.j.astype(np.int64)
    # raw is sorted by (i, j, k): the first occurrence of a key has the earliest step
    uniq, first = np.unique(key, return_index=True)
    ui = raw.i[first]
    uj = raw.j[first]
    uk = raw.k[first]
    counts = np.bincount(raw.k - k0, minlength=n_steps)[:n_steps].astype(np.int64)
    wij = np.sqrt(A["w"][ui] * B["w"][uj])
    y = float(np.sum(wij))
    e = A["E"][ui] + B["E"][uj]
    b = np.searchsorted(edges, e, side="right") - 1
    ok = (b >= 0) & (b < len(edges) - 1)
    spec = np.zeros(len(edges) - 1)
    np.add.at(spec, b[ok], wij[ok])
    return Summary(ui, uj, uk, counts, int(len(uniq)), y, spec)


def step_tau(t, dt, xi, ui, xj, uj) -> float:
    """Time of closest approach within the window [t, t + dt], measured from t."""
    return lib().orc_step_tau(t, dt, *xi, *ui, *xj, *uj)


def hit_tau(raw: RawHits, A, B, dt: float) -> np.ndarray:
    """tau* of every raw hit (i, j, k): the time of closest approach inside step k."""
    out = np.empty(len(raw.i))
    for h in range(len(raw.i)):
        i, j, k = int(raw.i[h]), int(raw.j[h]), int(raw.k[h])
        ui = (A["px"][i] / A["E"][i], A["py"][i] / A["E"][i], A["pz"][i] / A["E"][i])
        uj = (B["px"][j] / B["E"][j], B["py"][j] / B["E"][j], B["pz"][j] / B["E"][j])
        out[h] = step_tau(k * dt, dt, (A["x"][i], A["y"][i], A["z"][i]), ui,
                          (B["x"][j], B["y"][j], B["z"][j]), uj)
    return out


def annihilate(raw: RawHits, A, B, dt: float) -> RawHits:
    """Photons that collide are consumed (annihilation, Sec. 2.1), and the collisions of a
    step are taken in chronological order (Sec. 2.2): the raw hits are ordered by step,
    then by the time of closest approach inside the step, then by i and j (a strict
    order), and a hit is kept when neither of its photons was consumed by a hit kept
    before it. Hits of photons consumed in earlier steps are dropped the same way, as if
    those photons had left the beams. Returns the kept hits, sorted by (i, j, k)."""
    tau = hit_tau(raw, A, B, dt)
    order = sorted(range(len(raw.i)),
                   key=lambda h: (int(raw.k[h]), float(tau[h]), int(raw.i[h]), int(raw.j[h])))
    used_a, used_b, kept = set(), set(), []
    for h in order:
        i, j = int(raw.i[h]), int(raw.j[h])
        if i in used_a or j in used_b:
            continue
        used_a.add(i)
        used_b.add(j)
        kept.append(h)
    kept = np.array(sorted(kept, key=lambda h: (int(raw.i[h]), int(raw.j[h]), int(raw.k[h]))),
                    dtype=np.int64)
    return RawHits(raw.i[kept], raw.j[kept], raw.k[kept], raw.margin[kept], raw.knife_margin,
                   raw.knife_s, raw.pairs_tested, raw.pairs_full)


def run(A, B, dt: float, n_steps: int, edges: np.ndarray, strict: bool = False,
        rows: Optional[np.ndarray] = None):
    raw = collide(A, B, dt, n_steps, rows=rows, strict=strict)
    return raw, summarize(raw, A, B, n_steps, edges)


def run_instances(A, offA, B, offB, dt: float, n_steps: int, edges: np.ndarray,
                  strict: bool = False, rows_per_inst: Optional[list] = None):
    """Independent instances given as CSR slices; indices returned are global rows."""
    outs = []
    for m in range(len(offA) - 1):
        a0, a1, b0, b1 = int(offA[m]), int(offA[m + 1]), int(offB[m]), int(offB[m + 1])
        Am = {k: v[a0:a1] for k, v in A.items()}
        Bm = {k: v[b0:b1] for k, v in B.items()}
        rows = None if rows_per_inst is None else rows_per_inst[m]
        raw = collide(Am, Bm, dt, n_steps, rows=rows, strict=strict)
        raw.i = raw.i + a0
        raw.j = raw.j + b0
        outs.append(raw)
    i = np.concatenate([r.i for r in outs]) if outs else np.zeros(0, np.int32)
    j = np.concatenate([r.j for r in outs]) if outs else np.zeros(0, np.int32)
    k = np.concatenate([r.k for r in outs]) if outs else np.zeros(0, np.int32)
    mg = np.concatenate([r.margin for r in outs]) if outs else np.zeros(0)
    order = np.lexsort((k, j, i))
    raw = RawHits(i[order], j[order], k[order], mg[order],
                  sum(r.knife_margin for r in outs), sum(r.knife_s for r in outs),
                  sum(r.pairs_tested for r in outs), sum(r.pairs_full for r in outs))
    return raw, summarize(raw, A, B, n_steps, edges)
