"""Freeze the macro-particle weight w of each workload (test infrastructure).

The workloads fix photon numbers, shapes and energies but, apart from the
mono-energetic 2k case's "about 2% of photons collide", no weight.  With w = 1
the collision radius sqrt(w sigma / pi) is so small that a 1e6-photon run has
far below one colliding pair, leaving nothing to compare.  Every workload
therefore uses the same rule: w is set so that the expected number of colliding
pairs is 2% of the smaller beam.

The number of pairs within distance r of each other grows as r^2, i.e. linearly
in w (r_ij^2 = sqrt(w_i w_j) sigma / pi with equal weights), as long as r is small
against the beam size.  So one oracle run at a trial weight w0 on a uniform
subsample of n_A x n_B photons gives

    w = w0 * target / (hits(w0) * (N_A N_B) / (n_A n_B)).

w0 is chosen large enough that hits(w0) is in the thousands (small counting
noise) while r stays far below the beam size.  The result is written to
paper_1608_01125_amd/workload_weights.json; only this script writes it.

Run:  python oracle/calibrate_w.py [--only NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path = [ROOT] + [p for p in sys.path
                    if os.path.abspath(p or '.') != os.path.dirname(os.path.abspath(__file__))]

from oracle import oracle as O  # noqa: E402
from paper_1608_01125_amd import beams  # noqa: E402


def _hits(A, B, dt, n_steps) -> int:
    raw = O.collide(A, B, dt, n_steps)
    key = raw.i.astype(np.int64) * (1 << 32) + raw.j
    return int(len(np.unique(key)))


def calibrate(wl_fn, n_sub: int, w0: float, **kw) -> dict:
    wl = wl_fn(w=w0, **kw)
    A, B = beams.draw_pair(wl)
    NA, NB = len(A["E"]), len(B["E"])
    na, nb = min(NA, n_sub), min(NB, n_sub)
    As, Bs = beams.head(A, na), beams.head(B, nb)
    h = _hits(As, Bs, wl.dt, wl.n_steps)
    target = 0.02 * min(NA, NB)
    scale = (NA * NB) / float(na * nb)
    w = w0 * target / (h * scale)
    return {"w": w, "w0": w0, "hits_w0": h, "n_sub": [na, nb], "N": [NA, NB],
            "expected_pairs": target}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=None)
    args = ap.parse_args()
    out_path = beams.WEIGHTS_FILE
    res = {}
    if os.path.exists(out_path):
        with open(out_path) as f:
            res = json.load(f)
    meta = res.setdefault("_calibration", {})

    def put(key, info):
        res[key] = info["w"]
        meta[key] = info
        print(key, info, flush=True)

    if args.only in (None, "mono_headon_2k"):
        put("mono_headon_2k", calibrate(beams.mono_headon_2k, 2000, 2.3e14))
    if args.only in (None, "gauss_headon_1m"):
        put("gauss_headon_1m", calibrate(beams.gauss_headon_1m, 20000, 2.0e14))
    if args.only in (None, "broadband_16m"):
        put("broadband_16m", calibrate(beams.broadband_16m, 20000, 2.0e15))
    if args.only in (None, "batch64"):
        for m in range(beams.BATCH64_INSTANCES):
            put(f"batch64/{m}", calibrate(lambda w: beams.batch64_instance(m, w=w), 6000, 2.0e14))
    if args.only in (None, "uniform_headon_1m"):
        put("uniform_headon_1m", calibrate(beams.uniform_headon_1m, 20000, 1.0e12))
    if args.only in (None, "positron_spectra_1m"):
        for g1, g2 in ((5.0, 5.0), (7.0, 3.0)):
            put(f"positron_spectra_1m/{g1:g}_{g2:g}",
                calibrate(lambda w: beams.positron_spectra_1m(g1, g2, w=w), 20000, 2.0e16))
    if args.only in (None, "crossing_angle_1e4"):
        for phi in (180.0, 90.0, 45.0):
            put(f"crossing_angle_1e4/{phi:g}",
                calibrate(lambda w: beams.crossing_angle_1e4(phi, w=w), 10000, 2.0e12))
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
    print("wrote", out_path)


if __name__ == "__main__":
    main()
