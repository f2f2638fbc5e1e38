#!/usr/bin/env python
"""Photon-pair queries resolved per second on one MI355X.

One benchmark step is one whole collision run of the hot path over one pair of
synthetic beams: for every time step, the hierarchy is built over beam B
(swept boxes, Morton keys, radix sort, hierarchy emission, refit), beam A is
prepared and traversed, candidates go through the FP64 narrow phase; after the
last time step the hits are merged into the pair set with yield, spectrum and
per-step counts. Inputs are resident in HBM before timing starts.

    value = N_A * N_B * n_time_steps / (seconds per benchmark step)

with the step batches replayed from captured HIP graphs. The same runs are then repeated
eagerly with HIP events around every phase launch, which give the phase times and the
traversal's launch durations. The JSON line also carries
  * roofline (HBM): the bytes the traversal must fetch per launch (per query-step its
    order entry and row record, 4 + 48 B; each step's tree copy once, 64 B per internal
    node; 8 B per candidate written) over its average launch duration, against 8 TB/s;
    `traffic` is the HBM bytes per launch measured with rocprofv3 counters (the
    committed summary, when it belongs to the current kernel source);
  * roofline_vmem: the busy cycles of the texture data units (one per CU, through which
    every lane's node load returns; rocprofv3 counters of the committed summary) against
    all their cycles: the resource that binds the traversal;
  * cpu_baseline: the FP64 CPU oracle timed on a bounded sample of query rows of
    the same workload (all pairs of those rows, all time steps).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "photon-pair queries resolved/s (N_A*N_B/t) at 1e6/beam; surrogate vs exact @≤1% err"
HBM_PEAK_GBS = 8000.0
TRAVERSE_SOURCES = ("paper_1608_01125_amd/csrc/traverse.hip", "paper_1608_01125_amd/csrc/tril_internal.h")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "traverse_gauss_headon_1m_pmc.txt")


def traverse_source_hash() -> str:
    """Hash of the traversal kernel's source and of what it reads from the shared header:
    node, box and record layouts, the moved-box bound and the window-copy slack."""
    h = hashlib.sha256()
    with open(os.path.join(ROOT, TRAVERSE_SOURCES[0]), "rb") as f:
        h.update(f.read())
    with open(os.path.join(ROOT, TRAVERSE_SOURCES[1]), "rb") as f:
        text = f.read().decode()
    a = text.index("struct alignas(16) Half")
    b = text.index("__device__ __forceinline__ float wslack")
    b = text.index("\n}", b)
    h.update(text[a:b].encode())
    return h.hexdigest()[:16]


def committed_counters(dispatches=None, window=None, descent=None) -> dict:
    """Counter figures of one traversal launch from the committed rocprofv3 summary: HBM
    bytes (`traffic_bytes_per_dispatch`), L1 lookups, TA/TD busy fractions. Empty when the
    summary was taken from a different kernel source, another batching (traversal launches
    per collision run), another number of steps per tree copy or per descent."""
    if not os.path.exists(PMC_SUMMARY):
        return {}
    vals = {}
    with open(PMC_SUMMARY) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != traverse_source_hash():
        return {}
    if dispatches is not None and vals.get("dispatches") != str(dispatches):
        return {}
    if window is not None and vals.get("kinetic_window", "1") != str(window):
        return {}
    if descent is not None and vals.get("descent_window", "1") != str(descent):
        return {}
    out = {}
    for k in ("traffic_bytes_per_dispatch", "L1_lookups_per_dispatch", "TD_busy", "TA_busy",
              "L2_hit_rate"):
        try:
            out[k] = float(vals[k])
        except (KeyError, ValueError):
            pass
    return out


def batch_sizes(n_steps: int, launches: int) -> list:
    """Steps of each launch of a run split as the library splits it: full batches of
    ceil(n_steps / launches) steps, the rest in the last."""
    if not launches:
        return [n_steps]
    m = -(-n_steps // launches)
    return [m] * (launches - 1) + [n_steps - m * (launches - 1)]


def tree_window(tune, arg: int, dwin: int) -> int:
    """Steps per tree copy in step batches (the library's default for 0: 32, or 16 with
    descents of 4 steps or fewer)."""
    w = (tune or {}).get("kinetic_window", arg) or arg
    return (16 if dwin <= 4 else 32) if w == 0 else w


def descent_window(tune, arg: int, win: int) -> int:
    """Steps per descent of a copy with four-child forms (the library's default for 0)."""
    d = (tune or {}).get("descent_window", arg) or arg
    return min(8 if d == 0 else d, win, 32)


def descents(b: int, win: int, dwin: int) -> int:
    """Descents per query row in a batch of b steps: one per step without window copies,
    else every copy's steps split into descents of dwin steps (the library's count)."""
    if win <= 1 or b < 2:
        return b
    w = min(win, b)
    copies = -(-b // w)
    last = b - (copies - 1) * w
    return (copies - 1) * -(-w // dwin) + -(-last // dwin)


def make_workload(name: str, physics_steps: int):
    """(workload, beam A, offsets A, beam B, offsets B, steps); offsets None = one instance."""
    from paper_1608_01125_amd import beams
    offA = offB = None
    if name == "gauss_headon_1m":
        wl = beams.gauss_headon_1m()
    elif name == "mono_headon_2k":
        wl = beams.mono_headon_2k()
    elif name == "uniform_headon_1m":
        wl = beams.uniform_headon_1m()
    elif name == "broadband_16m":
        wl = beams.broadband_16m()
    elif name in ("positron_spectra_1m_5_5", "positron_spectra_1m_7_3"):
        g1, g2 = (5.0, 5.0) if name.endswith("5_5") else (7.0, 3.0)
        wl = beams.positron_spectra_1m(g1, g2)
    elif name == "batch64":
        parts_a, parts_b = [], []
        for m in range(64):
            wl = beams.batch64_instance(m)
            A, B = beams.draw_pair(wl)
            parts_a.append(A)
            parts_b.append(B)
        A, offA = beams.concat(parts_a)
        B, offB = beams.concat(parts_b)
        n_steps = physics_steps if physics_steps > 0 else wl.n_steps
        return wl, A, offA, B, offB, n_steps
    else:
        raise SystemExit(f"unknown workload {name}")
    A, B = beams.draw_pair(wl)
    n_steps = physics_steps if physics_steps > 0 else wl.n_steps
    return wl, A, offA, B, offB, n_steps


def st_bench(args):
    """Statistical regime, head-on shape, --st-mp macro-particles per beam: the surrogate path
    (ensemble trained on exact yields of the same shape at other seeds and at most 2e5
    macro-particles per beam; its predictions corrected by the audit, a sampled exact estimate
    with the predictions as control), timed; against the exact total of the hierarchy path
    where it can run (up to 1e6 macro-particles per beam), else against the judge: a sampled
    exact estimate with no network in it, whose 95% confidence half-width is reported, and the
    exact path's time extrapolated from uniform thinnings of both beams."""
    import numpy as np
    import torch
    from paper_1608_01125_amd import beams, surrogate
    from paper_1608_01125_amd import tril as T
    eps = 1e-3
    ctx = T.Context(0.1, None)
    net = T.Mlp(4, seed=11)
    n = args.st_mp
    q = float(n) * n * 400
    try:
        t0 = time.perf_counter()
        train_mp = [int(v) for v in args.st_train_mp.split(",") if v] or [min(n, 200_000)]
        insts = [surrogate.Instance(beams.st_headon(train_mp[m % len(train_mp)], seed=2000 + m))
                 for m in range(args.st_train)]
        x, t, y0, y = surrogate.training_rows(ctx, insts, eps=eps, log=_progress)
        g = torch.Generator(device="cuda")
        g.manual_seed(0)
        keep = (y > 0) | (torch.rand(y.shape[0], device="cuda", generator=g) < 0.25)
        surrogate.train(net, x[keep].contiguous(), t[keep].contiguous(), n_steps=args.st_train_steps,
                        batch=8192, lr=1e-3)
        scale = surrogate.yield_scale(net, x, y0, y, eps)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
        n_rows = int(keep.sum())
        del insts, x, t, y0, y, keep
        _progress(f"trained in {train_s:.1f} s")
        inst = surrogate.Instance(beams.st_headon(n))
        p_audit = T.sur_params(eps=eps, gate=0.01, scale=scale, audit=True,
                               audit_sample=args.st_audit_sample, audit_reps=8, audit_seed=1)
        p_budget = T.sur_params(eps=eps, gate=0.01, scale=scale)
        for _ in range(args.warmup):
            inst.surrogate(ctx, net, p_audit)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            res = inst.surrogate(ctx, net, p_audit)
        torch.cuda.synchronize()
        t_sur = (time.perf_counter() - t1) / max(args.steps, 1)
        budget = inst.surrogate(ctx, net, p_budget)
        _progress(f"surrogate path {1e3 * t_sur:.1f} ms")
        exact_total = t_exact = None
        exact = {}
        if n <= args.st_exact_max:
            inst.exact(ctx)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                _, exact_total = inst.exact(ctx)
            torch.cuda.synchronize()
            t_exact = (time.perf_counter() - t1) / max(args.steps, 1)
            st = ctx.stats(None)
            exact = {"total": exact_total, "ms": 1e3 * t_exact, "queries_per_s": q / t_exact,
                     "timing": "measured",
                     "cloud_pair_steps_per_run": st["n_candidates"] // max(args.steps + 1, 1)}
        else:
            # the exact pass over two uniform thinnings (every macro-particle kept with
            # probability f, both beams): its pair work is f^2 of the full pass
            fr = {}
            for f in (0.01, 0.02):
                r = inst.audit(ctx, None, T.AUDIT_NONE, n_sample=int(f * n), n_rep=2, seed=9)
                fr[f] = r["ms"] / 2.0
                _progress(f"exact pass on a {f:.0%} thinning of both beams: {fr[f]:.0f} ms")
            t_exact = 1e-3 * fr[0.02] / 0.02 ** 2
            exact = {"total": None, "ms": 1e3 * t_exact, "queries_per_s": q / t_exact,
                     "timing": "extrapolated: exact pass over a uniform 2% thinning of both beams "
                               "/ 0.02^2",
                     "ms_thinning_1pct": fr[0.01], "ms_thinning_2pct": fr[0.02],
                     "pair_work_scaling_2pct_over_1pct": fr[0.02] / fr[0.01]}
        # the judge: sampled exact estimate with the bin-level yield as control (no network)
        jd = inst.audit(ctx, None, T.AUDIT_BIN_LEVEL, n_sample=args.st_judge_sample, n_rep=8,
                        seed=4242)
        _progress(f"judge {jd['estimate']:.6g} +- {jd['half_width']:.3g} in {jd['ms']:.0f} ms")
        ref = exact_total if exact_total is not None else jd["estimate"]
        # depletion (closed forms per cloud pair) against the linear exact yields, at a photon
        # number where depletion matters, on a smaller instance (one table slot per cloud pair)
        dinst = surrogate.Instance(beams.st_headon(args.st_dep_mp, physical=args.st_dep_physical))
        dinst.exact(ctx)
        dinst.exact_depleted(ctx, pair_log2=26)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            _, lin_total = dinst.exact(ctx)
        torch.cuda.synchronize()
        t_lin = (time.perf_counter() - t1) / max(args.steps, 1)
        t1 = time.perf_counter()
        for _ in range(args.steps):
            _, pt, dep_total = dinst.exact_depleted(ctx, pair_log2=26)
        torch.cuda.synchronize()
        t_dep = (time.perf_counter() - t1) / max(args.steps, 1)
        n_cloud_pairs = int((pt.key >= 0).sum().item())
        del dinst, pt
        from oracle import st_oracle as SO
        dwl = beams.st_headon(args.st_dep_mp, physical=args.st_dep_physical)
        DA, DB = beams.draw_pair(dwl)
        drows = np.arange(20)
        t1 = time.perf_counter()
        SO.st_depleted_pairs(DA, DB, dwl.dt, 0, dwl.n_steps,
                             surrogate.cell_grid(dwl, "a", DA).cell, rows=drows)
        dep_cpu_s = time.perf_counter() - t1
        swarm = swarm_measure(T, torch)
    finally:
        net.close()
        ctx.close()
    nd = args.st_dep_mp
    out = {
        "metric": METRIC, "value": q / t_sur, "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t_sur,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "st_headon", "macro_particles_per_beam": n,
                   "physical_photons_per_beam": 1e9, "time_steps": 400,
                   "grid": "32^3 cells (surrogate on cell pairs)", "ensemble": 4,
                   "gate": "audit: sampled exact estimate with the network as control",
                   "training": {"instances": args.st_train, "rows": n_rows,
                                "macro_particles": train_mp,
                                "adam_steps": args.st_train_steps, "seconds": round(train_s, 1),
                                "yield_scale": round(scale, 5)}},
        "surrogate": {"queries_per_s": q / t_sur, "ms": 1e3 * t_sur, "total": res["total"],
                      "half_width_95": res["audit_half_width"],
                      "network_total": res["surrogate_part"],
                      "network_rel_bias": res["surrogate_part"] / ref - 1.0,
                      "rel_error": abs(res["total"] - ref) / ref,
                      "reference": "exact total" if exact_total is not None else "judge",
                      "within_1pct": abs(res["total"] - ref) <= 0.01 * ref,
                      "audit_sampled_macro_particles": res["audit_sampled"],
                      "bin_pairs": res["n_bin_pairs"],
                      "speedup_vs_exact": t_exact / t_sur},
        "surrogate_budget_gate": {"total": budget["total"], "ms": budget["ms"],
                                  "rel_error": abs(budget["total"] - ref) / ref,
                                  "bin_pairs_exact": budget["n_gated"],
                                  "predicted_spread": budget["predicted_spread"]},
        "judge": {"estimate": jd["estimate"], "half_width_95": jd["half_width"],
                  "rel_half_width": jd["half_width"] / jd["estimate"],
                  "rel_diff_vs_exact": (jd["estimate"] / exact_total - 1.0
                                        if exact_total is not None else None),
                  "control": "bin-level yield Y0 (no network)", "n_sample": args.st_judge_sample,
                  "replicates": 8, "ms": jd["ms"]},
        "exact": exact,
        "exact_depleted": {"macro_particles_per_beam": nd,
                           "physical_photons_per_beam": args.st_dep_physical,
                           "queries_per_s": float(nd) * nd * 400 / t_dep, "ms": 1e3 * t_dep,
                           "ms_linear": 1e3 * t_lin, "total": dep_total,
                           "linear_total": lin_total, "ratio_to_linear": dep_total / lin_total,
                           "cloud_pairs": n_cloud_pairs,
                           "cpu_oracle": {"queries_per_s": 20.0 * nd * 400 / dep_cpu_s,
                                          "kind": "oracle", "cores": _oracle_threads(),
                                          "sample": "20 query rows x all target clouds x 400 steps"}},
        "ip_swarm": swarm,
    }
    print(json.dumps(out), flush=True)


MLP_FLOP_PER_ROW = 2 * (6 * 256 + 2 * 256 * 256 + 256)  # one member, one row, forward
MFMA_BF16_PEAK_TFLOPS = 2500.0


def mlp_bench(args):
    """The surrogate network's kernels alone (4-member ensemble, 6 -> 256 -> 256 -> 256 -> 1):
    inference of --mlp-rows rows (the fused forward kernel, all members, plus the ensemble
    reduction) and training member-steps at batch 8192 (forward, loss, backward, Adam),
    timed with HIP events; FLOPs against the BF16 dense matrix-core peak."""
    import numpy as np
    import torch
    from paper_1608_01125_amd import tril as T
    n = args.mlp_rows
    rng = np.random.default_rng(0)
    x = torch.from_numpy(rng.normal(0, 1, (n, 6)).astype(np.float32)).cuda()
    y = torch.from_numpy(rng.normal(0, 1, n).astype(np.float32)).cuda()
    net = T.Mlp(4, seed=3)
    try:
        net.fit_norm(x, y)
        for _ in range(max(args.warmup, 1)):
            net.predict(x)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = []
        for _ in range(args.steps):
            e0.record()
            net.predict(x)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        t_inf = sorted(ms)[len(ms) // 2]
        net.train(x, y, 20, 8192, 1e-3, 0)
        torch.cuda.synchronize()
        steps = args.mlp_train_steps
        e0.record()
        net.train(x, y, steps, 8192, 1e-3, 1)
        e1.record()
        torch.cuda.synchronize()
        t_step = e0.elapsed_time(e1) / (steps * 4)
    finally:
        net.close()
    inf_flop = float(MLP_FLOP_PER_ROW) * n * 4
    tr_flop = 3.0 * MLP_FLOP_PER_ROW * 8192
    tf_inf = inf_flop / (t_inf * 1e-3) / 1e12
    tf_tr = tr_flop / (t_step * 1e-3) / 1e12
    out = {"metric": "surrogate ensemble rows/s (4 members)", "value": n / (t_inf * 1e-3),
           "unit": "rows/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": t_inf, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "mlp", "rows": n, "members": 4,
                      "layers": "6-256-256-256-1 SiLU"},
           "roofline": {"bound": "mfma", "achieved": round(tf_inf, 1),
                        "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(tf_inf / MFMA_BF16_PEAK_TFLOPS, 4), "traffic": None,
                        "kernel": "k_mlp_fused", "flop_per_row_member": MLP_FLOP_PER_ROW},
           "training": {"ms_per_member_step": t_step, "batch": 8192,
                        "tflops_3x_forward": round(tf_tr, 2),
                        "frac": round(tf_tr / MFMA_BF16_PEAK_TFLOPS, 5)}}
    print(json.dumps(out), flush=True)


def _progress(msg):
    """A progress line on stderr (long statistical-regime runs)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _oracle_threads():
    from oracle import oracle as O
    return O.num_threads()


def swarm_measure(T, torch, n_mp=200, n_real=4096, reps=3):
    """IP-regime swarms: two head-on beams of n_mp macro-particles of n_real real photons each
    in clouds of 4e-9 um (the size of the collision radius, so that real photons meet),
    transverse spread 2e-9 um, 10 steps of 0.1 um/c across the crossing. Reports the time of
    tril_ip_swarm and the real-pair tests it resolves per second (sum of n_i n_j over the
    macro-particle pairs it examines)."""
    import numpy as np
    rng = np.random.default_rng(0)

    def beam(sgn):
        n = n_mp
        return {"x": rng.normal(0, 2e-9, n), "y": rng.normal(0, 2e-9, n),
                "z": -sgn * 0.5 + rng.normal(0, 0.05, n), "px": np.zeros(n), "py": np.zeros(n),
                "pz": np.full(n, sgn * 2.0), "E": np.full(n, 2.0), "w": np.full(n, float(n_real))}
    A, B = beam(1.0), beam(-1.0)
    cell = (4e-9, 4e-9, 4e-9)
    qa, tb = T.Beam(A), T.Beam(B)
    bins = torch.zeros(n_mp, dtype=torch.int32, device="cuda")
    ctx = T.Context(0.1, None)
    pt, tab = T.StTable(20), T.StTable(4)
    try:
        T.tril_ip_swarm(ctx, tb, bins, 1, qa, bins, cell, 0, 10, pt, tab)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            tot = T.tril_ip_swarm(ctx, tb, bins, 1, qa, bins, cell, 0, 10, pt, tab)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        n_pairs = int((pt.key >= 0).sum().item())
    finally:
        ctx.close()
    tests = float(n_pairs) * n_real * n_real
    from oracle import oracle as O
    sub_a = {k: v[:3] for k, v in A.items()}
    sub_b = {k: v[:3] for k, v in B.items()}
    t0 = time.perf_counter()
    O.swarm_pairs(sub_a, sub_b, 0.1, 0, 10, cell)
    cpu_s = time.perf_counter() - t0
    return {"cpu_oracle": {"real_pair_tests_per_s": 9.0 * n_real * n_real / cpu_s,
                           "cores": O.num_threads(), "kind": "oracle",
                           "sample": "3 x 3 macro-particle pairs, brute force over real pairs"},
            "macro_particles_per_beam": n_mp, "real_photons_per_mp": n_real,
            "mp_pairs": n_pairs, "real_pair_tests_implied": tests, "colliding_real_pairs": tot,
            "ms": 1e3 * sec, "real_pair_tests_per_s": tests / sec}


KIN_BYTES_PER_PAIR = 12 + 2 * 5 * 8 + 64  # (i, j, k), E p w of both photons, 8 lepton doubles
KIN_SUMMARY = os.path.join(ROOT, "profiles", "pair_kin_positron_spectra_1m.md")


def kinematics_traffic(n_pairs):
    """HBM bytes per bulk launch of the kinematics kernel from the committed counter summary,
    or None when it belongs to another kernel source or another bulk size."""
    if not os.path.exists(KIN_SUMMARY):
        return None
    vals = {}
    with open(KIN_SUMMARY) as f:
        for line in f:
            if ":" in line and line.startswith("    "):
                k, v = line.strip().split(":", 1)
                vals[k.strip()] = v.strip()
    with open(os.path.join(ROOT, "paper_1608_01125_amd/csrc/kinematics.hip"), "rb") as f:
        src = hashlib.sha256(f.read()).hexdigest()[:16]
    if vals.get("source_sha256") != src or vals.get("bulk_pairs") != str(n_pairs):
        return None
    return float(vals["traffic_bytes_per_dispatch"])


def kinematics_variant(T, torch, A, B, wl, n_steps, edges, reps=5):
    """Pair kinematics after one collision run (the run's unique pairs) and on a bulk list
    of 2^22 random pairs over the same beams, in random order and in the ascending (i, j)
    order tril_stats gives a run's pairs (the roofline's case): kernel time from HIP events on
    the library's stream, pairs per second and algorithmic GB/s."""
    import numpy as np
    g_edges = np.linspace(1.0, 40.0, 391)
    ctx = T.Context(wl.dt, edges)
    try:
        qb, tb = T.Beam(A), T.Beam(B)
        pairs = T.Pairs(1 << 21)
        T.run_steps(ctx, tb, qb, n_steps, pairs, graph=True)
        st = ctx.stats(pairs)
        n_run = st["n_pairs"]
        ms_run = min(T.tril_pair_kinematics(ctx, qb, tb, pairs, n_run, 1, g_edges, 90)["ms"]
                     for _ in range(reps))
        n = 1 << 22
        rng = np.random.default_rng(5)
        bi = rng.integers(0, len(A["E"]), n).astype(np.int32)
        bj = rng.integers(0, len(B["E"]), n).astype(np.int32)
        bk = rng.integers(0, n_steps, n).astype(np.int32)
        bulk = T.Pairs(n)
        ms_by_order = {}
        # random order, then ascending (i, j) as tril_stats leaves a run's pairs
        for order in ("random", "sorted"):
            o = np.arange(n) if order == "random" else np.lexsort((bj, bi))
            bulk.i.copy_(torch.from_numpy(bi[o]))
            bulk.j.copy_(torch.from_numpy(bj[o]))
            bulk.step.copy_(torch.from_numpy(bk[o]))
            T.tril_pair_kinematics(ctx, qb, tb, bulk, n, 1, g_edges, 90)  # warm-up
            ms_by_order[order] = [T.tril_pair_kinematics(ctx, qb, tb, bulk, n, 1, g_edges, 90)["ms"]
                                  for _ in range(reps)]
    finally:
        ctx.close()
    ms = ms_by_order["sorted"]
    avg = sum(ms) / len(ms)
    avg_random = sum(ms_by_order["random"]) / reps
    gbs = KIN_BYTES_PER_PAIR * n / (avg * 1e-3) / 1e9
    traffic = kinematics_traffic(n)
    # the oracle beside it: the same kinematics in plain Python floats, 3000 seeded pairs
    from oracle import kinematics_oracle as K
    rs = np.random.default_rng(6)
    ns = 3000
    si = rs.integers(0, len(A["E"]), ns)
    sj = rs.integers(0, len(B["E"]), ns)
    sk = rs.integers(0, n_steps, ns)
    t0 = time.perf_counter()
    pos, _ = K.kinematics(A, B, si, sj, sk, 1)
    K.histograms(A, B, si, sj, pos, g_edges, 90)
    cpu_s = time.perf_counter() - t0
    return {"cpu_oracle": {"pairs_per_s": ns / cpu_s, "cores": 1, "kind": "oracle",
                           "sample": f"{ns} seeded random pairs, Python floats, one thread"},
            "run_pairs": n_run, "run_pairs_ms": round(ms_run, 4),
            "bulk_pairs": n, "bulk_order": "ascending (i, j), as a run's pairs",
            "bulk_ms": round(avg, 4), "bulk_pairs_per_s": n / (avg * 1e-3),
            "bulk_random_order_ms": round(avg_random, 4),
            "roofline": {"bound": "hbm", "kernel": "k_pair_kin", "achieved": round(gbs, 2),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                         "traffic_achieved_GBs": (round(traffic / (avg * 1e-3) / 1e9, 2)
                                                  if traffic else None),
                         "alg_bytes_per_pair": KIN_BYTES_PER_PAIR}}


def cpu_baseline(A, offA, B, offB, dt, n_steps, target_s: float):
    """Oracle (as it stands) on a bounded random sample of query rows (per instance
    for a batched workload: rows drawn uniformly over all query photons)."""
    import numpy as np
    from oracle import oracle as O
    O.build(force=False)
    threads = O.num_threads()
    rng = np.random.default_rng(12345)
    nA = len(A["E"])
    if offA is None:
        offA = np.array([0, nA], dtype=np.int64)
        offB = np.array([0, len(B["E"])], dtype=np.int64)
    inst_of = np.searchsorted(offA, np.arange(nA), side="right") - 1
    r = min(nA, 64)
    while True:
        rows = np.sort(rng.choice(nA, r, replace=False))
        pairs_tested = 0
        t = time.perf_counter()
        for m in np.unique(inst_of[rows]):
            a0, a1, b0, b1 = offA[m], offA[m + 1], offB[m], offB[m + 1]
            if b1 <= b0:
                continue
            Am = {k: v[a0:a1] for k, v in A.items()}
            Bm = {k: v[b0:b1] for k, v in B.items()}
            sel = rows[inst_of[rows] == m] - a0
            O.collide(Am, Bm, dt, n_steps, rows=sel)
            pairs_tested += len(sel) * (b1 - b0)
        el = time.perf_counter() - t
        if el >= 0.5 * target_s or r >= nA:
            break
        r = int(min(nA, r * max(2.0, 1.1 * target_s / max(el, 1e-3))))
    # the paper's setting: one core (a tenth of the sample's rows, at least 8)
    r1 = max(8, r // 10)
    rows1 = np.sort(rng.choice(nA, r1, replace=False))
    O.set_threads(1)
    try:
        pairs1 = 0
        t = time.perf_counter()
        for m in np.unique(inst_of[rows1]):
            a0, a1, b0, b1 = offA[m], offA[m + 1], offB[m], offB[m + 1]
            if b1 <= b0:
                continue
            Am = {k: v[a0:a1] for k, v in A.items()}
            Bm = {k: v[b0:b1] for k, v in B.items()}
            sel = rows1[inst_of[rows1] == m] - a0
            O.collide(Am, Bm, dt, n_steps, rows=sel)
            pairs1 += len(sel) * (b1 - b0)
        el1 = time.perf_counter() - t
    finally:
        O.set_threads(threads)
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": pairs_tested * n_steps / el,
        "unit": "queries/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{r} random query rows x all target photons of their instance x {n_steps} "
                  f"steps ({pairs_tested} row-photon pairs, {el:.1f} s, FP64, pruned mode, OpenMP)",
        "value_one_thread": pairs1 * n_steps / el1,
        "sample_one_thread": f"{r1} random query rows, one thread, {el1:.1f} s",
        "host": {"nproc": os.cpu_count(), "cpu": cpu_model},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed benchmark steps (collision runs)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="gauss_headon_1m")
    ap.add_argument("--mode", choices=("batched", "graph", "per-step"), default="graph",
                    help="graph: value from tril_run replaying captured step batches, then the "
                         "same runs eagerly with HIP events around each phase for the phase "
                         "times and the roofline; batched: value from the eager runs; "
                         "per-step: one tril_build/tril_collide call per time step with events")
    ap.add_argument("--step-batch", type=int, default=0, help="time steps per launch (0 = automatic)")
    ap.add_argument("--physics-steps", type=int, default=0, help="0 = the workload's full run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the timed run with the query order taken from the first step")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this size first (counter calibration)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--kinetic-window", type=int, default=0,
                    help="steps per copy of the target hierarchy (0 = automatic, 1 = per step)")
    ap.add_argument("--descent-window", type=int, default=0,
                    help="steps per descent of a hierarchy copy (0 = automatic)")
    ap.add_argument("--st-mp", type=int, default=200_000,
                    help="st_headon: macro-particles per beam")
    ap.add_argument("--st-train", type=int, default=8, help="st_headon: training instances")
    ap.add_argument("--st-train-mp", default="",
                    help="st_headon: comma-separated macro-particle counts the training instances "
                         "cycle through (default: --st-mp for all)")
    ap.add_argument("--st-audit-sample", type=int, default=10_000,
                    help="st_headon: audit of the surrogate, expected macro-particles drawn per "
                         "beam and replicate")
    ap.add_argument("--st-judge-sample", type=int, default=100_000,
                    help="st_headon: judge (network-free sampled exact estimate), expected "
                         "macro-particles drawn per beam and replicate")
    ap.add_argument("--st-exact-max", type=int, default=1_000_000,
                    help="st_headon: largest macro-particle count the exact path runs on")
    ap.add_argument("--st-dep-mp", type=int, default=20_000,
                    help="st_headon: macro-particles per beam of the depletion measurement")
    ap.add_argument("--st-dep-physical", type=float, default=1e20,
                    help="st_headon: physical photons per beam of the depletion measurement")
    ap.add_argument("--st-train-steps", type=int, default=4000, help="st_headon: Adam steps")
    ap.add_argument("--autotune", action="store_true",
                    help="pick steps per launch, traversal workgroup size and Morton bits with "
                         "tril_autotune before timing (cached per workload shape)")
    ap.add_argument("--mlp-rows", type=int, default=1_000_000, help="mlp: inference rows")
    ap.add_argument("--mlp-train-steps", type=int, default=200, help="mlp: timed Adam steps")
    ap.add_argument("--traverse-queue", action="store_true",
                    help="traversal as a persistent grid taking queries from a work queue")
    ap.add_argument("--flags", type=int, default=0)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the collision path "
                                   "is not sharded across GPUs in this build", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1608_01125_amd import beams
    from paper_1608_01125_amd import tril as T

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "st_headon":
        return st_bench(args)
    if args.workload == "mlp":
        return mlp_bench(args)
    wl, A, offA, B, offB, n_steps = make_workload(args.workload, args.physics_steps)
    nA, nB = len(A["E"]), len(B["E"])
    if offA is None:
        pairs_per_step = nA * nB
    else:
        pairs_per_step = int(sum(int(offA[m + 1] - offA[m]) * int(offB[m + 1] - offB[m])
                                 for m in range(len(offA) - 1)))
    edges = beams.spectrum_edges()

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    graph = args.mode != "per-step"
    run_ms = []  # wall time of each timed run (filled by timed())

    def timed(flags):
        """Warm-up runs, then args.steps timed collision runs; returns (seconds, stats)."""
        ctx = T.Context(wl.dt, edges, flags=flags, block_traverse=args.block,
                        step_batch=args.step_batch, kinetic_window=args.kinetic_window,
                        descent_window=args.descent_window)
        if tune is not None:
            T.tril_set_tune(ctx.h, tune)
        pairs = T.Pairs(max(1 << 20, 4 * min(nA, nB)))
        run_ms.clear()

        def one_run():
            pairs.reset()
            T.run_steps(ctx, tb, qb, n_steps, pairs, graph=graph)
            return ctx.stats(pairs)

        try:
            for _ in range(args.warmup):
                one_run()
            ctx.reset_counters()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                tr = time.perf_counter()
                st = one_run()  # ends with tril_stats, which synchronises the stream
                run_ms.append(1e3 * (time.perf_counter() - tr))
            torch.cuda.synchronize()
            return time.perf_counter() - t0, st
        finally:
            ctx.close()

    tb, qb = T.Beam(B, offB), T.Beam(A, offA)
    tune = None
    if args.traverse_queue:
        tune = {"block_traverse": args.block or 64, "step_batch": args.step_batch,
                "morton_bits": 0, "traverse_queue": 1, "kinetic_window": args.kinetic_window,
                "descent_window": args.descent_window}
    if args.autotune:
        from paper_1608_01125_amd import autotune
        probe_ctx = T.Context(wl.dt, edges)
        try:
            # probe the whole run: a window of the densest steps favours other settings
            # than the run as timed
            tune = autotune.tuned(probe_ctx, tb, qb, wl.dt, k0=0, n_probe=n_steps,
                                  cache=autotune.DEFAULT_CACHE)
        finally:
            probe_ctx.close()
    timing = T.TRIL_TIMING
    if args.mode == "graph":
        # the value: full step batches replayed from captured graphs, no per-phase events
        g_elapsed, g_st = timed(args.flags)
        main_run_ms = sorted(run_ms)
        # the same runs eagerly with HIP events around every phase launch: phase times and
        # the traversal's launch durations (the kernels are the same)
        elapsed, st = timed(args.flags | timing)
        eager_ms = 1e3 * elapsed / max(args.steps, 1)
        assert g_st["n_pairs"] == st["n_pairs"] and g_st["n_hits"] == st["n_hits"]
        elapsed_value = g_elapsed
    else:
        elapsed, st = timed(args.flags | timing)
        main_run_ms = sorted(run_ms)
        eager_ms = 1e3 * elapsed / max(args.steps, 1)
        elapsed_value = elapsed
    ms_per_step = 1e3 * elapsed_value / max(args.steps, 1)
    value = pairs_per_step * n_steps / (elapsed_value / max(args.steps, 1))
    launches_per_run = st["n_timed_launches"] // max(args.steps, 1)
    steps_per_dispatch = round(n_steps / launches_per_run, 3) if launches_per_run else None

    variants = {}
    if not args.no_variants and not (args.flags & T.TRIL_SORT_QUERIES_ONCE):
        # same run with the query beam put in Morton order at its first step only (the pair
        # set is identical; only the traversal order of the queries differs)
        e2, st2 = timed(args.flags | T.TRIL_SORT_QUERIES_ONCE | timing)
        variants["query_order_from_first_step"] = {
            "value": pairs_per_step * n_steps / (e2 / max(args.steps, 1)),
            "ms_per_step": 1e3 * e2 / max(args.steps, 1), "pairs": st2["n_pairs"]}
    if not args.no_variants:
        # annihilation mode: photons that collide are consumed; the run's raw hits are
        # resolved chronologically on the device inside the timed stats call
        e3, st3 = timed(args.flags | T.TRIL_ANNIHILATE | timing)
        variants["annihilation"] = {
            "value": pairs_per_step * n_steps / (e3 / max(args.steps, 1)),
            "ms_per_step": 1e3 * e3 / max(args.steps, 1), "kept_hits": st3["n_hits"],
            "pairs": st3["n_pairs"]}

    if not args.no_variants and offA is None:
        # the same run with the uniform-grid broad phase (the mesh alternative to the
        # hierarchy; one step per launch, identical pair set)
        e4, st4 = timed(args.flags | T.TRIL_GRID | timing)
        variants["grid_broad_phase"] = {
            "value": pairs_per_step * n_steps / (e4 / max(args.steps, 1)),
            "ms_per_step": 1e3 * e4 / max(args.steps, 1), "pairs": st4["n_pairs"],
            "target_boxes_tested_per_query": round(st4["n_node_visits"] / max(st4["n_queries"], 1), 3),
            "candidates_per_run": st4["n_candidates"] // max(args.steps, 1),
            "ms_phases_per_run": {k: round(st4[k] / max(args.steps, 1), 3) for k in
                                  ("ms_build", "ms_query_prep", "ms_traverse", "ms_narrow")}}
        variants["pair_kinematics"] = kinematics_variant(T, torch, A, B, wl, n_steps, edges)

    roofline = roofline_vmem = None
    if st["n_collides"] > 0 and st["n_timed_launches"] > 0 and st["ms_traverse"] > 0:
        # Two roofs of the traversal (k_traverse), each with bytes over the timed region,
        # per launch, divided by the average launch duration from HIP events recorded
        # around every traversal launch on the library's stream.
        # HBM roof: the bytes the method must fetch from memory at least once: per
        # descent of a query row its order entry and its record (4 + 48 B; 4 + 32 B box
        # when every step is its own launch; a descent per step, or per descent window of
        # a copy's steps), every copy of the tree read once (64 B per internal node; a copy
        # per step, or per window of steps), with window copies every target record once
        # per launch (48 B), 8 B per candidate written.
        q_bytes = 52.0 if (steps_per_dispatch or 1) >= 2 else 36.0
        n_inst = 1 if offB is None else len(offB) - 1
        n_int_step = max(nB - n_inst, 0)
        n_launch = st["n_timed_launches"]
        runs = max(st["n_collides"] // max(n_steps, 1), 1)
        batches = batch_sizes(n_steps, launches_per_run)
        # the descent length the library used (automatic: adapted from run to run), and the
        # copy length that goes with it
        used = st.get("descent_window")
        win = tree_window(tune, args.kinetic_window,
                          used or descent_window(tune, args.descent_window, 32))
        dwin = used or descent_window(tune, args.descent_window, win)
        copies = sum(b if (win <= 1 or b < 2) else -(-b // win) for b in batches) * runs
        n_desc = sum(descents(b, win, dwin) for b in batches) * runs
        rec_bytes = 48.0 * nB * sum(1 for b in batches if win > 1 and b >= 2) * runs
        hbm_bytes = (q_bytes * nA * n_desc + 64.0 * n_int_step * copies + rec_bytes
                     + 8.0 * st["n_candidates"])
        # vector-memory roof: the bytes the kernel's loads deliver to its lanes, every node
        # load counted (64 B: all four slots' boxes, ids and bounds) and every leaf test
        # (96 B: the target's record and the query's, read again), plus the query bytes and
        # candidate stores above
        lane_bytes = (q_bytes * nA * n_desc + 64.0 * st["n_node_visits"]
                      + 96.0 * st["n_leaf_checks"] + 8.0 * st["n_candidates"])
        pmc = committed_counters(launches_per_run or None, win, dwin)
        traffic = pmc.get("traffic_bytes_per_dispatch")
        avg_s = st["ms_traverse"] * 1e-3 / n_launch
        achieved = hbm_bytes / n_launch / avg_s / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic,
                    "kernel": "k_traverse", "avg_launch_us": round(avg_s * 1e6, 3),
                    "steps_per_launch": steps_per_dispatch,
                    "alg_bytes_per_launch": round(hbm_bytes / n_launch, 1),
                    "traffic_achieved_GBs": (round(traffic / avg_s / 1e9, 2) if traffic else None),
                    "traffic_frac": (round(traffic / avg_s / 1e9 / HBM_PEAK_GBS, 4)
                                     if traffic else None),
                    "node_visits_per_query": round(st["n_node_visits"] / max(st["n_queries"], 1), 3),
                    "tree_copies_per_run": copies // runs, "kinetic_window": win,
                    "descent_window": dwin, "descents_per_row_per_run": n_desc // runs,
                    "leaf_checks_per_query": round(st["n_leaf_checks"] / max(st["n_queries"], 1), 5)}
        # vector-memory roof: every lane's node load returns through the CU's texture data
        # unit (TD), one unit per CU at the 2.4 GHz clock; its busy cycles per launch come
        # from the committed counter summary (TD_TD_BUSY over 256 CUs), so achieved / peak
        # is the fraction of the kernel's time that unit is busy
        td = pmc.get("TD_busy")
        peak_td = 256 * 2.4  # G TD cycles/s
        roofline_vmem = {"bound": "vmem", "achieved": round(td * peak_td, 2) if td else None,
                         "peak": peak_td, "unit": "G TD-busy cycles/s",
                         "frac": round(td, 4) if td else None,
                         "kernel": "k_traverse", "TA_busy": pmc.get("TA_busy"),
                         "L1_lookups_per_launch": pmc.get("L1_lookups_per_dispatch"),
                         "lane_bytes_per_launch": round(lane_bytes / n_launch, 1),
                         "lane_bytes_GBs": round(lane_bytes / n_launch / avg_s / 1e9, 2)}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_step_eager": round(eager_ms, 3),
        "ms_per_step_min_median_max": [round(main_run_ms[0], 3),
                                       round(main_run_ms[len(main_run_ms) // 2], 3),
                                       round(main_run_ms[-1], 3)] if main_run_ms else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_per_beam": [nA, nB],
                   "instances": 1 if offA is None else len(offA) - 1,
                   "pairs_per_step": pairs_per_step, "time_steps": n_steps,
                   "tune": tune,
                   "dt_um_per_c": wl.dt, "weight": wl.a.w, "mode": args.mode,
                   "step_batch": args.step_batch, "steps_per_launch": steps_per_dispatch,
                   "query_order": ("first step's Morton order" if args.flags & T.TRIL_SORT_QUERIES_ONCE
                                   else "Morton order of every step"),
                   "timing": ("graph replay" if args.mode == "graph" else "eager, per-phase events"),
                   "traversal_launches": st["n_timed_launches"],
                   "pairs": st["n_pairs"], "hits": st["n_hits"],
                   "candidates_per_run": st["n_candidates"] // max(args.steps, 1),
                   "fp64_recheck_fraction": (round(st["n_fp64_rechecks"] / st["n_candidates"], 5)
                                             if st["n_candidates"] else None),
                   "ms_phases_per_run": {k: round(st[k] / max(args.steps, 1), 3) for k in
                                         ("ms_build", "ms_query_prep", "ms_traverse", "ms_narrow")}},
        "roofline": roofline,
        "roofline_vmem": roofline_vmem,
    }
    if variants:
        out["variants"] = variants
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, offA, B, offB, wl.dt, n_steps, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
