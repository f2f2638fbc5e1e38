"""Python binding of libtril (C ABI in include/tril.h and include/tril_debug.h).

Argument marshalling only: every step of the collision path runs in the HIP
kernels of libtril.so. PyTorch provides device memory and the HIP stream.
Importing this module without the built library raises immediately; there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtril.so")

TRIL_OK = 0
TRIL_E_INVAL = -1
TRIL_E_NOMEM = -2
TRIL_E_OVERFLOW = -3
TRIL_E_HIP = -4
TRIL_E_NOTIMPL = -5
TRIL_E_STATE = -6
TRIL_E_DATA = -7
TRIL_E_INTERNAL = -8

TRIL_TIMING = 0x1
TRIL_SORT_QUERIES_ONCE = 0x2
TRIL_FP64_NARROW = 0x4
TRIL_ANNIHILATE = 0x8
TRIL_GRID = 0x10

FIELDS = ("x", "y", "z", "px", "py", "pz", "E", "w")
_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


class tril_beam(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [(f, ctypes.c_void_p) for f in FIELDS] + [
        ("n_inst", ctypes.c_int32), ("inst_off", _i64p)]


class tril_params(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("flags", ctypes.c_uint32), ("n_bins", ctypes.c_int32),
                ("bin_edges", _dp), ("cand_cap", ctypes.c_int64),
                ("block_traverse", ctypes.c_int32), ("step_batch", ctypes.c_int32),
                ("morton_bits", ctypes.c_int32), ("kinetic_window", ctypes.c_int32),
                ("descent_window", ctypes.c_int32)]


class tril_pairs(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_int64), ("i", ctypes.c_void_p), ("j", ctypes.c_void_p),
                ("step", ctypes.c_void_p), ("count", ctypes.c_void_p)]


class tril_stats_t(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_int64), ("n_hits", ctypes.c_int64),
                ("n_candidates", ctypes.c_int64), ("n_node_visits", ctypes.c_int64),
                ("n_queries", ctypes.c_int64), ("n_sigma_evals", ctypes.c_int64),
                ("n_builds", ctypes.c_int64), ("n_collides", ctypes.c_int64),
                ("yield_", ctypes.c_double), ("spectrum", _dp), ("step_counts", _i64p),
                ("n_step_counts", ctypes.c_int32), ("descent_window", ctypes.c_int32),
                ("ms_build", ctypes.c_double), ("ms_query_prep", ctypes.c_double),
                ("ms_traverse", ctypes.c_double), ("ms_narrow", ctypes.c_double),
                ("n_timed_launches", ctypes.c_int64), ("n_fp64_rechecks", ctypes.c_int64),
                ("n_leaf_checks", ctypes.c_int64)]


class tril_tune(ctypes.Structure):
    _fields_ = [("block_traverse", ctypes.c_int32), ("step_batch", ctypes.c_int32),
                ("morton_bits", ctypes.c_int32), ("traverse_queue", ctypes.c_int32),
                ("kinetic_window", ctypes.c_int32), ("descent_window", ctypes.c_int32),
                ("ms_per_step", ctypes.c_double)]


class tril_st_grid(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("n_pos", ctypes.c_int32 * 3), ("n_e", ctypes.c_int32),
                ("e_lo", ctypes.c_double), ("e_hi", ctypes.c_double),
                ("n_th", ctypes.c_int32), ("pad0", ctypes.c_int32), ("th_max", ctypes.c_double),
                ("axis", ctypes.c_double * 3), ("t_bin", ctypes.c_double)]


class tril_st_table(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_int64), ("key", ctypes.c_void_p), ("yield_", ctypes.c_void_p)]


class tril_st_sur_params(ctypes.Structure):
    _fields_ = [("cloud_factor", ctypes.c_double), ("eps", ctypes.c_double),
                ("gate", ctypes.c_double), ("scale", ctypes.c_double),
                ("gate_mode", ctypes.c_int32), ("pad0", ctypes.c_int32),
                ("audit_sample", ctypes.c_int64), ("audit_reps", ctypes.c_int32),
                ("pad1", ctypes.c_int32), ("audit_seed", ctypes.c_uint64)]


class tril_st_sur_result(ctypes.Structure):
    _fields_ = [("total", ctypes.c_double), ("surrogate_part", ctypes.c_double),
                ("exact_part", ctypes.c_double), ("n_bin_pairs", ctypes.c_int64),
                ("n_gated", ctypes.c_int64), ("ms", ctypes.c_double),
                ("predicted_spread", ctypes.c_double), ("audit_half_width", ctypes.c_double),
                ("audit_sampled", ctypes.c_int64)]


class tril_st_audit_params(ctypes.Structure):
    _fields_ = [("n_sample", ctypes.c_int64), ("n_rep", ctypes.c_int32),
                ("control", ctypes.c_int32), ("seed", ctypes.c_uint64), ("mix", ctypes.c_double)]


class tril_st_audit_result(ctypes.Structure):
    _fields_ = [("estimate", ctypes.c_double), ("half_width", ctypes.c_double),
                ("control_total", ctypes.c_double), ("control_scale", ctypes.c_double),
                ("rep", ctypes.c_double * 64),
                ("n_rep", ctypes.c_int32), ("pad0", ctypes.c_int32),
                ("n_sampled", ctypes.c_int64 * 2), ("n_bin_pairs", ctypes.c_int64),
                ("ms", ctypes.c_double)]


class tril_kin_params(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("n_gamma", ctypes.c_int32),
                ("n_theta", ctypes.c_int32), ("gamma_edges", _dp)]


class tril_kin_out(ctypes.Structure):
    _fields_ = [("gamma_hist", _dp), ("theta_hist", _dp), ("ms_kernel", ctypes.c_double)]


TRIL_KIN_MAX_BINS = 2048

EXPORTS = ("tril_create", "tril_build", "tril_collide", "tril_run", "tril_stats",
           "tril_pair_kinematics", "tril_pair_kinematics_noalloc",
           "tril_autotune", "tril_set_tune", "tril_st_bin", "tril_st_exact",
           "tril_st_exact_depleted", "tril_ip_swarm",
           "tril_mlp_create", "tril_mlp_destroy", "tril_mlp_set_params", "tril_mlp_get_params",
           "tril_mlp_set_norm", "tril_mlp_fit_norm", "tril_mlp_grad", "tril_mlp_train",
           "tril_mlp_predict", "tril_st_features", "tril_st_targets", "tril_st_surrogate",
           "tril_st_audit", "tril_st_calibrate", "tril_dbg_st_audit_sample",
           "tril_dbg_gemm_bf16",
           "tril_reset_counters", "tril_destroy", "tril_strerror", "tril_last_hip_error",
           "tril_dbg_sort_u32", "tril_dbg_sort_u64", "tril_dbg_morton", "tril_dbg_pair_eval",
           "tril_dbg_pair_eval32", "tril_dbg_math",
           "tril_dbg_tree", "tril_dbg_keep_nodes", "tril_dbg_target_records", "tril_dbg_quad_nodes", "tril_dbg_boxes", "tril_dbg_target_rows", "tril_dbg_query_records", "tril_dbg_candidates")

_lib = None


def lib() -> ctypes.CDLL:
    """Load libtril.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libtril.so not built ({LIB_PATH}); run paper_1608_01125_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.tril_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(tril_params), vp]
    L.tril_build.argtypes = [vp, ctypes.POINTER(tril_beam), i32]
    L.tril_collide.argtypes = [vp, ctypes.POINTER(tril_beam), i32, ctypes.POINTER(tril_pairs)]
    L.tril_run.argtypes = [vp, ctypes.POINTER(tril_beam), ctypes.POINTER(tril_beam), i32, i32,
                           ctypes.POINTER(tril_pairs)]
    L.tril_stats.argtypes = [vp, ctypes.POINTER(tril_pairs), ctypes.POINTER(tril_stats_t)]
    L.tril_pair_kinematics_noalloc.argtypes = [ctypes.POINTER(tril_beam), ctypes.POINTER(tril_beam),
                                               ctypes.POINTER(tril_pairs), i64, ctypes.c_uint64,
                                               i32, vp, i32, vp, vp, vp, vp, vp]
    L.tril_pair_kinematics.argtypes = [vp, ctypes.POINTER(tril_beam), ctypes.POINTER(tril_beam),
                                       ctypes.POINTER(tril_pairs), i64,
                                       ctypes.POINTER(tril_kin_params), vp,
                                       ctypes.POINTER(tril_kin_out)]
    L.tril_autotune.argtypes = [vp, ctypes.POINTER(tril_beam), ctypes.POINTER(tril_beam), i32, i32,
                                ctypes.POINTER(tril_tune)]
    L.tril_set_tune.argtypes = [vp, ctypes.POINTER(tril_tune)]
    L.tril_st_bin.argtypes = [ctypes.POINTER(tril_beam), ctypes.POINTER(tril_st_grid), vp, vp, vp]
    L.tril_st_exact.argtypes = [vp, ctypes.POINTER(tril_beam), vp, i64, ctypes.POINTER(tril_beam),
                                vp, ctypes.POINTER(ctypes.c_double), i32, i32,
                                ctypes.POINTER(tril_st_table), ctypes.POINTER(ctypes.c_double)]
    L.tril_st_exact_depleted.argtypes = [vp, ctypes.POINTER(tril_beam), vp, i64,
                                         ctypes.POINTER(tril_beam), vp,
                                         ctypes.POINTER(ctypes.c_double), i32, i32,
                                         ctypes.POINTER(tril_st_table),
                                         ctypes.POINTER(tril_st_table),
                                         ctypes.POINTER(ctypes.c_double)]
    L.tril_ip_swarm.argtypes = [vp, ctypes.POINTER(tril_beam), vp, i64, ctypes.POINTER(tril_beam),
                                vp, ctypes.POINTER(ctypes.c_double), i32, i32,
                                ctypes.POINTER(tril_st_table), ctypes.POINTER(tril_st_table),
                                ctypes.POINTER(ctypes.c_int64)]
    fp, dp = ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)
    L.tril_mlp_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.c_uint64, vp]
    L.tril_mlp_destroy.argtypes = [vp]
    L.tril_mlp_destroy.restype = None
    L.tril_mlp_set_params.argtypes = [vp, i32, fp, i64]
    L.tril_mlp_get_params.argtypes = [vp, i32, fp, i64]
    L.tril_mlp_set_norm.argtypes = [vp, fp, fp, ctypes.c_float, ctypes.c_float]
    L.tril_mlp_fit_norm.argtypes = [vp, vp, vp, i64]
    L.tril_mlp_grad.argtypes = [vp, i32, vp, vp, i64, fp, dp]
    L.tril_mlp_train.argtypes = [vp, vp, vp, i64, i32, i32, ctypes.c_float, ctypes.c_uint64, dp]
    L.tril_mlp_predict.argtypes = [vp, vp, i64, vp, vp]
    L.tril_dbg_gemm_bf16.argtypes = [vp, i64, i64, vp, i64, i64, i32, i32, i32, vp, vp]
    gp = ctypes.POINTER(tril_st_grid)
    L.tril_st_features.argtypes = [vp, vp, gp, vp, gp, i32, i32, ctypes.POINTER(tril_st_sur_params),
                                   vp, vp, vp, i64, ctypes.POINTER(ctypes.c_int64)]
    L.tril_st_targets.argtypes = [vp, vp, i64, ctypes.POINTER(tril_st_table), ctypes.c_double, vp,
                                  vp, vp]
    L.tril_st_surrogate.argtypes = [vp, vp, ctypes.POINTER(tril_beam), vp, vp, gp,
                                    ctypes.POINTER(tril_beam), vp, vp, gp, i32, i32,
                                    ctypes.POINTER(tril_st_sur_params),
                                    ctypes.POINTER(tril_st_sur_result)]
    L.tril_reset_counters.argtypes = [vp]
    L.tril_destroy.argtypes = [vp]
    L.tril_destroy.restype = None
    L.tril_strerror.argtypes = [ctypes.c_int]
    L.tril_strerror.restype = ctypes.c_char_p
    L.tril_last_hip_error.argtypes = []
    L.tril_last_hip_error.restype = ctypes.c_char_p
    L.tril_dbg_sort_u32.argtypes = [vp, vp, i64, ctypes.c_int, vp]
    L.tril_dbg_sort_u64.argtypes = [vp, vp, i64, ctypes.c_int, vp]
    L.tril_dbg_morton.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_float), vp, vp]
    L.tril_dbg_pair_eval.argtypes = [i64, vp, vp, vp]
    L.tril_dbg_pair_eval32.argtypes = [i64, vp, vp, vp]
    L.tril_dbg_math.argtypes = [ctypes.c_int, i64, vp, vp, vp, vp]
    L.tril_dbg_tree.argtypes = [vp, vp, i64, _i64p, _i32p]
    L.tril_dbg_keep_nodes.argtypes = [vp, ctypes.c_int32]
    L.tril_dbg_target_records.argtypes = [vp, vp, i64, _i64p, _i32p]
    L.tril_dbg_quad_nodes.argtypes = [vp, vp, i64, _i64p, ctypes.POINTER(ctypes.c_float), _i32p]
    L.tril_st_audit.argtypes = [vp, vp, ctypes.POINTER(tril_beam), vp, vp, gp,
                                ctypes.POINTER(tril_beam), vp, vp, gp, i32, i32,
                                ctypes.POINTER(tril_st_sur_params),
                                ctypes.POINTER(tril_st_audit_params),
                                ctypes.POINTER(tril_st_audit_result)]
    L.tril_st_calibrate.argtypes = [vp, vp, vp, vp, i64, ctypes.c_double,
                                    ctypes.POINTER(ctypes.c_double)]
    L.tril_dbg_st_audit_sample.argtypes = [vp, ctypes.c_int, _i32p, _dp, i64, _i64p]
    L.tril_dbg_boxes.argtypes = [vp, ctypes.c_int, vp, i64, _i64p]
    L.tril_dbg_query_records.argtypes = [vp, i32, vp, i64, _i64p]
    L.tril_dbg_target_rows.argtypes = [vp, _i32p, i64, _i64p]
    L.tril_dbg_candidates.argtypes = [vp, _i32p, _i32p, i64, _i64p]
    _lib = L
    return L


class TrilError(RuntimeError):
    def __init__(self, code: int, where: str):
        L = lib()
        msg = L.tril_strerror(code).decode()
        hip = L.tril_last_hip_error().decode()
        super().__init__(f"{where}: {msg} ({code})" + (f" [{hip}]" if hip and code == TRIL_E_HIP else ""))
        self.code = code


def _check(code: int, where: str) -> None:
    if code != TRIL_OK:
        raise TrilError(code, where)


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


# ------------------------------------------------------------------ marshalling


class Beam:
    """Device-resident beam (FP64 SoA torch tensors) plus host CSR instance offsets."""

    def __init__(self, arrays: Dict[str, "object"], inst_off: Optional[Sequence[int]] = None,
                 device: str = "cuda"):
        import torch
        self.t = {}
        for f in FIELDS:
            a = arrays[f]
            if isinstance(a, np.ndarray):
                a = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
            self.t[f] = a.to(device=device, dtype=torch.float64).contiguous()
        self.n = int(self.t["E"].numel())
        if inst_off is None:
            self.off = None
            self.n_inst = 1
        else:
            self.off = np.ascontiguousarray(np.asarray(inst_off, dtype=np.int64))
            self.n_inst = len(self.off) - 1
        self._c = tril_beam()
        self._c.n = self.n
        for f in FIELDS:
            setattr(self._c, f, self.t[f].data_ptr() if self.n > 0 else None)
        self._c.n_inst = self.n_inst
        self._c.inst_off = (self.off.ctypes.data_as(_i64p) if self.off is not None else None)

    @property
    def c(self) -> tril_beam:
        return self._c


class Pairs:
    """Caller-owned device pair buffer (i, j, step) with a device counter."""

    def __init__(self, cap: int, device: str = "cuda"):
        import torch
        self.cap = int(cap)
        self.i = torch.empty(max(self.cap, 1), dtype=torch.int32, device=device)
        self.j = torch.empty(max(self.cap, 1), dtype=torch.int32, device=device)
        self.step = torch.empty(max(self.cap, 1), dtype=torch.int32, device=device)
        self.count = torch.zeros(1, dtype=torch.int64, device=device)
        self._c = tril_pairs(self.cap, self.i.data_ptr(), self.j.data_ptr(),
                             self.step.data_ptr(), self.count.data_ptr())

    def reset(self) -> None:
        self.count.zero_()

    @property
    def c(self) -> tril_pairs:
        return self._c

    def numpy(self):
        n = int(self.count.item())
        n = min(n, self.cap)
        return (self.i[:n].cpu().numpy(), self.j[:n].cpu().numpy(), self.step[:n].cpu().numpy())


# ------------------------------------------------------- C-named entry points


def tril_create(dt: float, edges: Optional[np.ndarray] = None, flags: int = 0,
                cand_cap: int = 0, block_traverse: int = 0, step_batch: int = 0,
                stream=None, morton_bits: int = 0, kinetic_window: int = 0,
                descent_window: int = 0) -> ctypes.c_void_p:
    L = lib()
    p = tril_params()
    p.dt = float(dt)
    p.flags = int(flags)
    keep = None
    if edges is not None and len(edges) > 1:
        keep = np.ascontiguousarray(edges, dtype=np.float64)
        p.n_bins = len(keep) - 1
        p.bin_edges = keep.ctypes.data_as(_dp)
    else:
        p.n_bins = 0
        p.bin_edges = None
    p.cand_cap = int(cand_cap)
    p.block_traverse = int(block_traverse)
    p.step_batch = int(step_batch)
    p.morton_bits = int(morton_bits)
    p.kinetic_window = int(kinetic_window)
    p.descent_window = int(descent_window)
    h = ctypes.c_void_p()
    _check(L.tril_create(ctypes.byref(h), ctypes.byref(p), ctypes.c_void_p(_stream(stream))),
           "tril_create")
    return h


def tril_build(ctx, target: Beam, step: int) -> None:
    _check(lib().tril_build(ctx, ctypes.byref(target.c), int(step)), "tril_build")


def tril_collide(ctx, query: Beam, step: int, pairs: Pairs) -> None:
    _check(lib().tril_collide(ctx, ctypes.byref(query.c), int(step), ctypes.byref(pairs.c)),
           "tril_collide")


def tril_run(ctx, target: Beam, query: Beam, k0: int, n_steps: int, pairs: Pairs) -> None:
    _check(lib().tril_run(ctx, ctypes.byref(target.c), ctypes.byref(query.c), int(k0),
                          int(n_steps), ctypes.byref(pairs.c)), "tril_run")


def tril_pair_kinematics(ctx, query: Beam, target: Beam, pairs: Pairs, n: int, seed: int,
                         gamma_edges: Optional[np.ndarray] = None, n_theta: int = 0,
                         leptons: bool = True, check: bool = True) -> dict:
    """Leptons (device float64 tensor (n, 8): positron E px py pz, electron E px py pz) of
    the first n pairs, and the positron Lorentz-factor and polar-angle histograms."""
    import torch
    kp = tril_kin_params()
    kp.seed = int(seed) & ((1 << 64) - 1)
    keep = None
    if gamma_edges is not None and len(gamma_edges) > 1:
        keep = np.ascontiguousarray(gamma_edges, dtype=np.float64)
        kp.n_gamma = len(keep) - 1
        kp.gamma_edges = keep.ctypes.data_as(_dp)
    else:
        kp.n_gamma = 0
        kp.gamma_edges = None
    kp.n_theta = int(n_theta)
    gh = np.zeros(max(kp.n_gamma, 1))
    th = np.zeros(max(kp.n_theta, 1))
    out = tril_kin_out()
    out.gamma_hist = gh.ctypes.data_as(_dp) if kp.n_gamma > 0 else None
    out.theta_hist = th.ctypes.data_as(_dp) if kp.n_theta > 0 else None
    lep = (torch.empty((max(int(n), 1), 8), dtype=torch.float64, device=pairs.i.device)
           if leptons else None)
    code = lib().tril_pair_kinematics(_h(ctx), ctypes.byref(query.c), ctypes.byref(target.c),
                                      ctypes.byref(pairs.c), int(n), ctypes.byref(kp),
                                      lep.data_ptr() if lep is not None else None,
                                      ctypes.byref(out))
    if check:
        _check(code, "tril_pair_kinematics")
    return {"code": code, "leptons": lep[:int(n)] if lep is not None else None,
            "gamma_hist": gh[:kp.n_gamma], "theta_hist": th[:kp.n_theta], "ms": out.ms_kernel}


def tril_pair_kinematics_noalloc(query: Beam, target: Beam, pairs: Pairs, n: int, seed: int,
                                 gamma_edges, gamma_hist, n_theta: int, theta_hist, leptons,
                                 status, stream=None) -> int:
    """The no-allocation variant: every array is a caller-owned device tensor (gamma_edges
    float64 n_gamma + 1 or None, gamma_hist float64 n_gamma, theta_hist float64 n_theta,
    leptons float64 (n, 8) or None, status int32 (1,)); asynchronous on the stream.
    Returns the call's return code (the device status lands in `status`)."""
    n_gamma = 0 if gamma_edges is None else int(gamma_edges.numel()) - 1
    return lib().tril_pair_kinematics_noalloc(
        ctypes.byref(query.c), ctypes.byref(target.c), ctypes.byref(pairs.c), int(n),
        int(seed) & ((1 << 64) - 1), n_gamma,
        gamma_edges.data_ptr() if gamma_edges is not None else None, int(n_theta),
        leptons.data_ptr() if leptons is not None else None,
        gamma_hist.data_ptr() if gamma_hist is not None else None,
        theta_hist.data_ptr() if theta_hist is not None else None, status.data_ptr(),
        _stream(stream))


TUNE_KEYS = ("block_traverse", "step_batch", "morton_bits", "traverse_queue", "kinetic_window",
             "descent_window")


def tril_autotune(ctx, target: Beam, query: Beam, k0: int, n_probe: int) -> dict:
    t = tril_tune()
    _check(lib().tril_autotune(_h(ctx), ctypes.byref(target.c), ctypes.byref(query.c), int(k0),
                               int(n_probe), ctypes.byref(t)), "tril_autotune")
    return {"block_traverse": t.block_traverse, "step_batch": t.step_batch,
            "morton_bits": t.morton_bits, "traverse_queue": t.traverse_queue,
            "kinetic_window": t.kinetic_window, "descent_window": t.descent_window,
            "ms_per_step": t.ms_per_step}


def tril_set_tune(ctx, tune: dict) -> None:
    t = tril_tune()
    for k in TUNE_KEYS:
        setattr(t, k, int(tune.get(k, 0)))
    _check(lib().tril_set_tune(_h(ctx), ctypes.byref(t)), "tril_set_tune")


def st_grid(g) -> tril_st_grid:
    """tril_st_grid from any object with the fields lo, hi, n_pos, n_e, e_lo, e_hi, n_th,
    th_max, axis, t_bin."""
    c = tril_st_grid()
    for a in range(3):
        c.lo[a] = float(g.lo[a])
        c.hi[a] = float(g.hi[a])
        c.n_pos[a] = int(g.n_pos[a])
        c.axis[a] = float(g.axis[a])
    c.n_e, c.e_lo, c.e_hi = int(g.n_e), float(g.e_lo), float(g.e_hi)
    c.n_th, c.th_max, c.t_bin = int(g.n_th), float(g.th_max), float(g.t_bin)
    return c


def tril_st_bin(beam: Beam, grid, bins, sums=None, stream=None) -> None:
    """bins: int32 device tensor (n); sums: float64 device tensor (n_bins, 5) or None."""
    g = st_grid(grid)
    _check(lib().tril_st_bin(ctypes.byref(beam.c), ctypes.byref(g), bins.data_ptr(),
                             sums.data_ptr() if sums is not None else None, _stream(stream)),
           "tril_st_bin")


class StTable:
    """Caller-owned bin-pair table on the device (open addressing, power-of-two slots)."""

    def __init__(self, cap_log2: int, device: str = "cuda"):
        import torch
        self.cap = 1 << int(cap_log2)
        self.key = torch.empty(self.cap, dtype=torch.int64, device=device)
        self.yield_ = torch.empty(self.cap, dtype=torch.float64, device=device)
        self._c = tril_st_table(self.cap, self.key.data_ptr(), self.yield_.data_ptr())

    @property
    def c(self) -> tril_st_table:
        return self._c

    def items(self):
        """(keys, yields) of the occupied slots, as numpy arrays sorted by key."""
        k = self.key.cpu().numpy()
        y = self.yield_.cpu().numpy()
        occ = k >= 0
        order = np.argsort(k[occ], kind="stable")
        return k[occ][order], y[occ][order]


def tril_st_exact(ctx, target: Beam, t_bins, n_target_bins: int, query: Beam, q_bins, cell,
                  k0: int, n_steps: int, table: StTable) -> float:
    c3 = (ctypes.c_double * 3)(*[float(v) for v in cell])
    tot = ctypes.c_double(0.0)
    _check(lib().tril_st_exact(_h(ctx), ctypes.byref(target.c),
                               t_bins.data_ptr() if target.n > 0 else None, int(n_target_bins),
                               ctypes.byref(query.c), q_bins.data_ptr() if query.n > 0 else None,
                               c3, int(k0), int(n_steps), ctypes.byref(table.c),
                               ctypes.byref(tot)), "tril_st_exact")
    return tot.value


def tril_st_exact_depleted(ctx, target: Beam, t_bins, n_target_bins: int, query: Beam, q_bins,
                           cell, k0: int, n_steps: int, pair_table: StTable,
                           table: StTable) -> float:
    """Depleted ST yields: per cloud pair in pair_table (key i * n_target + j), per bin pair in
    table; returns the total."""
    c3 = (ctypes.c_double * 3)(*[float(v) for v in cell])
    tot = ctypes.c_double(0.0)
    _check(lib().tril_st_exact_depleted(
        _h(ctx), ctypes.byref(target.c), t_bins.data_ptr() if target.n > 0 else None,
        int(n_target_bins), ctypes.byref(query.c), q_bins.data_ptr() if query.n > 0 else None,
        c3, int(k0), int(n_steps), ctypes.byref(pair_table.c), ctypes.byref(table.c),
        ctypes.byref(tot)), "tril_st_exact_depleted")
    return tot.value


def tril_ip_swarm(ctx, target: Beam, t_bins, n_target_bins: int, query: Beam, q_bins, cell,
                  k0: int, n_steps: int, pair_table: StTable, table: StTable) -> int:
    """IP-regime swarms: colliding real-photon pairs per macro-particle pair in pair_table
    (key i * n_target + j), per bin pair in table; returns the total."""
    c3 = (ctypes.c_double * 3)(*[float(v) for v in cell])
    tot = ctypes.c_int64(0)
    _check(lib().tril_ip_swarm(
        _h(ctx), ctypes.byref(target.c), t_bins.data_ptr() if target.n > 0 else None,
        int(n_target_bins), ctypes.byref(query.c), q_bins.data_ptr() if query.n > 0 else None,
        c3, int(k0), int(n_steps), ctypes.byref(pair_table.c), ctypes.byref(table.c),
        ctypes.byref(tot)), "tril_ip_swarm")
    return int(tot.value)


MLP_PARAMS = 133_633


class Mlp:
    """Surrogate ensemble (tril_mlp_*): device tensors in, device tensors out."""

    def __init__(self, n_members: int, seed: int = 0, stream=None):
        self.K = int(n_members)
        h = ctypes.c_void_p()
        _check(lib().tril_mlp_create(ctypes.byref(h), self.K, ctypes.c_uint64(seed),
                                     ctypes.c_void_p(_stream(stream))), "tril_mlp_create")
        self.h = h

    def close(self) -> None:
        if self.h:
            lib().tril_mlp_destroy(self.h)
            self.h = None

    def get_params(self, member: int) -> np.ndarray:
        out = np.empty(MLP_PARAMS, dtype=np.float32)
        _check(lib().tril_mlp_get_params(self.h, member, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                         MLP_PARAMS), "tril_mlp_get_params")
        return out

    def set_params(self, member: int, p: np.ndarray) -> None:
        a = np.ascontiguousarray(p, dtype=np.float32)
        _check(lib().tril_mlp_set_params(self.h, member, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                         len(a)), "tril_mlp_set_params")

    def set_norm(self, mu_x, sd_x, mu_y: float, sd_y: float) -> None:
        mx = np.ascontiguousarray(mu_x, dtype=np.float32)
        sx = np.ascontiguousarray(sd_x, dtype=np.float32)
        fp = ctypes.POINTER(ctypes.c_float)
        _check(lib().tril_mlp_set_norm(self.h, mx.ctypes.data_as(fp), sx.ctypes.data_as(fp),
                                       float(mu_y), float(sd_y)), "tril_mlp_set_norm")

    def fit_norm(self, x, y) -> None:
        _check(lib().tril_mlp_fit_norm(self.h, x.data_ptr(), y.data_ptr(), x.shape[0]),
               "tril_mlp_fit_norm")

    def grad(self, member: int, x, y):
        g = np.empty(MLP_PARAMS, dtype=np.float32)
        loss = ctypes.c_double(0.0)
        _check(lib().tril_mlp_grad(self.h, member, x.data_ptr(), y.data_ptr(), x.shape[0],
                                   g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                   ctypes.byref(loss)), "tril_mlp_grad")
        return loss.value, g

    def train(self, x, y, n_steps: int, batch: int, lr: float, seed: int = 0) -> np.ndarray:
        losses = np.zeros(self.K, dtype=np.float64)
        _check(lib().tril_mlp_train(self.h, x.data_ptr(), y.data_ptr(), x.shape[0], int(n_steps),
                                    int(batch), float(lr), ctypes.c_uint64(seed),
                                    losses.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "tril_mlp_train")
        return losses

    def predict(self, x):
        import torch
        n = x.shape[0]
        mean = torch.empty(max(n, 1), dtype=torch.float32, device=x.device)
        sdev = torch.empty(max(n, 1), dtype=torch.float32, device=x.device)
        _check(lib().tril_mlp_predict(self.h, x.data_ptr() if n else None, n, mean.data_ptr(),
                                      sdev.data_ptr()), "tril_mlp_predict")
        return mean[:n], sdev[:n]


def sur_params(cloud_factor: float = 0.0, eps: float = 0.0, gate: float = 0.0,
               scale: float = 0.0, per_pair: bool = False, audit: bool = False,
               audit_sample: int = 0, audit_reps: int = 0,
               audit_seed: int = 0) -> tril_st_sur_params:
    mode = 2 if audit else (1 if per_pair else 0)
    return tril_st_sur_params(cloud_factor, eps, gate, scale, mode, 0, int(audit_sample),
                              int(audit_reps), 0, int(audit_seed) & ((1 << 64) - 1))


AUDIT_NETWORK, AUDIT_BIN_LEVEL, AUDIT_NONE = 0, 1, 2


def tril_st_audit(ctx, mlp, target: Beam, t_bins, t_sums, t_grid, query: Beam, q_bins, q_sums,
                  q_grid, k0: int, n_steps: int, control: int, n_sample: int = 0, n_rep: int = 0,
                  seed: int = 0, mix: float = 0.0, sur=None) -> dict:
    """Sampled estimate of the exact total (see tril.h); returns the result fields, with the
    replicate estimates as a list."""
    r = tril_st_audit_result()
    gq, gt = st_grid(q_grid), st_grid(t_grid)
    ap = tril_st_audit_params(int(n_sample), int(n_rep), int(control),
                              int(seed) & ((1 << 64) - 1), float(mix))
    sp = sur or sur_params()
    _check(lib().tril_st_audit(_h(ctx), mlp.h if mlp is not None else None,
                               ctypes.byref(target.c), t_bins.data_ptr() if target.n else None,
                               t_sums.data_ptr(), ctypes.byref(gt), ctypes.byref(query.c),
                               q_bins.data_ptr() if query.n else None, q_sums.data_ptr(),
                               ctypes.byref(gq), int(k0), int(n_steps), ctypes.byref(sp),
                               ctypes.byref(ap), ctypes.byref(r)), "tril_st_audit")
    out = {k: getattr(r, k) for k, _ in tril_st_audit_result._fields_
           if k not in ("rep", "n_sampled", "pad0")}
    out["rep"] = list(r.rep[: r.n_rep])
    out["n_sampled"] = (r.n_sampled[0], r.n_sampled[1])
    return out


def tril_st_calibrate(mlp, x, y0, y_exact, eps: float = 1e-3) -> float:
    """Exact over predicted total on feature rows (device tensors), reduced in a fixed
    order in the library."""
    out = ctypes.c_double(0.0)
    _check(lib().tril_st_calibrate(mlp.h, x.data_ptr(), y0.data_ptr(), y_exact.data_ptr(),
                                   int(x.shape[0]), float(eps), ctypes.byref(out)),
           "tril_st_calibrate")
    return out.value


def tril_dbg_st_audit_sample(ctx, side: int, cap: int):
    """Rows and inclusion probabilities of the last replicate's thinned beam (side 0 query,
    1 target), host arrays."""
    rows = np.zeros(max(cap, 1), dtype=np.int32)
    pis = np.zeros(max(cap, 1), dtype=np.float64)
    n = ctypes.c_int64(0)
    _check(lib().tril_dbg_st_audit_sample(_h(ctx), int(side), rows.ctypes.data_as(_i32p),
                                          pis.ctypes.data_as(_dp), max(cap, 1), ctypes.byref(n)),
           "tril_dbg_st_audit_sample")
    return rows[: n.value], pis[: n.value]


def tril_st_features(ctx, q_sums, q_grid, t_sums, t_grid, k0: int, n_steps: int, params=None,
                     cap: int = 1 << 20):
    """Feature rows of the candidate bin pairs: (x [n, 6] float32, y0 [n] float64,
    key [n] int64), device tensors; grows the buffers once if cap is too small."""
    import torch
    gq, gt = st_grid(q_grid), st_grid(t_grid)
    p = params or sur_params()
    for _ in range(2):
        x = torch.empty((max(cap, 1), 6), dtype=torch.float32, device="cuda")
        y0 = torch.empty(max(cap, 1), dtype=torch.float64, device="cuda")
        key = torch.empty(max(cap, 1), dtype=torch.int64, device="cuda")
        n = ctypes.c_int64(0)
        code = lib().tril_st_features(_h(ctx), q_sums.data_ptr(), ctypes.byref(gq), t_sums.data_ptr(),
                                      ctypes.byref(gt), int(k0), int(n_steps), ctypes.byref(p),
                                      x.data_ptr(), y0.data_ptr(), key.data_ptr(), cap, ctypes.byref(n))
        if code == TRIL_E_OVERFLOW and n.value > cap:
            cap = n.value
            continue
        _check(code, f"tril_st_features (rows {n.value}, capacity {cap})")
        m = n.value
        return x[:m], y0[:m], key[:m]
    raise TrilError(TRIL_E_OVERFLOW, "tril_st_features")


def tril_st_targets(key, y0, exact: "StTable", eps: float = 1e-3, stream=None):
    import torch
    n = key.shape[0]
    target = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
    y_exact = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
    _check(lib().tril_st_targets(key.data_ptr() if n else None, y0.data_ptr() if n else None, n,
                                 ctypes.byref(exact.c), float(eps), target.data_ptr(),
                                 y_exact.data_ptr(), _stream(stream)), "tril_st_targets")
    return target[:n], y_exact[:n]


def tril_st_surrogate(ctx, mlp: "Mlp", target: Beam, t_bins, t_sums, t_grid, query: Beam, q_bins,
                      q_sums, q_grid, k0: int, n_steps: int, params=None) -> dict:
    r = tril_st_sur_result()
    gq, gt = st_grid(q_grid), st_grid(t_grid)
    p = params or sur_params()
    _check(lib().tril_st_surrogate(_h(ctx), mlp.h, ctypes.byref(target.c),
                                   t_bins.data_ptr() if target.n else None, t_sums.data_ptr(),
                                   ctypes.byref(gt), ctypes.byref(query.c),
                                   q_bins.data_ptr() if query.n else None, q_sums.data_ptr(),
                                   ctypes.byref(gq), int(k0), int(n_steps), ctypes.byref(p),
                                   ctypes.byref(r)), "tril_st_surrogate")
    return {k: getattr(r, k) for k, _ in tril_st_sur_result._fields_}


def tril_dbg_gemm_bf16(A, sam, sak, B, sbk, sbn, M, N, K, C, stream=None) -> None:
    """A, B: int16 device tensors holding BF16 bit patterns; C: float32 device [M, N]."""
    _check(lib().tril_dbg_gemm_bf16(A.data_ptr(), sam, sak, B.data_ptr(), sbk, sbn, M, N, K,
                                    C.data_ptr(), _stream(stream)), "tril_dbg_gemm_bf16")


def tril_stats(ctx, pairs: Optional[Pairs], n_bins: int = 0, n_step_counts: int = 0) -> dict:
    st = tril_stats_t()
    spec = np.zeros(max(n_bins, 1), dtype=np.float64)
    sc = np.zeros(max(n_step_counts, 1), dtype=np.int64)
    st.spectrum = spec.ctypes.data_as(_dp) if n_bins > 0 else None
    st.step_counts = sc.ctypes.data_as(_i64p) if n_step_counts > 0 else None
    st.n_step_counts = int(n_step_counts)
    code = lib().tril_stats(ctx, ctypes.byref(pairs.c) if pairs is not None else None,
                            ctypes.byref(st))
    out = {k: getattr(st, k) for k, _ in tril_stats_t._fields_
           if k not in ("spectrum", "step_counts", "pad0")}
    out["yield"] = out.pop("yield_")
    out["spectrum"] = spec[:n_bins].copy()
    out["step_counts"] = sc[:n_step_counts].copy()
    out["code"] = code
    return out


def tril_reset_counters(ctx) -> None:
    _check(lib().tril_reset_counters(ctx), "tril_reset_counters")


def tril_destroy(ctx) -> None:
    if ctx:
        lib().tril_destroy(ctx)


def tril_strerror(code: int) -> str:
    return lib().tril_strerror(code).decode()


# ------------------------------------------------------------ inspection calls


def tril_dbg_sort_u32(keys, vals, key_bits: int, stream=None) -> None:
    _check(lib().tril_dbg_sort_u32(keys.data_ptr(), vals.data_ptr(), keys.numel(), key_bits,
                                   _stream(stream)), "tril_dbg_sort_u32")


def tril_dbg_sort_u64(keys, vals, key_bits: int, stream=None) -> None:
    _check(lib().tril_dbg_sort_u64(keys.data_ptr(), vals.data_ptr(), keys.numel(), key_bits,
                                   _stream(stream)), "tril_dbg_sort_u64")


def tril_dbg_morton(boxes, bounds: Sequence[float], keys, stream=None) -> None:
    b = (ctypes.c_float * 6)(*[float(v) for v in bounds])
    _check(lib().tril_dbg_morton(boxes.data_ptr(), boxes.shape[0], b, keys.data_ptr(),
                                 _stream(stream)), "tril_dbg_morton")


def tril_dbg_pair_eval(inp, out, stream=None) -> None:
    _check(lib().tril_dbg_pair_eval(inp.shape[0], inp.data_ptr(), out.data_ptr(), _stream(stream)),
           "tril_dbg_pair_eval")


def tril_dbg_pair_eval32(inp, out, stream=None) -> None:
    _check(lib().tril_dbg_pair_eval32(inp.shape[0], inp.data_ptr(), out.data_ptr(), _stream(stream)),
           "tril_dbg_pair_eval32")


def _h(ctx):
    return ctx.h if isinstance(ctx, Context) else ctx


DBG_DIV64, DBG_SQRT64, DBG_DIV32, DBG_SQRT32, DBG_LOG32, DBG_LOG1P32 = range(6)


def tril_dbg_math(which: int, a, b, out, stream=None) -> None:
    """One narrow-phase device operation per element of float64 device tensors."""
    _check(lib().tril_dbg_math(int(which), int(a.numel()), a.data_ptr(),
                               b.data_ptr() if b is not None else None, out.data_ptr(),
                               _stream(stream)), "tril_dbg_math")


def tril_dbg_tree(ctx, n_target: int, n_inst: int = 1, m: int = 1):
    """Internal nodes of the last build: lo/hi (k, 2, 3) child boxes, link (k, 2) child
    links (>= 0 internal, <= -2 leaf: element -2 - link, or sorted position with window
    copies), roots (copies x n_inst), copies (per step: m)."""
    ctx = _h(ctx)
    cap = max(m * (n_target - 1), 1)
    nodes = np.zeros((cap, 16), dtype=np.float32)
    nn = ctypes.c_int64(0)
    roots = np.zeros(max(m * n_inst, 1), dtype=np.int32)
    _check(lib().tril_dbg_tree(ctx, nodes.ctypes.data, cap, ctypes.byref(nn),
                               roots.ctypes.data_as(_i32p)), "tril_dbg_tree")
    copies = nn.value // (n_target - 1) if n_target > 1 else m
    nodes = nodes[: nn.value].reshape(-1, 2, 8)
    ints = nodes.view(np.int32)
    return {"lo": nodes[:, :, 0:3].copy(), "hi": nodes[:, :, 4:7].copy(),
            "link": ints[:, :, 3].copy(), "e": nodes[:, :, 7].copy(),
            "roots": roots[: copies * n_inst], "copies": copies}


def tril_dbg_quad_nodes(ctx, n_target: int, m: int):
    """Four-child forms of the last build's window copies: (nodes (k, 16) uint32, frames
    (copies, 8) float32), or (None, None) without them."""
    ctx = _h(ctx)
    cap = max(m * (n_target - 1), 1)
    nodes = np.zeros((cap, 16), dtype=np.uint32)
    frames = np.zeros((max(m, 1), 8), dtype=np.float32)
    nn = ctypes.c_int64(0)
    nc = ctypes.c_int32(0)
    _check(lib().tril_dbg_quad_nodes(ctx, nodes.ctypes.data, cap, ctypes.byref(nn),
                                     frames.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                     ctypes.byref(nc)), "tril_dbg_quad_nodes")
    if nc.value == 0:
        return None, None
    return nodes[: nn.value].copy(), frames[: nc.value].copy()


def tril_dbg_keep_nodes(ctx, on: bool = True) -> None:
    """Later builds of ctx store every binary node of window copies (tril_dbg_tree needs
    them; the traversal reads the four-child forms)."""
    _check(lib().tril_dbg_keep_nodes(_h(ctx), 1 if on else 0), "tril_dbg_keep_nodes")


def tril_dbg_target_records(ctx, n_target: int):
    """Window copies of the last build: (win, records) with records a dict of lo (n, 3),
    d (n, 3), w (n, 3), e (n,), row (n,) per sorted position; (1, None) for per-step copies."""
    ctx = _h(ctx)
    rec = np.zeros((max(n_target, 1), 12), dtype=np.float32)
    nn = ctypes.c_int64(0)
    win = ctypes.c_int32(0)
    _check(lib().tril_dbg_target_records(ctx, rec.ctypes.data, max(n_target, 1), ctypes.byref(nn),
                                         ctypes.byref(win)), "tril_dbg_target_records")
    if win.value <= 1:
        return win.value, None
    rec = rec[: nn.value]
    ints = rec.view(np.int32)
    return win.value, {"lo": rec[:, 0:3].copy(), "d": rec[:, 4:7].copy(), "w": rec[:, 8:11].copy(),
                       "e": rec[:, 7].copy(), "row": ints[:, 3].copy()}


def tril_dbg_boxes(ctx, which: int, n: int):
    ctx = _h(ctx)
    boxes = np.zeros((max(n, 1), 8), dtype=np.float32)
    nn = ctypes.c_int64(0)
    _check(lib().tril_dbg_boxes(ctx, int(which), boxes.ctypes.data, max(n, 1), ctypes.byref(nn)),
           "tril_dbg_boxes")
    boxes = boxes[: nn.value]
    ints = boxes.view(np.int32)
    return {"lo": boxes[:, 0:3].copy(), "hi": boxes[:, 4:7].copy(), "tag": ints[:, 3].copy(),
            "inst": ints[:, 7].copy()}


def tril_dbg_target_rows(ctx, n: int) -> np.ndarray:
    """Caller row of each row of the last build's target view."""
    ctx = _h(ctx)
    rows = np.zeros(max(n, 1), dtype=np.int32)
    nn = ctypes.c_int64(0)
    _check(lib().tril_dbg_target_rows(ctx, rows.ctypes.data_as(_i32p), max(n, 1),
                                      ctypes.byref(nn)), "tril_dbg_target_rows")
    return rows[: nn.value]


def tril_dbg_query_records(ctx, s: int, n: int):
    """Query boxes of step offset s of the last step batch, formed from the batch's
    per-row records as the traversal forms them, in the caller's row order."""
    ctx = _h(ctx)
    boxes = np.zeros((max(n, 1), 8), dtype=np.float32)
    nn = ctypes.c_int64(0)
    _check(lib().tril_dbg_query_records(ctx, int(s), boxes.ctypes.data, max(n, 1),
                                        ctypes.byref(nn)), "tril_dbg_query_records")
    boxes = boxes[: nn.value]
    ints = boxes.view(np.int32)
    return {"lo": boxes[:, 0:3].copy(), "hi": boxes[:, 4:7].copy(), "tag": ints[:, 3].copy()}


def tril_dbg_candidates(ctx, cap: int = 1 << 22):
    ctx = _h(ctx)
    ci = np.zeros(cap, dtype=np.int32)
    cj = np.zeros(cap, dtype=np.int32)
    cnt = ctypes.c_int64(0)
    _check(lib().tril_dbg_candidates(ctx, ci.ctypes.data_as(_i32p), cj.ctypes.data_as(_i32p), cap,
                                     ctypes.byref(cnt)), "tril_dbg_candidates")
    m = min(cnt.value, cap)
    return ci[:m].copy(), cj[:m].copy(), cnt.value


# ---------------------------------------------------------------- convenience


class Context:
    """One collision context (owns the hierarchy and scratch on the device)."""

    def __init__(self, dt: float, edges: Optional[np.ndarray] = None, flags: int = 0,
                 cand_cap: int = 0, block_traverse: int = 0, step_batch: int = 0, stream=None,
                 morton_bits: int = 0, kinetic_window: int = 0, descent_window: int = 0):
        self.n_bins = 0 if edges is None else max(len(edges) - 1, 0)
        self.h = tril_create(dt, edges, flags, cand_cap, block_traverse, step_batch, stream,
                             morton_bits, kinetic_window, descent_window)

    def build(self, target: Beam, step: int) -> None:
        tril_build(self.h, target, step)

    def collide(self, query: Beam, step: int, pairs: Pairs) -> None:
        tril_collide(self.h, query, step, pairs)

    def run(self, target: Beam, query: Beam, k0: int, n_steps: int, pairs: Pairs) -> None:
        tril_run(self.h, target, query, k0, n_steps, pairs)

    def stats(self, pairs: Optional[Pairs], n_step_counts: int = 0, check: bool = True) -> dict:
        out = tril_stats(self.h, pairs, self.n_bins, n_step_counts)
        if check:
            _check(out["code"], "tril_stats")
        return out

    def reset_counters(self) -> None:
        tril_reset_counters(self.h)

    def close(self) -> None:
        if self.h:
            tril_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_steps(ctx: Context, target: Beam, query: Beam, n_steps: int, pairs: Pairs,
              k0: int = 0, graph: bool = True) -> None:
    """Build + collide for steps k0 .. k0+n_steps-1 (graph replay or one call per step)."""
    if graph:
        ctx.run(target, query, k0, n_steps, pairs)
    else:
        for k in range(k0, k0 + n_steps):
            ctx.build(target, k)
            ctx.collide(query, k, pairs)
