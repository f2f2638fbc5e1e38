"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
function the headers declare, and rejects bad parameters before any device call."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1608_01125_amd import tril as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in ("tril.h", "tril_debug.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(tril_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    L = T.lib()
    declared = _declared()
    assert {"tril_create", "tril_build", "tril_collide", "tril_stats", "tril_run",
            "tril_destroy", "tril_strerror"} <= declared
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(T.EXPORTS)


def test_binding_declares_every_argument_list():
    """ctypes passes an undeclared pointer argument as a C int, which truncates a 64-bit
    address: every entry point the binding exports has its argument types declared."""
    L = T.lib()
    missing = [n for n in T.EXPORTS if getattr(L, n).argtypes is None]
    assert not missing, missing


def test_strerror_texts():
    for code in range(0, -9, -1):
        assert T.tril_strerror(code) not in ("", "unknown error")
    assert T.tril_strerror(-99) == "unknown error"


def _create(**kw):
    p = T.tril_params()
    p.dt = kw.get("dt", 0.1)
    p.flags = kw.get("flags", 0)
    edges = kw.get("edges")
    keep = None
    if edges is not None:
        keep = np.ascontiguousarray(edges, dtype=np.float64)
        p.n_bins = kw.get("n_bins", len(keep) - 1)
        p.bin_edges = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    else:
        p.n_bins = kw.get("n_bins", 0)
        p.bin_edges = None
    p.cand_cap = kw.get("cand_cap", 0)
    p.block_traverse = kw.get("block", 0)
    p.step_batch = kw.get("step_batch", 0)
    p.morton_bits = kw.get("morton_bits", 0)
    h = ctypes.c_void_p()
    return T.lib().tril_create(ctypes.byref(h), ctypes.byref(p), None)


@pytest.mark.parametrize("kw", [
    {"dt": 0.0}, {"dt": -1.0}, {"dt": float("nan")}, {"dt": float("inf")},
    {"n_bins": -1}, {"n_bins": 3},                      # edges missing
    {"edges": [0.0, 1.0, 1.0]}, {"edges": [0.0, 2.0, 1.0]}, {"edges": [0.0, float("nan")]},
    {"cand_cap": -5}, {"block": 100}, {"block": 1024}, {"step_batch": -1},
    {"morton_bits": 2}, {"morton_bits": -3}, {"morton_bits": 31},
])
def test_create_rejects_bad_params(kw):
    assert _create(**kw) == T.TRIL_E_INVAL


def test_create_rejects_unknown_flags():
    assert _create(flags=0x80) == T.TRIL_E_NOTIMPL


def test_null_arguments():
    L = T.lib()
    assert L.tril_create(None, None, None) == T.TRIL_E_INVAL
    assert L.tril_build(None, None, 0) == T.TRIL_E_INVAL
    assert L.tril_collide(None, None, 0, None) == T.TRIL_E_INVAL
    assert L.tril_run(None, None, None, 0, 1, None) == T.TRIL_E_INVAL
    assert L.tril_stats(None, None, None) == T.TRIL_E_INVAL
    assert L.tril_reset_counters(None) == T.TRIL_E_INVAL
    assert L.tril_set_tune(None, None) == T.TRIL_E_INVAL
    assert L.tril_autotune(None, None, None, 0, 1, None) == T.TRIL_E_INVAL
    L.tril_destroy(None)
    assert L.tril_dbg_sort_u32(None, None, -1, 30, None) == T.TRIL_E_INVAL
    assert L.tril_dbg_sort_u32(None, None, 10, 0, None) == T.TRIL_E_INVAL
    assert L.tril_dbg_sort_u64(None, None, 10, 65, None) == T.TRIL_E_INVAL
    assert L.tril_dbg_pair_eval(-1, None, None, None) == T.TRIL_E_INVAL
    assert L.tril_dbg_tree(None, None, 0, None, None) == T.TRIL_E_INVAL
    assert L.tril_dbg_keep_nodes(None, 1) == T.TRIL_E_INVAL


def test_pair_kinematics_rejects_null_arguments():
    L = T.lib()
    assert L.tril_pair_kinematics(None, None, None, None, 0, None, None, None) == T.TRIL_E_INVAL


def test_new_entry_points_reject_null_arguments():
    L = T.lib()
    c3 = (ctypes.c_double * 3)(0.5, 0.5, 0.5)
    tot = ctypes.c_double(0.0)
    assert L.tril_st_exact_depleted(None, None, None, 1, None, None, c3, 0, 1, None, None,
                                    ctypes.byref(tot)) == T.TRIL_E_INVAL
    n = ctypes.c_int64(0)
    assert L.tril_ip_swarm(None, None, None, 1, None, None, c3, 0, 1, None, None,
                           ctypes.byref(n)) == T.TRIL_E_INVAL
