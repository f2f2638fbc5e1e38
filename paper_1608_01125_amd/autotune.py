"""Launch-configuration cache around the library's autotuner (tril_autotune).

The tuned values (steps per launch, traversal workgroup size, Morton bits) change only
the speed of tril_run, never its results. They are stored per workload shape and
device in a JSON file so that a later process reuses them without probing again."""
from __future__ import annotations

import hashlib
import json
import os
from typing import Optional

from . import tril as T

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_1608_01125_amd",
                             "tune.json")


def library_digest() -> str:
    """Digest of the built library: a rebuilt kernel invalidates every cached setting."""
    h = hashlib.sha256()
    with open(T.LIB_PATH, "rb") as f:
        for chunk in iter(lambda: f.read(1 << 20), b""):
            h.update(chunk)
    return h.hexdigest()[:16]


def shape_key(target: T.Beam, query: T.Beam, dt: float, device_name: str, k0: int = 0,
              n_probe: int = 0) -> str:
    """Key of a workload shape and probe: beam sizes, instance count, step length, device,
    the probed steps and the library build."""
    return (f"{device_name}|nt={target.n}|nq={query.n}|inst={target.n_inst}|dt={dt:.6g}"
            f"|k0={k0}|probe={n_probe}|lib={library_digest()}")


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def tuned(ctx: T.Context, target: T.Beam, query: T.Beam, dt: float, k0: int, n_probe: int,
          cache: Optional[str] = DEFAULT_CACHE, device_name: Optional[str] = None) -> dict:
    """Apply the cached configuration for this shape, or probe with tril_autotune over
    steps k0 .. k0+n_probe-1 and store the result. Returns the configuration and
    whether it came from the cache."""
    if device_name is None:
        import torch
        device_name = torch.cuda.get_device_name(0)
    key = shape_key(target, query, dt, device_name, k0, n_probe)
    data = _load(cache) if cache else {}
    if key in data:
        cfg = data[key]
        T.tril_set_tune(ctx.h, cfg)
        return dict(cfg, cached=True)
    cfg = T.tril_autotune(ctx.h, target, query, k0, n_probe)
    if cache:
        data = _load(cache)
        data[key] = cfg
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        tmp = cache + f".{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return dict(cfg, cached=False)
