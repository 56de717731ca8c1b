"""Launch-parameter tuning of the micro engine with a JSON cache.

The engine's own search (``lhmm_micro_autotune``: queue depth, drain level
and busy-lane rule of the pair-force kernel, binning workgroup size, fused
binning, stencil pruning, box groups, steps per captured graph; state put
back after every trial) is run once per workload shape; the result is cached
under a key made of the GPU architecture, the precision, a histogram of the
box sizes (boxes per power-of-two particle-count bucket) and a digest of the
built library, so a later engine over boxes of the same shape reuses it
without timing, and a rebuilt engine tunes afresh.  No parameter changes
results, only speed.

Cache file: ``$LHMM_TUNE_CACHE`` or ``~/.cache/lhmm/autotune.json``.
"""
from __future__ import annotations

import hashlib
import json
import math
import os

CACHE_ENV = "LHMM_TUNE_CACHE"


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "lhmm", "autotune.json")


def size_histogram(sizes) -> str:
    """'2^k:count' for every power-of-two bucket of particle counts, sorted."""
    hist = {}
    for n in sizes:
        k = int(math.floor(math.log2(max(int(n), 1))))
        hist[k] = hist.get(k, 0) + 1
    return ",".join(f"2^{k}:{hist[k]}" for k in sorted(hist))


def library_digest() -> str:
    """First 12 hex digits of the SHA-256 of the loaded library file."""
    from . import _lib

    try:
        with open(_lib.LIB_PATH, "rb") as f:
            return hashlib.sha256(f.read()).hexdigest()[:12]
    except OSError:
        return "unknown"


def cache_key(arch: str, precision: str, sizes, library: str | None = None) -> str:
    return f"{arch}|{precision}|{size_histogram(sizes)}|{library if library is not None else library_digest()}"


def load_cache(path=None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store(key: str, entry: dict, path=None) -> None:
    path = path or cache_path()
    data = load_cache(path)
    data[key] = entry
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def gpu_arch() -> str:
    import torch

    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return str(getattr(props, "gcnArchName", props.name)).split(":")[0]


def tune(engine, gradL, sizes, precision: str, trial_steps: int = 20, path=None, force: bool = False) -> dict:
    """Apply the cached configuration for this workload shape, or search and
    cache one.  Returns {"key", "config", "ms_per_step" (None if cached),
    "cached"}."""
    key = cache_key(gpu_arch(), precision, sizes)
    if not force:
        hit = load_cache(path).get(key)
        if hit and "config" in hit:
            try:
                engine.set_config(**hit["config"])
                return {"key": key, "config": engine.config(), "ms_per_step": hit.get("ms_per_step"),
                        "cached": True}
            except Exception:
                pass  # stale or invalid entry: search again
    cfg, ms = engine.autotune(gradL, trial_steps)
    store(key, {"config": cfg, "ms_per_step": ms, "trial_steps": trial_steps}, path)
    return {"key": key, "config": cfg, "ms_per_step": ms, "cached": False}
