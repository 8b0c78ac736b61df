"""Autotuner for the plot's implementation parameters (vx_tuning).

For a given k it times a small set of candidate tunings -- sort-group size,
match-chunk size, hash fused with the first pass or not -- on the current
GPU and keeps the fastest.
No candidate changes any output (they only move work between kernels), so
picking by time is safe.  Results are cached in JSON keyed by GPU
architecture and k (tuning_cache.json next to this file, or the path in
VX_TUNING_CACHE).
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, List, Optional

import torch

from . import _native as N
from .plotter import alloc_plot

CACHE_PATH = os.environ.get("VX_TUNING_CACHE",
                            os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                         "tuning_cache.json"))
FIELDS = ("group_bits", "pass1_bits", "group_cap", "h1_tiles", "match_chunk_bits", "pass2_bits",
          "fused_sort_match", "pipeline_slices", "separate_hash", "region_pct")


def arch() -> str:
    if not torch.cuda.is_available():
        return "cpu"
    props = torch.cuda.get_device_properties(0)
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def candidates(k: int) -> List[Dict[str, int]]:
    out = []
    for gb in (k - 12, k - 11, k - 10):
        if not 1 <= gb <= 20:
            continue
        for cb in (10, 11):
            # the hash with the first partition pass fused in (default), or
            # the two as separate kernels
            for sep in (0, 1):
                out.append({"group_bits": gb, "match_chunk_bits": cb, "separate_hash": sep})
    return out


def to_native(d: Optional[Dict[str, int]]) -> Optional[N.VxTuning]:
    if not d:
        return None
    return N.make_tuning(**{f: int(d.get(f, 0)) for f in FIELDS})


def _time_plot(k: int, tuning: N.VxTuning, reps: int, key: bytes) -> float:
    b = alloc_plot(k, tuning=tuning)
    p = N.make_params(key, k)
    nb = b.native()
    sh = torch.cuda.current_stream().cuda_stream
    N.vx_plot(p, nb, tuning, sh)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        N.vx_plot(p, nb, tuning, sh)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del b
    return dt


def tune(k: int, reps: int = 3, key: bytes = bytes(range(32)), verbose: bool = False) -> Dict:
    best, best_t, results = None, float("inf"), []
    for cand in candidates(k):
        t = _time_plot(k, to_native(cand), reps, key)
        results.append((cand, t))
        if verbose:
            print(f"k={k} {cand} {t * 1e3:.3f} ms", flush=True)
        if t < best_t:
            best, best_t = cand, t
    default_t = _time_plot(k, None, reps, key)
    return {"tuning": best, "ms": best_t * 1e3, "default_ms": default_t * 1e3,
            "tried": len(results)}


def load_cache(path: str = CACHE_PATH) -> Dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save_cache(cache: Dict, path: str = CACHE_PATH) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned(k: int, cache: Optional[Dict] = None) -> Optional[Dict[str, int]]:
    """Cached tuning for k on this GPU (None = built-in defaults)."""
    cache = load_cache() if cache is None else cache
    rec = cache.get(arch(), {}).get(str(k))
    if rec and rec.get("ms", 0) < rec.get("default_ms", 0):
        return rec["tuning"]
    return None


def tune_all(ks, reps: int = 3, verbose: bool = False, path: str = CACHE_PATH) -> Dict:
    cache = load_cache(path)
    a = arch()
    for k in ks:
        cache.setdefault(a, {})[str(k)] = tune(k, reps, verbose=verbose)
    save_cache(cache, path)
    return cache


if __name__ == "__main__":
    import sys
    ks = [int(x) for x in sys.argv[1:]] or list(range(22, 30))
    print(json.dumps(tune_all(ks, verbose=True), indent=1))
