"""Autotuner for the plot's implementation parameters (vx_tuning).

For a given k it searches the tunables that shape the plot's kernels -- the
hash's nonce slices (each slice's second partition pass runs beside the next
slice's hash), the first partition digit's width, the sort-group bits (how
finely the partition passes cut the bucket space), the sort group's LDS
capacity and the match chunk -- one at a time from the built-in default
(coordinate descent: each tunable's alternatives are timed with the others
at their best so far) and keeps the fastest.  No candidate changes any
output (they only move work between kernels), so picking by time is safe.
Results are cached in JSON keyed by GPU architecture and k
(tuning_cache.json next to this file, or the path in VX_TUNING_CACHE).
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
          "fused_sort_match", "pipeline_slices", "separate_hash", "region_pct", "hash_slices", "tail_slices",
          "batch_shared_hash")


def arch() -> str:
    if not torch.cuda.is_available():
        return "cpu"
    props = torch.cuda.get_device_properties(0)
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def axes(k: int) -> List[tuple]:
    """The tunables searched for k, each with its alternatives (0 = the
    built-in default for k)."""
    gb = [g for g in (k - 12, k - 11, k - 10) if 1 <= g <= 21]
    return [
        ("hash_slices", [0, 1, 4, 16]),            # hash work per launch (slices)
        ("group_bits", [0] + gb),                  # sort groups = bucket-partition granularity
        ("pass1_bits", [0, 4, 5, 6, 7, 8]),        # first partition digit
        ("group_cap", [0, 3072]),                  # sort group capacity in LDS
        ("match_chunk_bits", [0, 10]),             # match chunk (records)
    ]


def candidates(k: int) -> List[Dict[str, int]]:
    """Every single-axis variant of the default (the first round of the
    search); used by tests and as a quick list."""
    out = [{}]
    for name, vals in axes(k):
        out += [{name: v} for v in vals if v]
    return out


def to_native(d: Optional[Dict[str, int]]) -> Optional[N.VxTuning]:
    if not d:
        return None
    return N.make_tuning(**{f: int(d.get(f, 0)) for f in FIELDS})


def valid(k: int, d: Dict[str, int]) -> bool:
    p = N.make_params(bytes(32), k)
    return N.vx_workspace_bytes(p, N.VX_CALL_PLOT, to_native(d) or N.make_tuning()) > 0


def _time_plot(k: int, tuning, reps: int, key: bytes) -> float:
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
    """Coordinate descent over axes(k) from the default."""
    seen: Dict[str, float] = {}

    def timed(d):
        tag = json.dumps(d, sort_keys=True)
        if tag not in seen:
            seen[tag] = _time_plot(k, to_native(d), reps, key)
            if verbose:
                print(f"k={k} {d} {seen[tag] * 1e3:.3f} ms", flush=True)
        return seen[tag]

    best: Dict[str, int] = {}
    best_t = timed(best)
    default_t = best_t
    for name, vals in axes(k):
        for v in vals:
            cand = {**best, name: v} if v else {q: w for q, w in best.items() if q != name}
            if cand == best or not valid(k, cand):
                continue
            t = timed(cand)
            if t < best_t:
                best, best_t = cand, t
    return {"tuning": best or None, "ms": best_t * 1e3, "default_ms": default_t * 1e3, "tried": len(seen)}


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
    if rec and rec.get("tuning") and rec.get("ms", 0) < rec.get("default_ms", 0):
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
