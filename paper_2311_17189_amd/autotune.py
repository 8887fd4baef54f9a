"""Autotuner of the persistent mixed-diagram batch.

Tries batch tunings -- the specialized kernels where available as recorded
per-diagram launches (kernels 0), the specialized tile functions inside
persistent kernels (kernels 2), or the packed persistent kernels (kernels 1);
for the persistent ones a block size (lanes per tile, packed only), resident
waves per CU of the persistent grid, and the tile factor that sets how many
sample tiles one work item of a cheap diagram holds -- times each with HIP
events on the batch graph, and keeps the fastest.  Results are cached in a JSON file keyed by a
signature of the batch (every diagram's canonical term list, sample and
frequency counts, path), so a repeated workload is tuned once.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, List, Optional

# the specialized kernels as recorded launches (no tiling to tune), the
# specialized tile functions in persistent kernels over a few tilings, then the
# packed persistent kernels over a grid of tilings
DEFAULT_CANDIDATES: List[Dict[str, int]] = [{"block": 0, "waves_per_cu": 8, "tile_factor": 1, "kernels": 0}] + [
    {"block": 0, "waves_per_cu": w, "tile_factor": f, "kernels": 2} for w, f in ((32, 2), (32, 4), (16, 2))
] + [
    {"block": b, "waves_per_cu": w, "tile_factor": f, "kernels": 1}
    for b in (0, 64, 128) for w in (4, 8, 16) for f in (1, 4)
]


def cache_path() -> str:
    return os.environ.get("AMIGPU_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "amigpu", "batch_tuning.json"))


def signature(items) -> str:
    h = hashlib.sha256()
    for it in items:
        t = it["terms"]
        h.update(t.canonical().tobytes())
        x = it["k"] if it.get("k") is not None else it["energies"]
        h.update(f"{x.shape[0]}:{it['ext_freqs'].shape[0]}:{'k' if it.get('k') is not None else 'E'}"
                 f":{it.get('out') is not None}:{it.get('out_sum') is not None}".encode())
    return h.hexdigest()


def _load_cache(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store_cache(path, data):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def time_batch(batch, reps: int = 3, stream=None, warm_s: float = 0.05) -> float:
    """Median milliseconds of one batch graph launch, after launches for at
    least `warm_s` seconds (so timing does not start on a clock still ramping
    up) and at least one."""
    import time

    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    t_end = time.perf_counter() + warm_s
    batch.run(s)
    torch.cuda.synchronize()
    while time.perf_counter() < t_end:
        batch.run(s)
        torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s)
        batch.run(s)
        b.record(s)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def autotune(items, candidates: Optional[List[Dict[str, int]]] = None, reps: int = 3,
             use_cache: bool = True, path: Optional[str] = None):
    """Return ``(best_tuning, {str(tuning): ms})`` for a list of batch items."""
    from ._lib import AmiError, Batch
    path = path or cache_path()
    sig = signature(items)
    cache = _load_cache(path) if use_cache else {}
    if sig in cache:
        return cache[sig]["tuning"], cache[sig]["timings"]
    timings = {}
    best, best_ms = None, float("inf")
    for cand in (candidates or DEFAULT_CANDIDATES):
        try:
            b = Batch(items, cand)
        except AmiError:
            continue                      # e.g. a block too large for the LDS of this batch
        ms = time_batch(b, reps)
        b.close()
        timings[json.dumps(cand, sort_keys=True)] = ms
        if ms < best_ms:
            best, best_ms = cand, ms
    if best is None:
        raise AmiError(-7, "no candidate tuning could be built for this batch")
    if use_cache:
        cache[sig] = {"tuning": best, "timings": timings}
        _store_cache(path, cache)
    return best, timings
