"""Autotuner for batched passes: picks the launch shape (waves per CU of the
statistics launch, workgroups per CU of the gradient launch, planes per
gradient tile, and the gradient workgroup's shape: 512 x 16 columns x rows on
512 threads, 256 x 16 on 256 threads, or the general tile) by timing plan
launches of the actual batch.  Given several copies of the batch's streams
(together larger than the last-level caches), it launches them in turn, so
that no candidate is timed on cache-resident bytes.

Every candidate must reproduce the reference results bit for bit (they are
exact integer sums and identical per-element arithmetic whatever the launch
shape); a candidate that does not is rejected, not just skipped.  The best
choice is cached in a JSON file keyed by the device architecture and the
batch's shape class (per job: dtype, block size, operation, stage, field
shape and box volume bucket).
"""
from __future__ import annotations

import json
import os
import statistics

import torch

from . import hsz

# the narrow tiles (grad_tile_x 0 / 256) run at most two workgroups per
# compute unit whatever grad_groups_per_cu asks, so that axis is swept for the
# general tile only
CANDIDATES = [
    {"stats_waves_per_cu": w, "grad_groups_per_cu": g, "grad_tz": tz, "grad_tile_x": tx}
    for w in (4, 8, 16) for tx in (0, 256, -1) for g in ((2, 4, 6) if tx == -1 else (2,)) for tz in (16, 32, 64)
]

DEFAULT_CACHE = os.environ.get("HSZ_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "hsz_tune.json"))


def shape_class(jobs) -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName if torch.cuda.is_available() else "cpu"
    parts = []
    for j in jobs:
        h = j.c.header
        vol = 1
        if j.box is not None:
            for lo, hi in zip(*j.box):
                vol *= int(hi) - int(lo)
        else:
            vol = int(h.n)
        bucket = max(0, vol.bit_length() - 1)  # powers of two
        parts.append(f"{h.dtype}.{h.block}.{j.op}.{j.via}.{'x'.join(map(str, h.shape))}.{bucket}")
    return arch + "|" + ";".join(sorted(parts))


def _same(a, b) -> bool:
    if isinstance(a, dict):
        keys = ("n", "s1", "s2", "mean")
        return all(a[k] == b[k] for k in keys) and (a["var"] == b["var"] or (a["var"] != a["var"] and b["var"] != b["var"]))
    return torch.equal(a, b)


def time_plan(plan, reps: int) -> float:
    """Median HIP-event time of one launch; 'plan' is a Plan or a list of
    Plans on one stream (the same batch over distinct copies), launched in
    turn."""
    plans = plan if isinstance(plan, (list, tuple)) else [plan]
    stream = plans[0].stream
    for p in plans:
        p.launch()  # warm
    stream.synchronize()
    times = []
    for r in range(reps * len(plans)):
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        plans[r % len(plans)].launch()
        stop.record(stream)
        stop.synchronize()
        times.append(start.elapsed_time(stop))
    return statistics.median(times)


def tune(jobs, candidates=None, reps: int = 5, cache_path: str | None = DEFAULT_CACHE, log=None, alternates=()):
    """Return (best tuning dict, {candidate index: ms}); updates the cache.

    alternates: further job lists of the same batch over other copies of its
    streams; each candidate's plans over all the copies are launched in turn."""
    candidates = CANDIDATES if candidates is None else candidates
    ref = hsz.batch_run(jobs)
    timings = {}
    best, best_ms = None, float("inf")
    stream = torch.cuda.Stream()
    for k, cand in enumerate(candidates):
        plans = []
        try:
            for js in [jobs, *alternates]:
                plans.append(hsz.Plan(js, tune=cand, stream=stream))
            ms = time_plan(plans, reps)
            got = plans[0].results()
        finally:
            for p in plans:
                p.close()
        if not all(_same(a, b) for a, b in zip(ref, got)):
            raise RuntimeError(f"launch shape {cand} changed a result")
        timings[k] = ms
        if log:
            log(f"[tune] {cand} -> {ms:.3f} ms")
        if ms < best_ms:
            best, best_ms = cand, ms
    if cache_path:
        save(shape_class(jobs), best, cache_path)
    return best, timings


def load_cache(cache_path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(cache_path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save(key: str, choice: dict, cache_path: str = DEFAULT_CACHE):
    data = load_cache(cache_path)
    data[key] = choice
    os.makedirs(os.path.dirname(cache_path) or ".", exist_ok=True)
    tmp = cache_path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, cache_path)


def cached(jobs, cache_path: str = DEFAULT_CACHE):
    """The cached choice for this shape class, or None."""
    return load_cache(cache_path).get(shape_class(jobs))
