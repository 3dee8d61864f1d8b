"""Autotuner for batched fragment plans.

Chooses the radix threshold (fragments expecting more groups are partitioned
and aggregated in LDS region by region), the hash-table load factor, the
LDS-privatisation threshold, the tile size and the persistent grid size of a
gq_batch_plan by coordinate descent over candidate plans timed on a stratified
sample of the fragments, and caches the choice in a JSON file
keyed by the device name and a coarse shape bucket of the workload (number of
fragments, total rows, median cardinality, each as a power of two).

Cache file: $GQ_AUTOTUNE_CACHE, else ~/.cache/gq/autotune.json.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import torch

from . import gq

CANDIDATES = {
    "radix_min_groups": [-1, 257, 1024, 4096],
    "lds_max_groups": [-1, 64, 256],
    "load_factor": [0.5, 0.7],
    "tile_rows": [4096, 8192, 16384],
    "blocks_per_cu": [2, 4, 8],
}
# Starting point of the search (the library's defaults, radix from 257 groups).
START = {"radix_min_groups": 257, "lds_max_groups": 256, "load_factor": 0.5, "tile_rows": 8192, "blocks_per_cu": 4}


def cache_path() -> str:
    p = os.environ.get("GQ_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "gq", "autotune.json")


def shape_key(frags) -> str:
    rows = np.array([fr[0].nrows for fr in frags], dtype=np.int64)
    card = np.array([max(1, int(fr[2] or 1)) for fr in frags], dtype=np.int64)
    dev = torch.cuda.get_device_properties(torch.cuda.current_device())
    b = lambda x: int(round(math.log2(max(1, x))))  # noqa: E731
    return f"{dev.gcnArchName}|cu{dev.multi_processor_count}|f{b(len(frags))}|r{b(rows.sum())}|c{b(np.median(card))}"


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(d):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def sample_fragments(frags, k=512, seed=0):
    """Up to k fragments, stratified by row count so that every size class appears."""
    if len(frags) <= k:
        return list(frags)
    order = np.argsort([fr[0].nrows for fr in frags], kind="stable")
    idx = order[np.linspace(0, len(order) - 1, k).astype(np.int64)]
    return [frags[i] for i in sorted(set(idx.tolist()))]


def time_plan(ctx, frags, keys, aggs, cfg, reps=3) -> float:
    plan = gq.BatchPlan(ctx, frags, keys, aggs, **cfg)
    try:
        plan.launch()
        ctx.raise_status()
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            plan.launch()
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        ctx.raise_status()
        return float(sorted(ts)[len(ts) // 2])
    finally:
        plan.free()
        # A plan over the whole workload holds tens of GB; hand them back to
        # the device so that the next candidate (or the caller's plan) can
        # allocate its own size.
        torch.cuda.synchronize()
        torch.cuda.empty_cache()


def best_batch_config(ctx, frags, keys, aggs, use_cache=True) -> dict:
    key = shape_key(frags)
    cache = _load() if use_cache else {}
    if key in cache:
        return dict(cache[key]["config"])
    sample = sample_fragments(frags)
    # Coordinate descent: each parameter in turn over its candidates, the others
    # at their best so far; two sweeps.
    best = dict(START)
    best_ms = time_plan(ctx, sample, keys, aggs, best)
    results = [(best_ms, dict(best))]
    for _ in range(2):
        changed = False
        for name, values in CANDIDATES.items():
            for v in values:
                if v == best[name]:
                    continue
                cfg = dict(best, **{name: v})
                ms = time_plan(ctx, sample, keys, aggs, cfg)
                results.append((ms, cfg))
                if ms < best_ms:
                    best, best_ms, changed = cfg, ms, True
        if not changed:
            break
    full_ms = None
    if len(sample) < len(frags) and best != START:
        # The sample's winner must also beat the starting point on the whole
        # workload (fixed per-launch costs weigh more in a small sample).
        full_ms = time_plan(ctx, frags, keys, aggs, best)
        start_ms = time_plan(ctx, frags, keys, aggs, START)
        if start_ms <= full_ms:
            best, full_ms = dict(START), start_ms
    cache[key] = {"config": best, "sample_ms": best_ms, "full_ms": full_ms, "sample_fragments": len(sample),
                  "tried": len(results)}
    if use_cache:
        _save(cache)
    return dict(best)
