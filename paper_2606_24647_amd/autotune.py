"""Autotuner for batched fragment plans.

Chooses the hash-table load factor, the LDS-privatisation threshold, the tile
size and the persistent grid size of a gq_batch_plan by timing candidate plans
on a stratified sample of the fragments, and caches the choice in a JSON file
keyed by the device name and a coarse shape bucket of the workload (number of
fragments, total rows, median cardinality, each as a power of two).

Cache file: $GQ_AUTOTUNE_CACHE, else ~/.cache/gq/autotune.json.
"""
from __future__ import annotations

import itertools
import json
import math
import os

import numpy as np
import torch

from . import gq

CANDIDATES = {
    "lds_max_groups": [-1, 64, 256],
    "load_factor": [0.5, 0.7],
    "tile_rows": [4096, 8192, 16384],
    "blocks_per_cu": [2, 4, 8],
}


def cache_path() -> str:
    p = os.environ.get("GQ_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "gq", "autotune.json")


def shape_key(frags) -> str:
    rows = np.array([t.nrows for t, _, _ in frags], dtype=np.int64)
    card = np.array([max(1, int(c or 1)) for _, _, c in frags], dtype=np.int64)
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


def sample_fragments(frags, k=256, seed=0):
    """Up to k fragments, stratified by row count so that every size class appears."""
    if len(frags) <= k:
        return list(frags)
    order = np.argsort([t.nrows for t, _, _ in frags], kind="stable")
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


def best_batch_config(ctx, frags, keys, aggs, use_cache=True) -> dict:
    key = shape_key(frags)
    cache = _load() if use_cache else {}
    if key in cache:
        return dict(cache[key]["config"])
    sample = sample_fragments(frags)
    best, best_ms = None, float("inf")
    results = []
    names = list(CANDIDATES)
    for values in itertools.product(*(CANDIDATES[n] for n in names)):
        cfg = dict(zip(names, values))
        ms = time_plan(ctx, sample, keys, aggs, cfg)
        results.append((ms, cfg))
        if ms < best_ms:
            best, best_ms = cfg, ms
    cache[key] = {"config": best, "sample_ms": best_ms, "sample_fragments": len(sample),
                  "tried": len(results)}
    if use_cache:
        _save(cache)
    return dict(best)
