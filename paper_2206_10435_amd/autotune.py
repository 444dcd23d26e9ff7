"""Autotuner for the library's tile and bucket sizes.

Three groups of parameters are measured on the caller's own inputs:

* radix sort of the factor build -- keys per thread of a sort tile
  (``sort_items``: tile = 256 x sort_items keys) and digit width
  (``radix_bits``: 2^bits buckets per pass);
* expansion kernel -- tuples staged per lane per LDS round (``desum_stage``)
  and rounds per lane (``desum_rounds``);
* batch -- the sort parameters above for a whole many-query plan, timed as
  replays of its recorded graph.

Timings are HIP events on the context's stream (median of a few repeats).
Results are cached as JSON (``$GJ_TUNE_CACHE`` or ``~/.cache/gj_tune.json``)
under a signature of the device and the workload's shape, so a later run with
the same shape reuses them without measuring.
"""
from __future__ import annotations

import itertools
import json
import math
import os
import statistics
from typing import Dict, List, Optional, Sequence

SORT_ITEMS = (8, 16)
RADIX_BITS = (6, 7, 8)
DESUM_STAGE = (2, 4, 8)
DESUM_ROUNDS = (0, 4, 6, 8, 16, 32)  # 0: about 640 bytes per lane

DEFAULT = dict(sort_items=8, radix_bits=8, desum_rounds=0, desum_stage=4)


def _cache_path() -> str:
    return os.environ.get("GJ_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "gj_tune.json"))


def _load_cache() -> Dict[str, dict]:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, value: dict) -> None:
    cache = _load_cache()
    cache[key] = value
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home: tuning still applies to this process


def _device_name() -> str:
    import torch

    return torch.cuda.get_device_name(0).replace(" ", "_")


def _bucket(x: float) -> int:
    return int(round(math.log2(max(x, 1))))


def signature(kind: str, rows: Sequence[int], extra: str = "") -> str:
    return f"{_device_name()}|{kind}|n{len(rows)}|r{_bucket(sum(rows))}|{extra}"


def _time(ctx, fn, reps: int = 3) -> float:
    import torch

    st = ctx.stream
    fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(st)
        fn()
        b.record(st)
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b))
    return statistics.median(out)


def tune_factors(ctx, tables, parent, sep_col, parent_col, use_cache: bool = True) -> dict:
    """Best (sort_items, radix_bits) for building and summarizing one query."""
    rows = [int(c[0].numel()) for c in tables]
    key = signature("factors", rows)
    cache = _load_cache()
    if use_cache and key in cache:
        return cache[key]
    best, trials = None, []
    cur = dict(DEFAULT)
    for si, rb in itertools.product(SORT_ITEMS, RADIX_BITS):
        ctx.set_tune(si, rb, cur["desum_rounds"], cur["desum_stage"])

        def run():
            f = ctx.build_factors(tables, parent, sep_col, parent_col)
            ctx.summarize(f)

        ms = _time(ctx, run)
        trials.append(dict(sort_items=si, radix_bits=rb, ms=ms))
        if best is None or ms < best["ms"]:
            best = trials[-1]
    ctx.set_tune(**DEFAULT)
    res = dict(sort_items=best["sort_items"], radix_bits=best["radix_bits"], ms=best["ms"], trials=trials)
    _store(key, res)
    return res


def tune_desummarize(ctx, summary, out, first_row: int, n_rows: int, sort_items: int = 8, radix_bits: int = 8,
                     use_cache: bool = True) -> dict:
    """Best (desum_stage, desum_rounds) for expanding `n_rows` tuples into `out`."""
    key = signature("desum", [n_rows], f"t{summary.n_tables}|w{out.element_size()}")
    cache = _load_cache()
    if use_cache and key in cache:
        return cache[key]
    best, trials = None, []
    for stage, rounds in itertools.product(DESUM_STAGE, DESUM_ROUNDS):
        ctx.set_tune(sort_items, radix_bits, rounds, stage)
        ms = _time(ctx, lambda: ctx.desummarize(summary, first_row, n_rows, out))
        trials.append(dict(desum_stage=stage, desum_rounds=rounds, ms=ms))
        if best is None or ms < best["ms"]:
            best = trials[-1]
    ctx.set_tune(**DEFAULT)
    res = dict(desum_stage=best["desum_stage"], desum_rounds=best["desum_rounds"], ms=best["ms"], trials=trials)
    _store(key, res)
    return res


def tune_batch(ctx, queries: List[dict], use_cache: bool = True, reps: int = 3) -> dict:
    """Best (sort_items, radix_bits) for a many-query graph; returns the tune
    and the Batch built with it (ready to launch)."""
    from . import gj

    rows = [int(c[0].numel()) for q in queries for c in q["tables"]]
    key = signature("batch", rows, f"q{len(queries)}")
    cache = _load_cache()
    if use_cache and key in cache:
        rec = cache[key]
        t = gj.Tune(rec["sort_items"], rec["radix_bits"], DEFAULT["desum_rounds"], DEFAULT["desum_stage"])
        return dict(rec, batch=ctx.batch_create(queries, tune=t))
    best, trials, best_batch = None, [], None
    for si, rb in itertools.product(SORT_ITEMS, RADIX_BITS):
        b = ctx.batch_create(queries, tune=gj.Tune(si, rb, DEFAULT["desum_rounds"], DEFAULT["desum_stage"]))
        ms = _time(ctx, lambda: b.launch(graph=True), reps=reps)
        trials.append(dict(sort_items=si, radix_bits=rb, ms=ms))
        if best is None or ms < best["ms"]:
            best, best_batch = trials[-1], b
        else:
            del b
    res = dict(sort_items=best["sort_items"], radix_bits=best["radix_bits"], ms=best["ms"], trials=trials)
    _store(key, res)
    return dict(res, batch=best_batch)


def apply(ctx, factors_tune: Optional[dict] = None, desum_tune: Optional[dict] = None) -> dict:
    """Set the context's tune from tuner results; returns the applied values."""
    t = dict(DEFAULT)
    if factors_tune:
        t.update(sort_items=factors_tune["sort_items"], radix_bits=factors_tune["radix_bits"])
    if desum_tune:
        t.update(desum_stage=desum_tune["desum_stage"], desum_rounds=desum_tune["desum_rounds"])
    ctx.set_tune(**t)
    return t
