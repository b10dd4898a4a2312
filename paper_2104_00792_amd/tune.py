"""Autotuner for the sorted build: picks the build's two speed knobs by timing.

The knobs never change a table, only how it is built:
  - ``log2_subbin``: sub-bins of 2^x buckets (10..13).  It sets how many keys
    one workgroup of the LDS build takes (about 2^x times the keys per
    bucket, held 20 per thread by 512 threads), and so the number of
    workgroups and their register and LDS load;
  - ``split_bits``: at most 2^x level-2 digits per level-1 segment (7..10):
    the fan-out of the second split, traded against the first.

``tune_table`` and ``tune_batched`` time build + probe (+ free) for every
candidate on the caller's own device data, a few repetitions each after a
warm-up, keep the fastest, and remember it in a JSON cache keyed by the
workload's shape (key type, log2 of the key count, partitions, ratio, number
of tables) and the device name.  The cache lives at ``$HG_TUNE_CACHE`` or
``~/.cache/hg_tune.json``.
"""

from __future__ import annotations

import json
import math
import os
import time

from . import (HG_KEY_U32, hg_build, hg_build_batched, hg_count, hg_count_batched)

SUBBIN_CANDIDATES = (11, 12, 13)
SPLIT_CANDIDATES = (7, 8, 9)


def cache_path() -> str:
    return os.environ.get("HG_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "hg_tune.json"))


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, entry: dict) -> None:
    data = _load()
    data[key] = entry
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only loses the cache


def _device_name() -> str:
    import torch

    return torch.cuda.get_device_name(torch.cuda.current_device())


def _signature(kind: str, n: int, key_type: int, P: int, ratio, tables: int) -> str:
    lg = int(math.log2(n)) if n > 0 else 0
    kt = "u32" if key_type == HG_KEY_U32 else "u64"
    return f"{kind}|{kt}|2^{lg}|P{P}|r{ratio[0]}/{ratio[1]}|T{tables}|{_device_name()}"


def _time(step, reps: int) -> float:
    import torch

    step()  # warm-up (and the pool's first allocations)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def tune_table(keys, queries, P: int = 1, ratio=(1, 1), reps: int = 3, use_cache: bool = True) -> dict:
    """Best (log2_subbin, split_bits) for hg_build + hg_count on these keys
    and queries.  Returns {"log2_subbin", "split_bits", "ms", "default_ms",
    "trials": [...], "cached": bool}."""
    import torch

    sig = _signature("table", keys.numel(), 0 if keys.element_size() == 4 else 1, P, ratio, 1)
    if use_cache:
        hit = _load().get(sig)
        if hit is not None:
            return dict(hit, cached=True)
    counts = torch.empty(queries.numel(), dtype=torch.uint32, device=queries.device)

    def run(sub, bits):
        def step():
            t = hg_build(keys, P=P, ratio=ratio, log2_subbin=sub, split_bits=bits)
            hg_count(t, queries, out=counts)
            t.free()
        return _time(step, reps) * 1000.0

    trials = [{"log2_subbin": 0, "split_bits": 0, "ms": run(0, 0)}]
    for sub in SUBBIN_CANDIDATES:
        for bits in SPLIT_CANDIDATES:
            trials.append({"log2_subbin": sub, "split_bits": bits, "ms": run(sub, bits)})
    best = min(trials, key=lambda r: r["ms"])
    entry = {"log2_subbin": best["log2_subbin"], "split_bits": best["split_bits"], "ms": best["ms"],
             "default_ms": trials[0]["ms"], "trials": trials}
    if use_cache:
        _store(sig, entry)
    return dict(entry, cached=False)


def tune_batched(keys, table_offsets, queries, query_offsets, ratio=(1, 1), reps: int = 3,
                 use_cache: bool = True) -> dict:
    """Best log2_subbin for hg_build_batched + hg_count_batched on this batch
    (the batched build has no level-1 split, so split_bits does not apply)."""
    import torch

    T = table_offsets.numel() - 1
    sig = _signature("batched", keys.numel(), 0 if keys.element_size() == 4 else 1, 1, ratio, T)
    if use_cache:
        hit = _load().get(sig)
        if hit is not None:
            return dict(hit, cached=True)
    counts = torch.empty(queries.numel(), dtype=torch.uint32, device=queries.device)

    def run(sub):
        def step():
            t = hg_build_batched(keys, table_offsets, ratio=ratio, log2_subbin=sub)
            hg_count_batched(t, queries, query_offsets, out=counts)
            t.free()
        return _time(step, reps) * 1000.0

    trials = [{"log2_subbin": 0, "ms": run(0)}]
    for sub in SUBBIN_CANDIDATES:
        trials.append({"log2_subbin": sub, "ms": run(sub)})
    best = min(trials, key=lambda r: r["ms"])
    entry = {"log2_subbin": best["log2_subbin"], "ms": best["ms"], "default_ms": trials[0]["ms"], "trials": trials}
    if use_cache:
        _store(sig, entry)
    return dict(entry, cached=False)
