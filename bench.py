#!/usr/bin/env python3
"""Benchmark: HashGraph build + probe on one MI355X.

One step = hg_build of n keys (P hash-range partitions, local tables with
V_p = n_p) + hg_count of q = n queries + freeing the table, on device-resident
synthetic inputs.  Prints ONE JSON line on stdout; progress goes to stderr.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

value = n * K / (timed seconds): build+probe keys/s.  The per-kernel launch
durations come from HIP events that the library records around each of its
launches on the launch stream, over the timed steps.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "build+probe keys/s and % HBM peak at 2^28 u32; serving p50/p99 latency"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# Serving: request streams beside the client's payload stream; with four
# streams in all, each has a hardware queue of its own (four per process).
SERVING_SLOTS = 3
KERNEL_SOURCES = os.path.join(ROOT, "paper_2104_00792_amd", "csrc")

DESCRIPTIONS = {
    "p16_u32_2^28": "n=2^28 uint32 keys uniform; P=16 hash-range partitions (top 4 bits of fmix32); "
                    "local tables V_p=n_p; 2^28 queries at 50% hit",
    "plain_u32_2^28": "n=2^28 uint32 keys uniform; plain table V=n; 2^28 queries at 50% hit",
    "plain_u32_2^20": "n=2^20 uint32 keys uniform; plain table V=n; 2^20 queries at 50% hit",
    "zipf_u64_2^27": "n=2^27 uint64 keys Zipf(1.0) over 2^20 values (value of rank r = the SplitMix64 output "
                     "mixer of r, a bijection like fmix64); hash fmix64; V=n/2; 2^27 Zipf queries",
    "zipf_u32_2^28": "n=2^28 uint32 keys Zipf(1.0) over 2^20 ranks (value of rank r = the high half of the "
                     "SplitMix64 output mixer of r); hash fmix32; V=n/2; 2^28 Zipf queries",
    "batched_u32_4096": "4096 uint32 tables, sizes log-uniform in [2^10, 2^20] (622M keys), per-table seeds, "
                        "V_t = n_t; each probed by n_t queries at 50% hit; one hg_build_batched + "
                        "hg_count_batched per step",
    "copy_ceiling": "device-to-device streaming ceilings of the GPU with torch's own kernels: copy, fill and a "
                    "read-only sum over 1 GiB buffers (HIP events around each launch)",
    "dup_sweep_u32_2^28": "the duplicate study of Sec. 5.4 on the headline's keys: n=2^28 uint32 keys uniform, P=16, "
                          "hash range shrunk to V_p = n_p / occ for occ (average keys per bucket) = 1, 4, 16, 64, "
                          "256, 1024, 4096; 2^28 queries at 50% hit; build and probe timed apart",
    "serving": "Poisson stream of requests, 30% builds (uint32, sizes log-uniform in [2^10, 2^24]) and 70% probes "
               "(sizes log-uniform in [2^8, 2^22], 50% hits) against earlier tables; 200 GB HBM cap with LRU "
               "eviction; 3 concurrent request streams plus one client stream; open loop at 0.8 of the "
               "closed-loop capacity",
}


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of every kernel and launcher source: counter figures taken on
    other sources are not reported."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(KERNEL_SOURCES)):
        if name.endswith((".hip", ".h", ".cpp")):
            h.update(name.encode())
            with open(os.path.join(KERNEL_SOURCES, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def survey_bytes(kernel: str, n: int, q: int, B: int, ks: int, P: int) -> float:
    """Algorithmic bytes per launch of a kernel under the scope table's model
    of the path (HBM bytes per key and per query of each step of the method,
    with the O(V_p) working sets of a partition group in the Infinity Cache),
    charged to the kernel that carries that step out.  Kernels that carry
    out no step of the model (the second split level and its gather, the
    coarse-range count) are charged 0: their bytes are this design's
    overhead.  Per 32-bit key: partition count 4, partition scatter 8, local
    histogram 4, offsets 4 per bucket, local scatter 8 (28 per key with
    V = n); per query: count + stable scatter 12, probe in partition order 8
    (query in, count out; table reads from the cache), un-partition 12."""
    cnt = 4  # counts are u32 in the model
    part = P > 1
    table = {
        # sorted build: a2 and a4 exist only with partitions
        "part_count": ks * n if part else 0,              # a2: read keys
        "split1_count": 0 if part else ks * n,            # plain table: a5 reads the keys; else overhead
        "split1_scatter": 2 * ks * n if part else 0,      # a4: keys in, buffer out
        "split2_count": ks * n if part else 0,            # a5: read the buffer
        "split2_scatter": 0,
        "lds_build": 2 * ks * n + 4 * B,                  # a7 read + write keys, a6 offsets
        # sorted probe
        "qsplit1_count": ks * q,                          # a9 count
        "qsplit1_scatter": 2 * ks * q,                    # a9 stable scatter
        "qsplit2_count": 0,
        "qsplit2_scatter": 0,
        "lds_probe": ks * q + cnt * q,                    # probe in partition order
        "qgather2": 0,
        "qgather1": (ks + 2 * cnt) * q,                   # un-partition
        # batched tables: each table is a plain table
        "bsplit_count": ks * n,
        "blds_build": 2 * ks * n + 4 * B,
        "bqsplit_count": ks * q,
        "bqsplit_scatter": 2 * ks * q,
        "blds_probe": ks * q + cnt * q,
        "bqgather": (ks + 2 * cnt) * q,
        # atomic build and direct probe (small tables): the streaming part
        "bucket_hist": ks * n,
        "bucket_scan": 4 * B,
        "bucket_scatter": 2 * ks * n,
        "probe_count": ks * q + cnt * q,
        "probe_found": ks * q + q,
    }
    return float(table.get(kernel, 0))


def survey_step_bytes(n: int, q: int, B: int, ks: int, P: int) -> float:
    """The model's bytes for one build + probe step (sum over its steps):
    60 per key and query pair for 32-bit keys, P > 1 and V = n."""
    build = (3 * ks * n if P > 1 else 0) + ks * n + 4 * B + 2 * ks * n
    probe = (5 * ks + 3 * 4) * q
    return float(build + probe)


def algorithmic_bytes(kernel: str, n: int, q: int, B: int, ks: int, P: int, cb: int = 4) -> float:
    """Bytes the kernel's own function must move per launch in this design,
    independent of how the kernel moves them (n keys of ks bytes, q
    queries, B buckets; cb = bytes per count passed between the probe's
    kernels, 1 for a table without long buckets, else 4).  Split passes run
    once on the keys (build) and once on the queries (probe)."""
    table = {
        # build, sorted path
        "part_count": ks * n,                       # read keys
        "split1_count": ks * n,                     # read keys
        "split1_scatter": 2 * ks * n,               # keys in, keys out
        "split2_count": ks * n,                     # read keys
        "split2_scatter": 2 * ks * n,               # keys in, keys out
        "lds_build": 2 * ks * n + 4 * B,            # keys in, keys out, offsets out
        # probe, sorted path
        "qsplit1_count": ks * q,                    # read queries
        "qsplit1_scatter": (2 * ks + 2) * q,        # queries in and out, 16-bit tile slots out
        "qsplit2_count": ks * q,
        "qsplit2_scatter": (2 * ks + 2) * q,
        "lds_probe": ks * q + 4 * B + ks * n + cb * q,  # queries, offsets, table keys, counts out
        "qgather2": (2 + 2 * cb) * q,               # tile slots, counts in, counts out
        "qgather1": (2 + cb + 4) * q,               # tile slots, counts in, u32 counts out
        # batched tables
        "bsplit_count": ks * n,
        "bsplit_scatter": 2 * ks * n,
        "blds_build": 2 * ks * n + 4 * B,
        "bqsplit_count": ks * q,
        "bqsplit_scatter": (2 * ks + 2) * q,
        "blds_probe": ks * q + 4 * B + ks * n + cb * q,
        "bqgather": (2 + cb + 4) * q,
        # atomic path and direct probe
        "zero_counts": 4 * (B + 1),                 # counters written
        "bucket_hist": ks * n + 4 * B,              # keys in, counters out once
        "bucket_scan": 8 * B,                       # counters in, offsets out
        "bucket_scatter": 2 * ks * n + 8 * B,       # keys in and out, cursors in and out
        "part_scatter": 2 * ks * n,
        "probe_count": q * (ks + 4 + 8 + ks),       # query, count, two offsets, one key
        "probe_found": q * (ks + 1 + 8 + ks),
    }
    return float(table.get(kernel, 0))


def read_traffic_file(workload: str) -> dict | None:
    """The committed rocprofv3 counter summary of a workload as key -> value
    strings, or None when absent or taken on another kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#") and "=" in line:
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return vals


def read_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when absent or taken on another kernel source."""
    vals = read_traffic_file(workload)
    if vals is None:
        return None
    key = f"hbm_bytes_per_launch.{kernel}"
    return float(vals[key]) if key in vals else None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(workload: str, n_one: int, n_all: int):
    """The oracle, as it stands, on bounded samples of the same workload: the
    plain build on one thread, and the same source built for all host cores
    (OpenMP, GNU parallel-mode sort) on the threads OpenMP takes."""
    import oracle
    from paper_2104_00792_amd import inputs

    def run(n):
        keys, queries, opts = inputs.make_workload(workload, n=n)
        t0 = time.perf_counter()
        oracle.build_table(keys, P=opts["P"], num=opts["num"], den=opts["den"])
        oracle.count(keys, queries)
        return time.perf_counter() - t0

    dt1 = run(n_one)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    with oracle.all_cores(threads):
        dt_all = run(n_all)
    what = ("oracle build (sort of (p,b,key) tuples + run-length) + oracle count (sorted copy + "
            "equal_range)")
    return {"value": n_all / dt_all, "unit": "keys/s", "cores": threads, "kind": "oracle",
            "sample": f"{workload} recipe at n=q={n_all}: {what}, all-core build of the oracle on {threads} "
                      f"threads, {dt_all:.1f} s",
            "single_thread": {"value": n_one / dt1, "unit": "keys/s", "cores": 1,
                              "sample": f"same recipe at n=q={n_one}, single thread, {dt1:.1f} s"},
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


def full_size_parity(workload: str, table, counts) -> dict | None:
    """Compare one step's outputs with the digests of the oracle's outputs
    at this workload's full size (tests/golden/fullsize_digests.json,
    written from the oracle alone).  None when no digest exists for it."""
    import importlib.util

    path = os.path.join(ROOT, "tests", "golden", "fullsize.py")
    spec = importlib.util.spec_from_file_location("fullsize", path)
    fs = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(fs)
    want = fs.load().get(workload)
    if want is None or want["inputs"]["n"] != table.n or want["inputs"]["q"] != counts.numel():
        return None
    po, bb, offs, tk = table.export()
    got = fs.digest(po.cpu().numpy(), bb.cpu().numpy(), offs.cpu().numpy(), tk.cpu().numpy(),
                    counts.cpu().numpy())
    fields = fs.compare(got, want)
    return {"match": all(fields.values()), "fields": fields,
            "against": "digests of the oracle's outputs at full size (offsets and counts bit for bit, "
                       "bucket contents as an order-free multiset hash), tests/golden/fullsize_digests.json"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="p16_u32_2^28", choices=sorted(DESCRIPTIONS))
    ap.add_argument("--n", type=int, default=None, help="override the key count (same recipe)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true", help="skip the full-size parity check")
    ap.add_argument("--cpu-sample", type=int, default=1 << 24, help="keys of the single-thread oracle sample")
    ap.add_argument("--cpu-sample-all", type=int, default=1 << 26, help="keys of the all-core oracle sample")
    ap.add_argument("--requests", type=int, default=100000, help="serving: requests in the stream")
    ap.add_argument("--tables", type=int, default=4096, help="batched: number of tables")
    ap.add_argument("--occ", default=None, help="dup sweep: comma-separated keys per bucket (default: all)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed steps, copy 256 MiB once (device to device) so that a counter "
                         "run of this command also measures a plain copy of known size")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(one GPU's share of the paper's multi-GPU build is what it measures)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2104_00792_amd as hg
    from paper_2104_00792_amd import inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    hg.lib()
    if args.workload == "batched_u32_4096":
        return run_batched(args, dev)
    if args.workload == "serving":
        return run_serving(args, dev)
    if args.workload == "copy_ceiling":
        return run_ceiling(args, dev)
    if args.workload == "dup_sweep_u32_2^28":
        return run_dup_sweep(args, dev)

    w = inputs.WORKLOADS[args.workload]
    n = w["n"] if args.n is None else args.n
    log(f"generating {args.workload} n={n} on {torch.cuda.get_device_name(dev)}")
    keys, queries, opts = inputs.make_workload(args.workload, n=n, device=dev)
    q = queries.numel()
    ks = keys.element_size()
    counts = torch.empty(q, dtype=torch.uint32, device=dev)
    torch.cuda.synchronize()

    def step():
        t = hg.hg_build(keys, P=opts["P"], ratio=(opts["num"], opts["den"]))
        hg.hg_count(t, queries, out=counts)
        t.free()

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t_probe = hg.hg_build(keys, P=opts["P"], ratio=(opts["num"], opts["den"]))
    info = t_probe.info()
    B = info["num_buckets"]
    ws, tb = hg.hg_workspace_size(hg.HG_OP_BUILD, n=n, key_type=0 if ks == 4 else 1, P=opts["P"],
                                  ratio=(opts["num"], opts["den"]))
    wq, _ = hg.hg_workspace_size(hg.HG_OP_COUNT, n=q, table=t_probe)
    t_probe.free()

    log(f"timing {args.steps} steps")
    sizes = dict(n=n, q=q, B=B, ks=ks, P=opts["P"])
    sec, kernels, roof = timed_with_roofline(hg, step, args.steps, sizes, args.workload,
                                             cb=info["probe_count_bytes"])
    ms_per_step = sec * 1000.0
    value = n / sec
    log("graph replays")
    graph = graph_timing(step, ws + tb + wq, counts, args.steps)
    parity = None
    if not args.no_parity:
        log("full-size parity against the oracle's digests")
        t_chk = hg.hg_build(keys, P=opts["P"], ratio=(opts["num"], opts["den"]))
        hg.hg_count(t_chk, queries, out=counts)
        torch.cuda.synchronize()
        parity = full_size_parity(args.workload, t_chk, counts)
        t_chk.free()

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "keys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32" if ks == 4 else "u64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {DESCRIPTIONS[args.workload]}", "n": n, "q": q,
                   "P": opts["P"], "table_ratio": f"{opts['num']}/{opts['den']}", "num_buckets": B},
        "roofline": roof,
        "graph": dict(graph, keys_per_s=n / (graph["ms_per_step"] / 1000.0)),
        "kernels": kernels,
        "launch_share": launch_share(kernels, ms_per_step),
    }
    if parity is not None:
        result["parity"] = parity
    if args.calibrate_copy:
        src = torch.ones(1 << 26, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu_baseline:
        log(f"cpu baseline on samples of {args.cpu_sample} (one thread) and {args.cpu_sample_all} (all cores)")
        result["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_sample, args.cpu_sample_all)
    print(json.dumps(result), flush=True)


def timed_with_roofline(hg, step, steps: int, sizes: dict, workload: str, cb: int = 4):
    """Per-kernel table from one pass with every launch bracketed by HIP
    events; then the timed pass, with events around the dominant kernel's
    launches only (the events of the other launches cost the step about
    3%).  Returns (seconds per step, kernel table, roofline entry).

    The dominant kernel is the slowest one that carries out a step of the
    scope table's model; `achieved` is that step's model bytes per launch
    (survey_bytes) over the kernel's average launch time in the timed pass.
    `kernel_model` gives the same kernel's rate under this design's own
    bytes (algorithmic_bytes), and `step` the whole step against the
    model's bytes per step, with the counter total of the committed
    profile beside it when that profile matches the kernel sources."""
    with hg.profile() as prof_all:
        timed(step, steps, 0)
    kernels = kernel_table(prof_all.results, steps, sizes, cb)
    dom = max((k for k in kernels if survey_bytes(k, **sizes) > 0), key=lambda k: kernels[k]["ms_per_step"])
    with hg.profile(only=dom) as prof:
        sec = timed(step, steps, 0)
    launches, total_ms = prof.results[dom]
    avg_s = total_ms / launches / 1000.0
    achieved = survey_bytes(dom, **sizes) / avg_s / 1e9
    own = algorithmic_bytes(dom, **sizes, cb=cb) / avg_s / 1e9
    step_bytes = survey_step_bytes(**sizes)
    step_gbs = step_bytes / sec / 1e9
    vals = read_traffic_file(workload)
    counter = float(vals["hbm_bytes_per_step"]) if vals and "hbm_bytes_per_step" in vals else None
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": read_traffic(workload, dom),
            "traffic_scale": ({"fetch": float(vals["fetch_scale"]), "write": float(vals["write_scale"])}
                              if vals else None),
            "kernel_model": {"bytes_per_launch": algorithmic_bytes(dom, **sizes, cb=cb), "achieved": round(own, 1),
                             "frac": round(own / HBM_PEAK_GBS, 4)},
            "step": {"alg_bytes": step_bytes, "alg_bytes_per_pair": round(step_bytes / sizes["n"], 2),
                     "achieved": round(step_gbs, 1), "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                     "counter_bytes": counter,
                     "counter_achieved": round(counter / sec / 1e9, 1) if counter else None,
                     "counter_frac": round(counter / sec / 1e9 / HBM_PEAK_GBS, 4) if counter else None,
                     "design_bytes": sum(algorithmic_bytes(k, **sizes, cb=cb) * v["launches_per_step"]
                                         for k, v in kernels.items())}}
    return sec, kernels, roof


def launch_share(kernels: dict, ms_per_step: float) -> dict:
    """How much of a step lies between launches: the step's time against the
    sum of its launch groups' event times (each group one or more dispatches
    of one library call site, such as the LDS build with its heavy-key passes)."""
    busy = sum(v["ms_per_step"] for v in kernels.values())
    groups = sum(v["launches_per_step"] for v in kernels.values())
    between = max(0.0, ms_per_step - busy)
    return {"launch_groups_per_step": groups, "kernel_ms_per_step": round(busy, 4),
            "between_launches_ms": round(between, 4), "between_frac": round(between / ms_per_step, 4)}


def kernel_table(prof_results: dict, steps: int, sizes: dict, cb: int = 4) -> dict:
    out = {}
    for name, (launches, total_ms) in prof_results.items():
        avg = total_ms / launches
        ab = algorithmic_bytes(name, **sizes, cb=cb)
        out[name] = {"launches_per_step": launches // steps, "avg_ms": round(avg, 5),
                     "ms_per_step": round(total_ms / steps, 5),
                     "alg_GBs": round(ab / (avg / 1000.0) / 1e9, 1) if avg > 0 and ab else None}
    return out


def graph_timing(step, arena_bytes: int, out, steps: int) -> dict:
    """One step captured in a HIP graph (library memory from an arena of
    the size hg_workspace_size reports), replayed `steps` times; the replay's
    output must equal the eager step's."""
    import torch

    from paper_2104_00792_amd.graph import Arena, Captured

    step()
    torch.cuda.synchronize()
    eager = out.clone()
    cap = Captured(step, Arena(arena_bytes))
    out.view(torch.int32).zero_()
    sec = timed(cap.replay, steps, 1)
    same = bool(torch.equal(out.view(torch.int32), eager.view(torch.int32)))
    del cap, eager
    torch.cuda.synchronize()
    return {"ms_per_step": sec * 1000.0, "arena_bytes": arena_bytes, "replays_match_eager": same}


def timed(fn, steps: int, warmup: int):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def run_batched(args, dev):
    """4096 tables built and probed in one call each, against the same keys
    as one plain table and against one hg_build + hg_count per table."""
    import numpy as np
    import torch

    import paper_2104_00792_amd as hg
    from paper_2104_00792_amd import inputs

    sizes = inputs.batch_sizes(args.tables)
    total = int(sizes.sum())
    log(f"generating {args.tables} tables, {total} keys")
    keys = inputs.batch_keys_t(sizes, dev)
    queries = inputs.batch_queries_t(keys, sizes, sizes, dev)
    koff = torch.from_numpy(inputs.segment_offsets(sizes)).to(dev)
    counts = torch.empty(total, dtype=torch.uint32, device=dev)
    torch.cuda.synchronize()

    from paper_2104_00792_amd import tune

    log("tuning the sub-bin size (untimed)")
    tuned = tune.tune_batched(keys, koff, queries, koff, reps=2, use_cache=False)
    sub = tuned["log2_subbin"]
    log(f"tuned: log2_subbin={sub} ({tuned['ms']:.3f} ms vs {tuned['default_ms']:.3f} ms by default)")

    def step():
        t = hg.hg_build_batched(keys, koff, log2_subbin=sub)
        hg.hg_count_batched(t, queries, koff, out=counts)
        t.free()

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    t = hg.hg_build_batched(keys, koff, log2_subbin=sub)
    B = t.info()["num_buckets"]
    ws, tb = hg.hg_workspace_size(hg.HG_OP_BUILD_BATCHED, n=total, aux=args.tables, log2_subbin=sub)
    wq, _ = hg.hg_workspace_size(hg.HG_OP_COUNT_BATCHED, n=total, table=t)
    t.free()
    log(f"timing {args.steps} steps")
    sz = dict(n=total, q=total, B=B, ks=4, P=1)
    sec, kernels, roof = timed_with_roofline(hg, step, args.steps, sz, "batched_u32_4096")
    graph = graph_timing(step, ws + tb + wq, counts, args.steps)

    def plain():
        t1 = hg.hg_build(keys)
        hg.hg_count(t1, queries, out=counts)
        t1.free()

    log("plain single table over the same keys")
    sec_plain = timed(plain, max(1, args.steps // 2), 1)
    o = inputs.segment_offsets(sizes).astype(np.int64)

    def loop():
        for i in range(args.tables):
            a, b = int(o[i]), int(o[i + 1])
            t1 = hg.hg_build(keys[a:b])
            hg.hg_count(t1, queries[a:b], out=counts[a:b])
            t1.free()

    log("one build + count per table")
    sec_loop = timed(loop, 1, 1)
    result = {
        "metric": "batched build+probe keys/s (4096 tables of 2^10..2^20 keys)",
        "value": total / sec, "unit": "keys/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1000.0, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"batched_u32_4096: {DESCRIPTIONS['batched_u32_4096']}", "tables": args.tables,
                   "keys": total, "queries": total, "num_buckets": B},
        "vs_plain_path": {"single_table_same_keys_keys_per_s": total / sec_plain,
                          "one_call_per_table_keys_per_s": total / sec_loop,
                          "speedup_over_one_call_per_table": sec_loop / sec},
        "tuning": tuned,
        "graph": dict(graph, keys_per_s=total / (graph["ms_per_step"] / 1000.0)),
        "roofline": roof,
        "kernels": kernels,
        "launch_share": launch_share(kernels, sec * 1000.0),
    }
    print(json.dumps(result), flush=True)


def run_ceiling(args, dev):
    """What plain streaming reaches on this GPU: torch's copy (read + write),
    fill (write) and sum (read) of 1 GiB, each timed with HIP events over
    `steps` launches after one warm-up."""
    import torch

    nbytes = 1 << 30
    a = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    out = torch.empty((), dtype=torch.int64, device=dev)

    def rate(fn, moved):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        return {"ms": round(ms, 4), "GBs": round(moved / (ms / 1000.0) / 1e9, 1),
                "frac_of_peak": round(moved / (ms / 1000.0) / 1e9 / HBM_PEAK_GBS, 4)}

    res = {"copy": rate(lambda: b.copy_(a), 2 * nbytes), "fill": rate(lambda: b.fill_(7), nbytes),
           "read_sum": rate(lambda: torch.sum(a, 0, dtype=torch.int64, out=out), nbytes)}
    best = max(v["GBs"] for v in res.values())
    print(json.dumps({"metric": "streaming ceiling GB/s", "value": best, "unit": "GB/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": 1, "ms_per_step": res["copy"]["ms"], "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "i32", "data": "synthetic",
                      "config": {"workload": f"copy_ceiling: {DESCRIPTIONS['copy_ceiling']}", "bytes": nbytes},
                      "ceilings": res, "peak": HBM_PEAK_GBS}), flush=True)


DUP_OCCUPANCIES = (1, 4, 16, 64, 256, 1024, 4096)


def run_dup_sweep(args, dev):
    """Build and probe rates as the hash range shrinks (the paper varies V with
    the key count fixed; the average number of keys per bucket is n / V).
    Per point: `steps` builds (each freed) and `steps` probes of one table,
    each series timed with HIP events after one warm-up, and 256 sampled
    queries checked against their exact multiplicity (a count of equal keys
    over the whole key array, outside the timed region)."""
    import torch
    import paper_2104_00792_amd as hg
    from paper_2104_00792_amd import inputs

    n = 1 << 28 if args.n is None else args.n
    keys, queries, opts = inputs.make_workload("p16_u32_2^28", n=n, device=dev)
    P = opts["P"]
    q = queries.numel()
    counts = torch.empty(q, dtype=torch.uint32, device=dev)
    ki = keys.view(torch.int32)
    pick = torch.randint(0, q, (256,), generator=torch.Generator().manual_seed(0x5EED), dtype=torch.int64).to(dev)
    sample = queries.view(torch.int32)[pick]
    exact = torch.stack([(ki == sample[j]).sum() for j in range(sample.numel())]).to(torch.int64).cpu()
    torch.cuda.synchronize()

    def series(fn, steps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    occs = DUP_OCCUPANCIES if args.occ is None else tuple(int(x) for x in args.occ.split(","))
    points = []
    for occ in occs:
        log(f"keys per bucket {occ}")
        ratio = (1, occ)
        build_ms = series(lambda: hg.hg_build(keys, P=P, ratio=ratio).free(), args.steps)
        t = hg.hg_build(keys, P=P, ratio=ratio)
        B = t.info()["num_buckets"]
        count_ms = series(lambda: hg.hg_count(t, queries, out=counts), args.steps)
        got = counts.view(torch.int32)[pick].to(torch.int64).cpu()
        t.free()
        points.append({"occ": occ, "num_buckets": B, "build_ms": round(build_ms, 4), "count_ms": round(count_ms, 4),
                       "build_keys_per_s": n / (build_ms / 1000.0), "count_queries_per_s": q / (count_ms / 1000.0),
                       "sample_exact": bool(torch.equal(got, exact))})
    worst = max(points, key=lambda p: p["build_ms"] + p["count_ms"])
    step_ms = worst["build_ms"] + worst["count_ms"]
    print(json.dumps({"metric": "build+probe keys/s across keys per bucket (Sec. 5.4 duplicate study), worst point",
                      "value": n / (step_ms / 1000.0), "unit": "keys/s", "n_gpus": 1, "steps": args.steps,
                      "warmup": 1, "ms_per_step": step_ms, "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "u32", "data": "synthetic",
                      "config": {"workload": f"dup_sweep_u32_2^28: {DESCRIPTIONS['dup_sweep_u32_2^28']}", "n": n,
                                 "q": q, "P": P},
                      "points": points}), flush=True)


def run_serving(args, dev):
    """Closed loop (every request present at t = 0) for capacity, then the
    open-loop Poisson stream at 0.5, 0.8 and 0.95 of it (0.8 is the headline);
    latencies from arrival to completion."""
    from paper_2104_00792_amd import serve

    log(f"serving {args.requests} requests")
    closed, opened, _ = serve.run_serving(num=args.requests, slots=SERVING_SLOTS, capacity_bytes=200 * 10**9,
                                          loads=(0.5, 0.8, 0.95), progress=lambda m: log(m))
    head = opened[0.8]
    result = {
        "metric": "serving p50/p99 latency and throughput (open loop at 0.8 of capacity)",
        "value": head["keys_per_s"], "unit": "keys/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": head["wall_s"] * 1000.0, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"serving: {DESCRIPTIONS['serving']}", "requests": args.requests},
        "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"],
        "open_loop": head, "open_loop_by_load": {str(k): v for k, v in opened.items()}, "closed_loop": closed,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
