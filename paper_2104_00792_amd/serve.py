"""Serving loop: continuous batching of build and probe requests.

Requests arrive over time (a Poisson stream), each carrying its data: the
keys of a build, the queries of a probe.  The client side prepares that
payload on its own stream shortly before the request arrives (a bounded
lookahead), so a request's latency covers the server's work, not the
generation of its input.

A request is admitted as soon as an execution slot is free, its payload is
ready and its device memory fits under the HBM cap, evicting
least-recently-used tables that no in-flight request holds.  Admission
follows arrival order, but a request that must wait (for memory, for its
payload, or for the build of its table) does not hold up later requests
that can start, until it has waited `max_wait` seconds: from then on nothing
behind it starts before it, so no request starves.  Admitted requests run
concurrently, each on the stream of its slot, so the work of requests that
arrived at different times overlaps on the device.  Built tables stay
resident for later probes.  A probe whose table was evicted rebuilds it from
the table's seed first, on the probe's own stream, so every result is the
same whatever the mix.

The executor does the work: ``GpuExecutor`` calls the HIP library on torch
streams; tests plug in a CPU executor with a virtual clock.
"""

from __future__ import annotations

import dataclasses
import math
import time
from collections import OrderedDict

import numpy as np

from . import inputs

KEY_BYTES = 4


@dataclasses.dataclass
class Request:
    rid: int
    kind: str          # "build" or "probe"
    table: int         # table id (a build creates it, a probe reads it)
    size: int          # keys to build, or queries to probe
    seed: int          # build: key stream; probe: query stream
    arrival: float     # seconds from the start of the stream
    start: float = math.nan
    finish: float = math.nan
    result: object = None
    payload: object = None  # the request's keys or queries, once the client has prepared them


def table_bytes(n: int) -> int:
    """Resident bytes of a table of n 32-bit keys at table ratio 1."""
    return KEY_BYTES * n + 4 * (n + 2) + 4096


def build_work_bytes(n: int) -> int:
    """Transient device memory of a build of n keys: the keys (the request's
    payload, or regenerated for a rebuild), two split buffers and the split
    counts."""
    return 3 * KEY_BYTES * n + n // 2 + (1 << 20)


def probe_work_bytes(q: int, table_n: int) -> int:
    """Transient device memory of a probe: the queries (its payload), two
    split buffers, the slot and count arrays.  (table_n: kept for callers
    that size by table; the queries no longer need the table's keys.)"""
    return 3 * KEY_BYTES * q + 12 * q + (1 << 20)


def payload_bytes(req: Request) -> int:
    return KEY_BYTES * req.size


def make_trace(num: int, seed: int = 0x5EED0500, build_frac: float = 0.3, build_log2=(10, 24),
               probe_log2=(8, 22), rate: float = 1000.0):
    """A Poisson stream of `num` requests at `rate` per second.  Builds create
    new tables (uint32 keys, sizes log-uniform over 2^build_log2); probes
    (sizes log-uniform over 2^probe_log2, 50% hits) target a table chosen
    uniformly among those created earlier.  Returns (requests, table sizes,
    table seeds)."""
    w = inputs.splitmix64(seed, 0, 4 * num)
    u = (w >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    t = 0.0
    reqs, sizes, seeds = [], [], []
    for i in range(num):
        u0, u1, u2, u3 = (float(x) for x in u[4 * i:4 * i + 4])
        t += -math.log(1.0 - u0) / rate
        if u1 < build_frac or not sizes:
            lo, hi = build_log2
            size = int(round(2.0 ** (lo + (hi - lo) * u2)))
            sizes.append(size)
            seeds.append(seed + 1 + i)
            reqs.append(Request(i, "build", len(sizes) - 1, size, seed + 1 + i, t))
        else:
            lo, hi = probe_log2
            size = int(round(2.0 ** (lo + (hi - lo) * u2)))
            tid = min(int(u3 * len(sizes)), len(sizes) - 1)
            reqs.append(Request(i, "probe", tid, size, seed + 1 + i, t))
    return reqs, sizes, seeds


class TableCache:
    """Resident tables under a byte budget, least recently used evicted first;
    a table pinned by an in-flight request is never evicted."""

    def __init__(self, capacity: int, free_fn):
        self.capacity = capacity
        self.used = 0       # bytes of resident tables
        self.reserved = 0   # bytes held by in-flight requests
        self.entries: OrderedDict[int, list] = OrderedDict()  # tid -> [table, bytes, pins]
        self.free_fn = free_fn
        self.evictions = 0
        self.peak = 0

    def resident(self, tid: int) -> bool:
        return tid in self.entries

    def pin(self, tid: int):
        self.entries[tid][2] += 1
        self.entries.move_to_end(tid)

    def unpin(self, tid: int):
        self.entries[tid][2] -= 1

    def fits(self, need: int) -> bool:
        return self.used + self.reserved + need <= self.capacity

    def make_room(self, need: int) -> bool:
        """Evict unpinned tables, least recently used first, until `need`
        more bytes fit."""
        for tid in list(self.entries):
            if self.fits(need):
                break
            table, nbytes, pins = self.entries[tid]
            if pins == 0:
                del self.entries[tid]
                self.used -= nbytes
                self.free_fn(table)
                self.evictions += 1
        return self.fits(need)

    def add(self, tid: int, table, nbytes: int, pins: int = 0):
        self.entries[tid] = [table, nbytes, pins]
        self.used += nbytes
        self.peak = max(self.peak, self.used + self.reserved)


class Server:
    """Continuous batching over `slots` concurrent requests.

    lookahead: the client prepares the payloads of requests that arrive
    within this many seconds, at most `max_prepared` (or `max_prepared_bytes`)
    at a time.  max_wait: seconds a waiting request may be passed over by
    later ones."""

    def __init__(self, executor, table_sizes, table_seeds, capacity_bytes: int, slots: int = 4,
                 lookahead: float = 0.02, max_prepared: int = 64, max_prepared_bytes: int = 4 << 30,
                 max_wait: float = 0.05, scan: int = 64):
        self.ex = executor
        self.sizes = table_sizes
        self.seeds = table_seeds
        self.cache = TableCache(capacity_bytes, executor.free)
        self.slots = slots
        self.inflight = []  # [token, request, reserved bytes, output]
        self.rebuilds = 0
        self.lookahead = lookahead
        self.max_prepared = max_prepared
        self.max_prepared_bytes = max_prepared_bytes
        self.max_wait = max_wait
        self.scan = scan
        self.overtakes = 0  # admissions ahead of an earlier waiting request
        self.unbuilt = set()

    def _admit(self, req: Request, now: float) -> bool:
        tid = req.table
        if req.kind == "build":
            need = table_bytes(req.size) + build_work_bytes(req.size)
            if not self.cache.make_room(need):
                return False
            rebuild = False
        else:
            n = self.sizes[tid]
            rebuild = not self.cache.resident(tid)
            need = probe_work_bytes(req.size, n)
            if rebuild:
                need += table_bytes(n) + build_work_bytes(n)
            else:
                self.cache.pin(tid)  # never evict the probe's own table
            if not self.cache.make_room(need):
                if not rebuild:
                    self.cache.unpin(tid)
                return False
        stream = self.ex.pick_stream()
        if req.kind == "build":
            out = self.ex.build(req.payload, stream)
        else:
            if rebuild:
                # The rebuilt table is resident from now on: its bytes move
                # from this request's reservation to the cache.
                self.rebuilds += 1
                table = self.ex.build(self.ex.table_keys(self.sizes[tid], self.seeds[tid], stream), stream)
                tb = table_bytes(self.sizes[tid])
                self.cache.add(tid, table, tb, pins=1)
                need -= tb
            out = self.ex.probe(self.cache.entries[tid][0], req.payload, stream)
        req.payload = None  # the stream holds it until the request's work is done
        self.cache.reserved += need
        self.cache.peak = max(self.cache.peak, self.cache.used + self.cache.reserved)
        req.start = now
        self.inflight.append([self.ex.record(stream), req, need, out])
        return True

    def _retire(self, now: float):
        still = []
        for token, req, need, out in self.inflight:
            if not self.ex.done(token, now):
                still.append([token, req, need, out])
                continue
            req.finish = self.ex.finish_time(token, now)
            self.cache.reserved -= need
            if req.kind == "build":
                self.unbuilt.discard(req.table)
                if self.cache.resident(req.table):  # rebuilt for a probe meanwhile
                    self.ex.free(out)
                else:
                    self.cache.add(req.table, out, table_bytes(req.size))
            else:
                req.result = self.ex.fetch(out)
                self.cache.unpin(req.table)
        self.inflight = still

    def _prepare(self, reqs, j: int, now: float, pending: list) -> int:
        """Client side: prepare the payloads of requests j.. that arrive
        within the lookahead, keeping at most max_prepared of them (and
        max_prepared_bytes) prepared but not yet admitted."""
        held = sum(payload_bytes(r) for r in pending)
        while j < len(reqs) and reqs[j].arrival <= now + self.lookahead and len(pending) < self.max_prepared:
            if pending and held + payload_bytes(reqs[j]) > self.max_prepared_bytes:
                break
            reqs[j].payload = self.ex.prepare(reqs[j], self.sizes, self.seeds)
            held += payload_bytes(reqs[j])
            pending.append(reqs[j])
            j += 1
        return j

    def run(self, reqs, clock, progress=None, every: int = 5000):
        """Serve `reqs` (sorted by arrival) against `clock`; `progress(msg)`
        is called each time `every` more requests have been admitted."""
        queue = []    # arrived, not admitted, in arrival order
        pending = []  # payload prepared, not admitted
        i = j = 0
        admitted = 0
        # Tables whose first build has not completed: their probes wait.
        self.unbuilt = {r.table for r in reqs if r.kind == "build"}
        while i < len(reqs) or queue or self.inflight:
            now = clock.now()
            j = self._prepare(reqs, j, now, pending)
            while i < len(reqs) and reqs[i].arrival <= now and i < j:
                queue.append(reqs[i])
                i += 1
            self._retire(now)
            # Admit in arrival order while slots allow.  A request that
            # cannot start yet (payload not ready, its table's build still
            # running, memory short) is passed over, unless it has waited
            # max_wait: then nothing behind it starts first.
            k = 0
            while k < len(queue) and k < self.scan and len(self.inflight) < self.slots:
                req = queue[k]
                aged = now - req.arrival > self.max_wait
                if not self.ex.ready(req.payload):
                    if aged:
                        break
                    k += 1
                    continue
                if req.kind == "probe" and req.table in self.unbuilt:
                    k += 1  # its table's build (earlier in the queue, or running) comes first
                    continue
                if not self._admit(req, now):
                    if not self.inflight:
                        raise MemoryError(f"request {req.rid} needs more than the HBM cap")
                    if aged:
                        break
                    k += 1
                    continue
                if k > 0:
                    self.overtakes += 1
                queue.pop(k)
                pending.remove(req)
                admitted += 1
                if progress is not None and admitted % every == 0:
                    progress(f"admitted {admitted} of {len(reqs)}")
            # The next event that is not a completion: the next prepared
            # request's arrival, or the moment the next one enters the
            # lookahead (none while the prepared ones fill the limit).
            if i < j:
                nxt = reqs[i].arrival
            elif j < len(reqs) and len(pending) < self.max_prepared:
                nxt = max(now, reqs[j].arrival - self.lookahead)
            else:
                nxt = None
            clock.wait(self, nxt)
        return reqs


def latency_report(reqs, wall: float) -> dict:
    lat = np.array([r.finish - r.arrival for r in reqs])
    keys = sum(r.size for r in reqs)
    return {
        "requests": len(reqs),
        "wall_s": round(wall, 4),
        "requests_per_s": len(reqs) / wall if wall > 0 else None,
        "keys_per_s": keys / wall if wall > 0 else None,
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
    }


# --------------------------------------------------------------------------
# GPU execution: the HIP library, each slot on its own torch stream (all at
# the default priority).
# --------------------------------------------------------------------------

class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def wait(self, server, next_arrival):
        if not server.inflight and next_arrival is not None:
            dt = next_arrival - self.now()
            if dt > 0:
                time.sleep(min(dt, 0.005))


class GpuExecutor:
    """Requests on `slots` torch streams.  keep_results=False drops each
    probe's counts once it completes (a long stream would otherwise hold
    every result in device memory)."""

    def __init__(self, slots: int, device=None, keep_results: bool = True):
        import torch

        import paper_2104_00792_amd as hg

        self.torch = torch
        self.hg = hg
        self.dev = device or torch.device("cuda:0")
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(slots)]
        self.client = torch.cuda.Stream(device=self.dev)  # where payloads are drawn
        self.next = 0
        self.oom_retries = 0
        self.keep_results = keep_results

    def pick_stream(self):
        s = self.streams[self.next % len(self.streams)]
        self.next += 1
        return s

    def _retry_on_oom(self, fn):
        """Run fn; if the device is out of memory (both torch's cache and the
        library's block cache keep freed blocks of many sizes), wait for the device,
        hand both caches back and run it once more."""
        try:
            return fn()
        except (self.hg.HGError, self.torch.cuda.OutOfMemoryError) as e:
            if isinstance(e, self.hg.HGError) and e.status != 2:
                raise
            self.torch.cuda.synchronize()
            self.torch.cuda.empty_cache()
            self.hg.hg_trim_pool(0)
            self.oom_retries += 1
            return fn()

    def prepare(self, req, sizes, seeds):
        """The client's payload of `req`, drawn on the client stream: a
        build's keys, or a probe's queries (50% hits among its table's keys,
        drawn without the table's key array).  Returns (tensor, event)."""
        def run():
            with self.torch.cuda.stream(self.client):
                if req.kind == "build":
                    x = inputs.uniform_u32_t(req.size, req.seed, self.dev)
                else:
                    x = inputs.table_queries_t(sizes[req.table], seeds[req.table], req.size, req.seed, self.dev)
                ev = self.torch.cuda.Event()
                ev.record(self.client)
            return x, ev

        return self._retry_on_oom(run)

    def ready(self, payload) -> bool:
        return payload[1].query()

    def table_keys(self, n: int, seed: int, stream):
        """A table's keys regenerated by the server (rebuild after an
        eviction), on the request's stream."""
        with self.torch.cuda.stream(stream):
            x = inputs.uniform_u32_t(n, seed, self.dev)
            ev = self.torch.cuda.Event()
            ev.record(stream)
        return x, ev

    def _use(self, payload, stream):
        x, ev = payload
        stream.wait_event(ev)
        x.record_stream(stream)
        return x

    def build(self, payload, stream):
        def run():
            keys = self._use(payload, stream)
            with self.torch.cuda.stream(stream):
                return self.hg.hg_build(keys, stream=stream)

        return self._retry_on_oom(run)

    def probe(self, table, payload, stream):
        def run():
            queries = self._use(payload, stream)
            with self.torch.cuda.stream(stream):
                return self.hg.hg_count(table, queries, stream=stream)

        return self._retry_on_oom(run)

    def record(self, stream):
        ev = self.torch.cuda.Event()
        ev.record(stream)
        return ev

    def done(self, token, now) -> bool:
        return token.query()

    def finish_time(self, token, now: float) -> float:
        return now

    def fetch(self, out):
        return out if self.keep_results else None

    def free(self, table):
        table.free()


def run_serving(num: int = 2000, slots: int = 4, capacity_bytes: int = 200 * 10**9, rate: float | None = None,
                build_log2=(10, 24), probe_log2=(8, 22), loads=(0.8,), progress=None):
    """Closed-loop capacity first (every request present at t = 0), then an
    open-loop Poisson stream at each of `loads` times that capacity (or at
    `rate` requests/s).  Returns the closed-loop report, the open-loop
    reports by load, and the last open-loop requests."""
    import torch

    reqs, sizes, seeds = make_trace(num, build_log2=build_log2, probe_log2=probe_log2, rate=1.0)
    for r in reqs:
        r.arrival = 0.0
    clock = WallClock()
    ex = GpuExecutor(slots, keep_results=False)
    srv = Server(ex, sizes, seeds, capacity_bytes, slots)
    srv.run(reqs, clock, progress)
    torch.cuda.synchronize()
    closed = latency_report(reqs, clock.now())
    closed.update(evictions=srv.cache.evictions, rebuilds=srv.rebuilds, peak_reserved_bytes=srv.cache.peak,
                  oom_retries=ex.oom_retries, overtakes=srv.overtakes)
    _release(srv, ex)
    opened = {}
    for load in loads:
        lam = rate if rate is not None else load * closed["requests_per_s"]
        if progress is not None:
            progress(f"open loop at {load} of capacity ({lam:.0f} requests/s offered)")
        reqs, sizes, seeds = make_trace(num, build_log2=build_log2, probe_log2=probe_log2, rate=lam)
        clock = WallClock()
        ex = GpuExecutor(slots, keep_results=False)
        srv = Server(ex, sizes, seeds, capacity_bytes, slots)
        srv.run(reqs, clock, progress)
        torch.cuda.synchronize()
        rep = latency_report(reqs, clock.now())
        rep.update(load=load, offered_requests_per_s=lam, evictions=srv.cache.evictions, rebuilds=srv.rebuilds,
                   peak_reserved_bytes=srv.cache.peak, oom_retries=ex.oom_retries, overtakes=srv.overtakes,
                   sustained=rep["requests_per_s"] >= 0.97 * lam)
        opened[load] = rep
        _release(srv, ex)
    return closed, opened, reqs


def _release(srv, ex):
    """Free every resident table and hand the device memory back."""
    import torch

    for tid in list(srv.cache.entries):
        ex.free(srv.cache.entries.pop(tid)[0])
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    ex.hg.hg_trim_pool(0)
