"""Serving loop: admission under an HBM cap, LRU eviction with pins, rebuilds,
latency accounting, and results that are the same alone and in the mix.

CPU tests drive the server with an executor built on the oracle and a
virtual clock; the GPU test drives the HIP library on concurrent streams.
Counts are integers, so "the same" means exactly equal."""

import numpy as np
import pytest

import oracle
from paper_2104_00792_amd import inputs, serve


class Token:
    def __init__(self, finish):
        self.finish = finish


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def wait(self, server, next_arrival):
        cands = [tok.finish for tok, _, _, _ in server.inflight]
        if next_arrival is not None:
            cands.append(next_arrival)
        if cands:
            self.t = max(self.t, min(cands))


class OracleExecutor:
    """A device that serves each request in time proportional to its size."""

    def __init__(self, clock, per_key=1e-8, fixed=1e-5):
        self.clock = clock
        self.per_key, self.fixed = per_key, fixed
        self.cost = 0.0
        self.freed = 0

    def pick_stream(self):
        return None

    def prepare(self, req, sizes, seeds):
        if req.kind == "build":
            return inputs.uniform_u32(req.size, req.seed)
        return inputs.table_queries(sizes[req.table], seeds[req.table], req.size, req.seed)

    def ready(self, payload):
        return True

    def table_keys(self, n, seed, stream):
        return inputs.uniform_u32(n, seed)

    def build(self, keys, stream):
        self.cost += self.fixed + self.per_key * keys.size
        return keys

    def probe(self, table, queries, stream):
        self.cost += self.fixed + self.per_key * queries.size
        return oracle.count(table, queries)

    def record(self, stream):
        tok = Token(self.clock.now() + self.cost)
        self.cost = 0.0
        return tok

    def done(self, token, now):
        return now >= token.finish

    def finish_time(self, token, now):
        return token.finish

    def fetch(self, out):
        return out

    def free(self, table):
        self.freed += 1


def alone(req, sizes, seeds):
    keys = inputs.uniform_u32(sizes[req.table], seeds[req.table])
    queries = inputs.queries_hit50(keys, req.size, req.seed)
    return oracle.count(keys, queries)


def small_trace(num=80, rate=2e4):
    return serve.make_trace(num, seed=0x77, build_log2=(12, 16), probe_log2=(4, 11), rate=rate)


def tight_cap(sizes):
    """Room for any one request plus about three of the largest tables."""
    big = max(sizes)
    return serve.table_bytes(big) * 4 + serve.build_work_bytes(big) + serve.probe_work_bytes(1 << 11, big)


@pytest.mark.parametrize("slots", [1, 3, 8])
def test_mix_equals_alone_with_evictions(slots):
    reqs, sizes, seeds = small_trace()
    cap = tight_cap(sizes)
    clock = VirtualClock()
    ex = OracleExecutor(clock)
    srv = serve.Server(ex, sizes, seeds, cap, slots)
    srv.run(reqs, clock)
    probes = [r for r in reqs if r.kind == "probe"]
    assert probes
    for r in probes:
        assert np.array_equal(r.result, alone(r, sizes, seeds)), r
    assert srv.cache.peak <= cap
    assert srv.cache.evictions > 0 and srv.rebuilds > 0  # the cap forced both
    assert all(r.finish >= r.start >= r.arrival for r in reqs)


def test_concurrency_overlaps_requests():
    reqs, sizes, seeds = small_trace(rate=1e7)  # everything arrives at once
    clock = VirtualClock()
    srv = serve.Server(OracleExecutor(clock), sizes, seeds, 1 << 40, slots=4)
    srv.run(reqs, clock)
    spans = sorted((r.start, r.finish) for r in reqs)
    overlapping = sum(1 for (s0, f0), (s1, f1) in zip(spans, spans[1:]) if s1 < f0)
    assert overlapping > 0


def test_probe_waits_for_its_build():
    reqs, sizes, seeds = small_trace(rate=1e7)
    clock = VirtualClock()
    serve.Server(OracleExecutor(clock), sizes, seeds, 1 << 40, slots=8).run(reqs, clock)
    built = {}
    for r in reqs:
        if r.kind == "build":
            built.setdefault(r.table, r.finish)
    for r in reqs:
        if r.kind == "probe":
            assert r.start >= built[r.table]


def _blocked_build_scenario():
    """Table A is built, then one long probe of A pins it; a build of table B
    arrives and does not fit beside A and that probe; small probes of A
    arrive after it and do fit."""
    big, small = 1 << 20, 1 << 8
    n = 1 << 16
    reqs = [serve.Request(0, "build", 0, n, 101, 0.0), serve.Request(1, "probe", 0, big, 201, 0.001),
            serve.Request(2, "build", 1, n, 102, 0.002)]
    reqs += [serve.Request(3 + k, "probe", 0, small, 301 + k, 0.003 + 0.001 * k) for k in range(6)]
    cap = serve.table_bytes(n) + serve.probe_work_bytes(big, n) + 2 * serve.probe_work_bytes(small, n) + 100000
    assert serve.table_bytes(n) + serve.build_work_bytes(n) > cap - serve.table_bytes(n) - \
        serve.probe_work_bytes(big, n)
    return reqs, [n, n], [101, 102], cap


def test_waiting_request_does_not_block_later_ones():
    """The build of B waits for memory; the small probes behind it start
    first (no head-of-line blocking), and every result is still exact."""
    reqs, sizes, seeds, cap = _blocked_build_scenario()
    clock = VirtualClock()
    srv = serve.Server(OracleExecutor(clock), sizes, seeds, cap, slots=4, max_wait=1.0)
    srv.run(reqs, clock)
    b = reqs[2]
    assert all(r.start < b.start for r in reqs[3:]), [(r.rid, r.start) for r in reqs]
    assert srv.overtakes >= 6
    for r in reqs:
        if r.kind == "probe":
            assert np.array_equal(r.result, alone(r, sizes, seeds))
    assert srv.cache.peak <= cap


def test_age_bound_stops_overtaking():
    """With no waiting allowed (max_wait = 0) the build of B is never passed
    over: the small probes that arrived after it start after it."""
    reqs, sizes, seeds, cap = _blocked_build_scenario()
    clock = VirtualClock()
    srv = serve.Server(OracleExecutor(clock), sizes, seeds, cap, slots=4, max_wait=0.0)
    srv.run(reqs, clock)
    b = reqs[2]
    assert all(r.start >= b.start for r in reqs[3:]), [(r.rid, r.start) for r in reqs]
    for r in reqs:
        if r.kind == "probe":
            assert np.array_equal(r.result, alone(r, sizes, seeds))


def test_payload_prepared_within_lookahead():
    """The client prepares at most max_prepared payloads ahead, and only
    for requests arriving within the lookahead."""
    reqs, sizes, seeds = small_trace(num=40, rate=100.0)  # 10 ms apart on average
    clock = VirtualClock()
    srv = serve.Server(OracleExecutor(clock), sizes, seeds, 1 << 40, slots=2, lookahead=0.005, max_prepared=3)
    pending = []
    j = srv._prepare(reqs, 0, 0.0, pending)
    assert 1 <= j <= 3 and all(r.arrival <= 0.005 for r in reqs[:j]) and reqs[j].payload is None
    srv.run(reqs, clock)
    assert all(r.finish >= r.arrival for r in reqs)


def test_lru_evicts_oldest_unpinned_first():
    freed = []
    c = serve.TableCache(100, freed.append)
    c.add(1, "a", 30)
    c.add(2, "b", 30)
    c.add(3, "c", 30)
    c.pin(1)          # 1 is in use and now most recent
    assert c.make_room(40)
    assert freed == ["b"]            # 2 is the oldest unpinned
    assert c.resident(1) and c.resident(3) and not c.resident(2)
    c.unpin(1)
    assert c.make_room(70) and freed == ["b", "c", "a"][: len(freed)]
    assert not c.make_room(101)


def test_request_larger_than_cap_is_refused():
    reqs, sizes, seeds = serve.make_trace(3, seed=5, build_log2=(12, 12), probe_log2=(4, 4))
    clock = VirtualClock()
    with pytest.raises(MemoryError):
        serve.Server(OracleExecutor(clock), sizes, seeds, 1000, slots=2).run(reqs, clock)


def test_latency_report_percentiles():
    reqs = [serve.Request(i, "probe", 0, 10, 0, 0.0, 0.0, (i + 1) * 1e-3) for i in range(100)]
    rep = serve.latency_report(reqs, 1.0)
    assert abs(rep["p50_ms"] - 50.5) < 1e-9
    assert abs(rep["p99_ms"] - 99.01) < 1e-6
    assert rep["requests_per_s"] == 100


@pytest.mark.gpu
def test_gpu_mix_equals_alone(gpu):
    """Requests on four concurrent streams with a cap that forces evictions
    and rebuilds; every probe equals the same probe run alone."""
    import torch

    reqs, sizes, seeds = serve.make_trace(60, seed=0x99, build_log2=(8, 16), probe_log2=(6, 14), rate=1e7)
    cap = 3 * serve.table_bytes(max(sizes)) + 4 * serve.build_work_bytes(1 << 16) + \
        4 * serve.probe_work_bytes(1 << 14, 1 << 16)
    clock = serve.WallClock()
    srv = serve.Server(serve.GpuExecutor(4), sizes, seeds, cap, slots=4)
    srv.run(reqs, clock)
    torch.cuda.synchronize()
    for r in reqs:
        if r.kind != "probe":
            continue
        want = alone(r, sizes, seeds)
        assert np.array_equal(r.result.cpu().numpy(), want), r.rid
        keys_np = inputs.uniform_u32(sizes[r.table], seeds[r.table])
        t = gpu.hg_build(torch.from_numpy(keys_np).cuda())
        q = torch.from_numpy(inputs.queries_hit50(keys_np, r.size, r.seed)).cuda()
        assert np.array_equal(gpu.hg_count(t, q).cpu().numpy(), want)
        t.free()
    assert srv.cache.peak <= cap
