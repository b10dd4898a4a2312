"""Device memory from a caller's allocator (hg_set_allocator) and the sizes
that hg_workspace_size reports, on the GPU.

An arena of exactly the reported size serves each call; the results equal
those of the same calls served by the library's block cache; every block goes back
once, tables to the allocator they were built with; an allocator that fails
or breaks the alignment contract turns into an error with nothing leaked.
Counts and offsets are integers, so "equal" means bit-exact."""

import numpy as np
import pytest

from paper_2104_00792_amd import inputs

pytestmark = pytest.mark.gpu


class Arena:
    """Bump allocator over one torch buffer, rounding blocks to 256 bytes as
    the library's sizes do."""

    def __init__(self, nbytes):
        import torch

        self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")
        self.base = self.buf.data_ptr()
        assert self.base % 256 == 0
        self.size = nbytes
        self.off = 0
        self.live = {}
        self.calls = 0
        self.fail_at = None
        self.misalign = False

    def alloc(self, nbytes, stream):
        self.calls += 1
        if self.fail_at is not None and self.calls == self.fail_at:
            return 0
        r = (nbytes + 255) & ~255
        if self.off + r > self.size:
            return 0
        p = self.base + self.off + (16 if self.misalign else 0)
        self.off += r
        self.live[p] = nbytes
        return p

    def free(self, ptr, nbytes, stream):
        assert self.live.pop(ptr) == nbytes


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def pool_reference(hg, keys, queries, P, ratio):
    import torch

    t = hg.hg_build(keys, P=P, ratio=ratio)
    counts = hg.hg_count(t, queries)
    _, _, offs, _ = t.export()
    torch.cuda.synchronize()
    out = counts.cpu().numpy(), offs.cpu().numpy()
    t.free()
    return out


@pytest.mark.parametrize("n, dtype, P, ratio", [
    ((1 << 22) + 12345, np.uint32, 16, (1, 1)),   # sorted build, sorted probe
    (5000, np.uint32, 1, (1, 1)),                 # atomic build, direct probe
    ((1 << 21) + 7, np.uint64, 1, (1, 2)),         # 64-bit keys
])
def test_arena_of_the_reported_size_serves_build_and_probe(gpu, n, dtype, P, ratio):
    import torch

    hg = gpu
    raw = inputs.uniform_u32(n, 0xA110C) if dtype == np.uint32 else inputs.uniform_u64(n, 0xA110C)
    keys = to_dev(raw)
    queries = to_dev(inputs.queries_hit50(raw, n, 0xA110D))
    want_counts, want_offs = pool_reference(hg, keys, queries, P, ratio)
    kt = hg.HG_KEY_U32 if dtype == np.uint32 else hg.HG_KEY_U64

    ws, tb = hg.hg_workspace_size(hg.HG_OP_BUILD, n=n, key_type=kt, P=P, ratio=ratio)
    build_arena = Arena(ws + tb)
    try:
        hg.hg_set_allocator(build_arena.alloc, build_arena.free)
        t = hg.hg_build(keys, P=P, ratio=ratio)
        torch.cuda.synchronize()
        assert build_arena.off == ws + tb            # every block came from the arena
        assert sum((b + 255) & ~255 for b in build_arena.live.values()) == tb  # the table's blocks

        wq, tq = hg.hg_workspace_size(hg.HG_OP_COUNT, n=n, table=t)
        assert tq == 0
        probe_arena = Arena(wq)
        hg.hg_set_allocator(probe_arena.alloc, probe_arena.free)
        counts = hg.hg_count(t, queries)
        torch.cuda.synchronize()
        assert probe_arena.off == wq and not probe_arena.live
    finally:
        hg.hg_set_allocator()
    _, _, offs, _ = t.export()
    torch.cuda.synchronize()
    assert np.array_equal(counts.cpu().numpy(), want_counts)
    assert np.array_equal(offs.cpu().numpy(), want_offs)
    t.free()  # back to the build arena, not to the pool or the probe arena
    torch.cuda.synchronize()
    assert not build_arena.live


def test_batched_calls_in_an_arena(gpu):
    import torch

    hg = gpu
    sizes = inputs.batch_sizes(64)[:64] // 16 + 1
    keys_np = np.concatenate([inputs.uniform_u32(int(s), 0xB0 + i) for i, s in enumerate(sizes)])
    o = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
    keys, offs = to_dev(keys_np), to_dev(o)
    queries = to_dev(inputs.queries_hit50(keys_np, keys_np.size, 0xB1))
    t0 = hg.hg_build_batched(keys, offs)
    want = hg.hg_count_batched(t0, queries, offs).cpu().numpy()
    t0.free()

    ws, tb = hg.hg_workspace_size(hg.HG_OP_BUILD_BATCHED, n=keys_np.size, aux=len(sizes))
    arena = Arena(ws + tb)
    try:
        hg.hg_set_allocator(arena.alloc, arena.free)
        t = hg.hg_build_batched(keys, offs)
        wq, _ = hg.hg_workspace_size(hg.HG_OP_COUNT_BATCHED, n=keys_np.size, table=t)
        qa = Arena(wq)
        hg.hg_set_allocator(qa.alloc, qa.free)
        got = hg.hg_count_batched(t, queries, offs)
        torch.cuda.synchronize()
        assert arena.off == ws + tb and qa.off == wq and not qa.live
    finally:
        hg.hg_set_allocator()
    assert np.array_equal(got.cpu().numpy(), want)
    t.free()
    torch.cuda.synchronize()
    assert not arena.live


def test_torch_caching_allocator(gpu):
    import torch

    hg = gpu
    n = (1 << 22) + 99
    raw = inputs.uniform_u32(n, 0xC0)
    keys = to_dev(raw)
    queries = to_dev(inputs.queries_hit50(raw, n, 0xC1))
    want_counts, want_offs = pool_reference(hg, keys, queries, 16, (1, 1))
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    _, tb = hg.hg_workspace_size(hg.HG_OP_BUILD, n=n, P=16)
    with hg.torch_allocator():
        t = hg.hg_build(keys, P=16)
        counts = hg.hg_count(t, queries)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() - before >= tb + 4 * n  # the table and the counts
    po, bb, offs, tk = t.export()
    torch.cuda.synchronize()
    assert np.array_equal(counts.cpu().numpy(), want_counts)
    assert np.array_equal(offs.cpu().numpy(), want_offs)
    del counts, po, bb, offs, tk
    t.free()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before


@pytest.mark.parametrize("fail_at", [1, 2, 3])
def test_allocator_failure_is_out_of_memory_and_leaks_nothing(gpu, fail_at):
    """The first blocks of a build are taken before its first launch, so the
    failing call enqueues no work."""
    hg = gpu
    keys = to_dev(inputs.uniform_u32(100000, 0xD0))
    arena = Arena(1 << 26)
    arena.fail_at = fail_at
    try:
        hg.hg_set_allocator(arena.alloc, arena.free)
        with pytest.raises(hg.HGError) as err:
            hg.hg_build(keys, P=4)
    finally:
        hg.hg_set_allocator()
    assert err.value.status == 2
    assert not arena.live


def test_misaligned_block_is_rejected_and_returned(gpu):
    hg = gpu
    keys = to_dev(inputs.uniform_u32(1000, 0xD1))
    arena = Arena(1 << 22)
    arena.misalign = True
    try:
        hg.hg_set_allocator(arena.alloc, arena.free)
        with pytest.raises(hg.HGError) as err:
            hg.hg_build(keys)
    finally:
        hg.hg_set_allocator()
    assert err.value.status == 1 and "aligned" in str(err.value)
    assert not arena.live and arena.calls == 1


def test_block_cache_reuses_freed_blocks(gpu):
    """Repeated build + count + free on one stream is served from the
    library's block cache: device memory does not grow after the first
    round, every round's results are equal, and hg_trim_pool(0) hands the
    idle blocks back."""
    import torch

    hg = gpu
    n = (1 << 22) + 5
    raw = inputs.uniform_u32(n, 0xE0)
    keys = to_dev(raw)
    queries = to_dev(inputs.queries_hit50(raw, n, 0xE1))
    counts = torch.empty(n, dtype=torch.uint32, device="cuda")

    def round_trip():
        t = hg.hg_build(keys, P=16)
        hg.hg_count(t, queries, out=counts)
        t.free()

    round_trip()
    torch.cuda.synchronize()
    want = counts.cpu().numpy().copy()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(5):
        counts.zero_()
        round_trip()
        torch.cuda.synchronize()
        assert np.array_equal(counts.cpu().numpy(), want)
    _, tb = hg.hg_workspace_size(hg.HG_OP_BUILD, n=n, P=16)
    # Without reuse every round would take at least one more table; the HIP
    # runtime's own buffers may move the figure by a few MiB.
    assert free0 - torch.cuda.mem_get_info()[0] <= 8 << 20 < tb
    hg.hg_trim_pool(0)
    assert torch.cuda.mem_get_info()[0] >= free0 + tb


def test_block_cache_across_streams(gpu):
    """Blocks freed on one stream and requested on another while the first
    stream may still be working: every result equals the one computed
    alone (a block handed over before its last use had completed would
    corrupt the first stream's table or counts)."""
    import torch

    hg = gpu
    sizes = [(1 << 21) + 17, (1 << 20) + 3]
    raws = [inputs.uniform_u32(m, 0xE10 + i) for i, m in enumerate(sizes)]
    keys = [to_dev(r) for r in raws]
    queries = [to_dev(inputs.queries_hit50(r, m, 0xE20 + i)) for i, (r, m) in enumerate(zip(raws, sizes))]
    want = []
    for k, q in zip(keys, queries):
        t = hg.hg_build(k, P=4)
        want.append(hg.hg_count(t, q).cpu().numpy())
        t.free()
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())
    outs = []
    for it in range(6):
        for j, s in enumerate(streams):
            w = (it + j) % 2
            with torch.cuda.stream(s):
                t = hg.hg_build(keys[w], P=4)
                c = hg.hg_count(t, queries[w])
                t.free()
            outs.append((w, c, s))
    torch.cuda.synchronize()
    for w, c, _ in outs:
        assert np.array_equal(c.cpu().numpy(), want[w])
