"""Build + probe captured in a HIP graph and replayed.

The library's blocks come from an arena sized by hg_workspace_size, so the
graph holds kernel launches only.  Each test replays the graph several times
with eager library work and synchronizations in between, and checks every
replay's counts against the eager result (bit-exact, integers)."""

import numpy as np
import pytest

from paper_2104_00792_amd import inputs

pytestmark = pytest.mark.gpu


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def test_plain_build_and_count_replay(gpu):
    import torch
    from paper_2104_00792_amd.graph import Arena, Captured

    hg = gpu
    n = (1 << 22) + 123  # sorted build and sorted probe, P = 16
    raw = inputs.uniform_u32(n, 0xE0)
    keys = to_dev(raw)
    queries = to_dev(inputs.queries_hit50(raw, n, 0xE1))
    t0 = hg.hg_build(keys, P=16)
    want = hg.hg_count(t0, queries).cpu().numpy()
    ws, tb = hg.hg_workspace_size(hg.HG_OP_BUILD, n=n, P=16)
    wq, _ = hg.hg_workspace_size(hg.HG_OP_COUNT, n=n, table=t0)
    t0.free()

    counts = torch.zeros(n, dtype=torch.uint32, device="cuda")

    def step():
        t = hg.hg_build(keys, P=16)
        hg.hg_count(t, queries, out=counts)
        t.free()

    cap = Captured(step, Arena(ws + tb + wq))
    assert cap.arena.high == ws + tb + wq  # every block of both calls from the arena
    other = to_dev(inputs.uniform_u32(100000, 0xE2))
    for r in range(3):
        counts.view(torch.int32).zero_()
        cap.replay()
        torch.cuda.synchronize()
        assert np.array_equal(counts.cpu().numpy(), want), f"replay {r}"
        # eager library work between replays, from the pool
        t = hg.hg_build(other)
        hg.hg_count(t, other)
        t.free()
        torch.cuda.synchronize()


def test_batched_build_and_count_replay(gpu):
    import torch
    from paper_2104_00792_amd.graph import Arena, Captured

    hg = gpu
    sizes = inputs.batch_sizes(96) // 8 + 1
    keys_np = np.concatenate([inputs.uniform_u32(int(s), 0xF0 + i) for i, s in enumerate(sizes)])
    o = to_dev(np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32))
    keys = to_dev(keys_np)
    queries = to_dev(inputs.queries_hit50(keys_np, keys_np.size, 0xF1))
    t0 = hg.hg_build_batched(keys, o)
    want = hg.hg_count_batched(t0, queries, o).cpu().numpy()
    ws, tb = hg.hg_workspace_size(hg.HG_OP_BUILD_BATCHED, n=keys_np.size, aux=len(sizes))
    wq, _ = hg.hg_workspace_size(hg.HG_OP_COUNT_BATCHED, n=keys_np.size, table=t0)
    t0.free()

    counts = torch.zeros(keys_np.size, dtype=torch.uint32, device="cuda")

    def step():
        t = hg.hg_build_batched(keys, o)
        hg.hg_count_batched(t, queries, o, out=counts)
        t.free()

    cap = Captured(step, Arena(ws + tb + wq))
    for r in range(3):
        counts.view(torch.int32).zero_()
        cap.replay()
        torch.cuda.synchronize()
        assert np.array_equal(counts.cpu().numpy(), want), f"replay {r}"
        t = hg.hg_build_batched(keys, o)
        assert np.array_equal(hg.hg_count_batched(t, queries, o).cpu().numpy(), want)
        t.free()
        torch.cuda.synchronize()


def test_tuning_knobs_do_not_change_the_table(gpu):
    """log2_subbin and split_bits change speed only: for every setting the
    partition offsets, bucket bases, offsets, bucket contents and counts are
    the oracle's.  (10, 7) makes level-1 segments smaller than a partition's
    table, so the build splits by coarse bucket ranges (it launches the
    partition count first); the other settings split by partition."""
    import torch

    import oracle

    hg = gpu
    n = (1 << 22) + 777
    raw = inputs.uniform_u32(n, 0xD5)
    raw_q = inputs.queries_hit50(raw, n, 0xD6)
    keys = to_dev(raw)
    queries = to_dev(raw_q)
    ref = oracle.build_table(raw, P=16)
    want = oracle.count(raw, raw_q)
    coarse = {}
    for sub, bits in [(0, 0), (11, 7), (12, 9), (13, 10), (10, 8), (10, 7)]:
        with hg.profile() as prof:
            t = hg.hg_build(keys, P=16, log2_subbin=sub, split_bits=bits)
            po, bb, offs, tk = t.export()
            c = hg.hg_count(t, queries)
            torch.cuda.synchronize()
        coarse[(sub, bits)] = "part_count" in prof.results
        offs, tk, c = offs.cpu().numpy(), tk.cpu().numpy(), c.cpu().numpy()
        assert np.array_equal(po.cpu().numpy(), ref["part_offsets"]), (sub, bits)
        assert np.array_equal(bb.cpu().numpy(), ref["bucket_base"]), (sub, bits)
        assert np.array_equal(offs, ref["offsets"]), (sub, bits)
        assert np.array_equal(oracle.canonicalize(offs, tk), ref["keys"]), (sub, bits)
        assert np.array_equal(c, want), (sub, bits)
        t.free()
    assert coarse[(10, 7)] and not coarse[(0, 0)], coarse


def test_batched_subbin_knob(gpu):
    import torch

    hg = gpu
    sizes = inputs.batch_sizes(64) // 4 + 1
    keys_np = np.concatenate([inputs.uniform_u32(int(s), 0xC5 + i) for i, s in enumerate(sizes)])
    o = to_dev(np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32))
    keys = to_dev(keys_np)
    queries = to_dev(inputs.queries_hit50(keys_np, keys_np.size, 0xC6))
    ref = None
    for sub in (0, 11, 12, 13):
        t = hg.hg_build_batched(keys, o, log2_subbin=sub)
        _, _, offs, _ = t.export()
        c = hg.hg_count_batched(t, queries, o)
        torch.cuda.synchronize()
        got = (offs.cpu().numpy(), c.cpu().numpy())
        if ref is None:
            ref = got
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), sub
        t.free()
