"""GPU parity of the large-table build path: the coarse-range level-1 split.

When a partition's table is larger than one level-1 segment can cover
(2^split_bits sub-bins of 2^log2_subbin buckets), the sorted build first
counts and scans the hash-range partitions (Algorithm 2, Phase 2) to fix
every table size V_p, and then splits the keys by coarse ranges of global
buckets, which cross the partition bases.  The 2^28-key, 16-partition
workload runs exactly this path.  Each case here asserts from the launch
record that the path was taken (the partition count `part_count` runs only
in that mode), then compares with the oracle element by element: partition
offsets, bucket bases and offsets raw, keys with each bucket sorted, counts
raw, found == (count > 0).  Queries go through the same coarse split.
"""

import numpy as np
import pytest

import oracle
from paper_2104_00792_amd import inputs

pytestmark = pytest.mark.gpu


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def check_coarse(hg, keys, queries, P, num=1, den=1, log2_subbin=0, split_bits=0):
    import torch

    kd, qd = to_dev(keys), to_dev(queries)
    with hg.profile() as prof:
        t = hg.hg_build(kd, P=P, ratio=(num, den), log2_subbin=log2_subbin, split_bits=split_bits)
        po, bb, offs, tk = t.export()
        counts = hg.hg_count(t, qd, flags=hg.HG_PROBE_SORTED)
        found = hg.hg_query(t, qd, flags=hg.HG_PROBE_SORTED)
        torch.cuda.synchronize()
    names = set(prof.results)
    assert "part_count" in names and "split1_count" in names, f"coarse-range split not taken: {sorted(names)}"
    assert "qsplit1_scatter" in names and "lds_probe" in names, "sorted probe not taken"
    ref = oracle.build_table(keys, P=P, num=num, den=den)
    assert np.array_equal(po.cpu().numpy(), ref["part_offsets"]), "part_offsets"
    assert np.array_equal(bb.cpu().numpy(), ref["bucket_base"]), "bucket_base"
    got_offs = offs.cpu().numpy()
    assert np.array_equal(got_offs, ref["offsets"]), "offsets"
    assert np.array_equal(oracle.canonicalize(got_offs, tk.cpu().numpy()), ref["keys"]), "bucket contents"
    want = oracle.count(keys, queries)
    got = counts.cpu().numpy()
    assert np.array_equal(got, want), f"counts: {np.count_nonzero(got != want)} of {want.size} differ"
    assert np.array_equal(found.cpu().numpy(), (want > 0).astype(np.uint8)), "found"
    t.free()


def test_default_knobs_p16_u32(gpu):
    """2^25 + 2^22 + 7 uniform u32 keys, 16 partitions, default knobs: each
    partition's table (about 2.4 M buckets) exceeds one segment of 255
    sub-bins of 2^13 buckets, so the build takes the coarse-range split with
    the same knobs as the 2^28 workload.  Queries: 2^22 at 50% hits."""
    n = (1 << 25) + (1 << 22) + 7
    keys = inputs.uniform_u32(n, 0x5EED0002)
    queries = inputs.queries_hit50(keys, 1 << 22, 0x5EED0102)
    check_coarse(gpu, keys, queries, P=16)


# (P, table ratio): every case gives partitions of more than
# 127 * 2^10 + 2^13 buckets, the most one level-1 segment covers at
# log2_subbin = 10 and split_bits = 7.
SMALL_KNOB_CASES = [(2, 1, 1), (16, 1, 1), (256, 16, 1)]


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64], ids=["u32", "u64"])
@pytest.mark.parametrize("P, num, den", SMALL_KNOB_CASES)
def test_small_knobs_cross_partition_bases(gpu, dtype, P, num, den):
    """2^22 + 777 keys with 2^10-bucket sub-bins and at most 2^7 level-2
    digits: the coarse ranges (2^17 buckets) are far smaller than a
    partition's table, do not start at partition bases, and the last range
    of each partition spills into the next one."""
    n = (1 << 22) + 777
    gen = inputs.uniform_u32 if dtype == np.uint32 else inputs.uniform_u64
    keys = gen(n, 0xC0A5 + P)
    queries = inputs.queries_hit50(keys, n, 0xC0A6 + P)
    check_coarse(gpu, keys, queries, P=P, num=num, den=den, log2_subbin=10, split_bits=7)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64], ids=["u32", "u64"])
def test_small_knobs_heavy_keys(gpu, dtype):
    """Zipf(1.0) keys over 2^16 values (the most frequent with about 180000
    copies) among uniform ones, 16 partitions, the same small knobs: heavy
    sub-bins shared by many workgroups and sorted long buckets inside the
    coarse-range path; queries Zipf-distributed the same way plus uniform."""
    n = (1 << 22) + 777
    z = inputs.zipf_u64(n // 2, 1 << 16, 0xC0B1)
    u = inputs.uniform_u64(n - n // 2, 0xC0B2)
    keys = np.concatenate([z, u])
    keys = keys[np.argsort(inputs.uniform_u32(keys.size, 0xC0B3), kind="stable")]
    qz = inputs.zipf_u64(1 << 21, 1 << 16, 0xC0B4)
    queries = np.concatenate([qz, inputs.queries_hit50(keys, 1 << 21, 0xC0B5)])
    if dtype == np.uint32:
        keys = (keys >> np.uint64(32)).astype(np.uint32)
        queries = (queries >> np.uint64(32)).astype(np.uint32)
    check_coarse(gpu, keys, queries, P=16, log2_subbin=10, split_bits=7)
