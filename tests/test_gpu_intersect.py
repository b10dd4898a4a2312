"""Querying by a HashGraph of the queries and per-bucket intersections
(Sec. 3.3) on the GPU, bit-exact against the oracle: the query table's
part_offsets, bucket_base and offsets raw, its buckets as sorted multisets;
the intersection counts against the definition (count of each query key
among the table's keys) and against hg_count of the same keys."""

import numpy as np
import pytest

import oracle
from paper_2104_00792_amd import inputs

pytestmark = pytest.mark.gpu


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


CASES = [
    # (key kind, n, q, P, num, den, V)
    ("u32", 5000, 3000, 1, 1, 1, 0),           # atomic build, direct probe sizes
    ("u32", (1 << 20) + 7, (1 << 19) + 3, 16, 1, 1, 0),
    ("u32", (1 << 22) + 13, (1 << 21) + 1, 16, 1, 1, 0),  # sorted build of both tables
    ("u32", 100000, 0, 4, 1, 1, 0),            # empty query set
    ("u32", 70000, 90000, 1, 1, 1, 1 << 16),   # plain table, fixed V
    ("u64", 300000, 200000, 8, 1, 2, 0),
    ("zipf", 1 << 18, 1 << 17, 1, 1, 2, 0),    # long buckets in both tables
    ("u32", (1 << 21) + 5, (1 << 20) + 9, 16, 1, 64, 0),  # 64 keys per bucket: small sub-bins, sorted long buckets
    ("u32", (1 << 21) + 5, (1 << 20) + 9, 1, 1, 2048, 0),  # 2048 keys per bucket: wave and workgroup sorts
]


@pytest.mark.parametrize("kind, n, q, P, num, den, V", CASES)
def test_query_table_and_intersections(gpu, kind, n, q, P, num, den, V):
    import torch

    hg = gpu
    if kind == "zipf":
        keys = inputs.zipf_u64(n, 1 << 12, 0x1A)
        queries = inputs.zipf_u64(q, 1 << 12, 0x1B)
    else:
        keys = inputs.uniform_u32(n, 0x1C) if kind == "u32" else inputs.uniform_u64(n, 0x1C)
        queries = inputs.queries_hit50(keys, q, 0x1D)
    t = hg.hg_build(to_dev(keys), P=P, ratio=(num, den), num_buckets=V)
    qt = hg.hg_build_like(t, to_dev(queries))
    po, bb, offs, qk = qt.export()
    counts = hg.hg_intersect(t, qt)
    direct = hg.hg_count(t, qk, flags=hg.HG_PROBE_DIRECT) if q else counts
    torch.cuda.synchronize()
    want = oracle.build_like(keys, queries, P, num, den, V)
    assert np.array_equal(po.cpu().numpy(), want["part_offsets"]), "query partition offsets"
    assert np.array_equal(bb.cpu().numpy(), want["bucket_base"]), "bucket bases (the table's)"
    got_offs = offs.cpu().numpy()
    assert np.array_equal(got_offs, want["offsets"]), "query table offsets"
    qk = qk.cpu().numpy()
    assert np.array_equal(oracle.canonicalize(got_offs, qk), want["keys"]), "query buckets"
    got = counts.cpu().numpy()
    assert np.array_equal(got, oracle.count(keys, qk)), "intersection counts"
    assert np.array_equal(got, direct.cpu().numpy())
    qt.free()
    t.free()


def test_intersect_rejects_a_table_not_built_like(gpu):
    hg = gpu
    keys = to_dev(inputs.uniform_u32(10000, 0x2A))
    t1 = hg.hg_build(keys)
    t2 = hg.hg_build(keys)
    qt = hg.hg_build_like(t1, keys)
    with pytest.raises(hg.HGError) as err:
        hg.hg_intersect(t2, qt)
    assert err.value.status == 1
    for t in (qt, t2, t1):
        t.free()
