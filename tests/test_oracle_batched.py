"""The oracle's batch of tables, pinned to its definition: each table is
the plain single-table oracle on its own keys, and the batch is their CSRs
laid end to end."""

import numpy as np

import oracle
from paper_2104_00792_amd import inputs


def test_clamp_offsets_examples():
    assert oracle.clamp_offsets([0, 5, 9], 9).tolist() == [0, 5, 9]
    assert oracle.clamp_offsets([7, 5, 3, 9], 9).tolist() == [0, 5, 5, 9]  # first entry forced to 0
    assert oracle.clamp_offsets([0, 12, 4, 3], 10).tolist() == [0, 10, 10, 10]
    assert oracle.clamp_offsets([0, 2, 1, 5], 4).tolist() == [0, 2, 2, 4]  # last entry forced to n


def test_single_table_batch_is_the_plain_table():
    keys = inputs.uniform_u32(3000, 5)
    a = oracle.build_batched(keys, np.array([0, 3000]), 3, 2)
    b = oracle.build_table(keys, P=1, num=3, den=2)
    for k in ("part_offsets", "bucket_base", "offsets", "keys"):
        assert np.array_equal(a[k], b[k]), k


def test_batch_is_tables_end_to_end():
    sizes = [0, 1, 700, 5, 2048]
    parts = [inputs.uniform_u32(s, 100 + i) for i, s in enumerate(sizes)]
    keys = np.concatenate(parts)
    o = np.concatenate([[0], np.cumsum(sizes)])
    r = oracle.build_batched(keys, o)
    base = 0
    for t, part in enumerate(parts):
        one = oracle.build_table(part)
        V = int(one["bucket_base"][1])
        assert r["bucket_base"][t] == base and V == max(1, sizes[t])
        seg = r["offsets"][base:base + V + 1].astype(np.int64) - int(o[t])
        assert np.array_equal(seg, one["offsets"].astype(np.int64))
        assert np.array_equal(r["keys"][o[t]:o[t + 1]], one["keys"])
        base += V
    assert r["bucket_base"][-1] == base and r["offsets"][-1] == keys.size
    q = np.concatenate([inputs.queries_hit50(p, max(1, p.size), 9) if p.size else p for p in parts])
    qo = np.concatenate([[0], np.cumsum([max(1, s) if s else 0 for s in sizes])])
    got = oracle.count_batched(keys, o, q, qo)
    want = np.concatenate([oracle.count(p, q[qo[t]:qo[t + 1]]) for t, p in enumerate(parts)])
    assert np.array_equal(got, want)
