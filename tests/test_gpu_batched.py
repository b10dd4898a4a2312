"""Batched tables on the GPU against the oracle, bit-exact: T tables of
uneven sizes (empty, one key, several sub-bins), 32- and 64-bit keys,
duplicates, table ratios, query segments of other sizes, and offsets that
the library must clamp."""

import numpy as np
import pytest

import oracle
from paper_2104_00792_amd import inputs

pytestmark = pytest.mark.gpu


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def make_batch(sizes, dtype, seed, dup=False):
    parts = []
    for i, s in enumerate(sizes):
        if dup:
            p = inputs.sample_with_replacement(s, seed + i, dtype)
        elif dtype == np.uint32:
            p = inputs.uniform_u32(s, seed + i)
        else:
            p = inputs.uniform_u64(s, seed + i)
        parts.append(p)
    keys = np.concatenate(parts) if parts else np.empty(0, dtype)
    return parts, keys, np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)


def check_batch(hg, keys, o, queries, qo, num=1, den=1):
    import torch

    t = hg.hg_build_batched(to_dev(keys), to_dev(o.astype(np.uint32)), ratio=(num, den))
    po, bb, offs, tk = t.export()
    counts = hg.hg_count_batched(t, to_dev(queries), to_dev(qo.astype(np.uint32)))
    found = hg.hg_query_batched(t, to_dev(queries), to_dev(qo.astype(np.uint32)))
    torch.cuda.synchronize()
    ref = oracle.build_batched(keys, o, num, den)
    assert np.array_equal(po.cpu().numpy(), ref["part_offsets"]), "table offsets"
    assert np.array_equal(bb.cpu().numpy(), ref["bucket_base"]), "bucket bases"
    got_offs = offs.cpu().numpy()
    assert np.array_equal(got_offs, ref["offsets"]), "offsets"
    assert np.array_equal(oracle.canonicalize(got_offs, tk.cpu().numpy()), ref["keys"]), "bucket contents"
    want = oracle.count_batched(keys, o, queries, qo)
    got = counts.cpu().numpy()
    assert np.array_equal(got, want), f"{np.count_nonzero(got != want)} of {want.size} counts differ"
    assert np.array_equal(found.cpu().numpy(), (want > 0).astype(np.uint8))
    t.free()


def queries_for(parts, qsizes, seed):
    qs = []
    for i, (p, q) in enumerate(zip(parts, qsizes)):
        if p.size == 0:
            qs.append(inputs.uniform_u32(q, seed + i).astype(p.dtype))
        else:
            qs.append(inputs.queries_hit50(p, q, seed + i))
    dtype = parts[0].dtype
    return (np.concatenate(qs).astype(dtype) if qs else np.empty(0, dtype),
            np.concatenate([[0], np.cumsum(qsizes)]).astype(np.uint32))


CASES = {
    "one_table": [5000],
    "uneven": [0, 1, 3, 1000, 70000, 0, 17, 4097],
    "many_small": [int(x) for x in np.random.default_rng(3).integers(0, 300, 300)],
    "multi_subbin": [(1 << 16) + 5, 3, (1 << 15) - 1, 40000],
    "all_empty": [0, 0, 0],
    # 8390000 buckets at 2^13 per sub-bin: the sub-bin count is capped at
    # 1024, so the last sub-bin holds 9584 buckets and takes the build's
    # 16-bit counters (every other sub-bin takes the 32-bit ones)
    "capped_last_subbin": [8390000, 1000],
}


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64], ids=["u32", "u64"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_batched_tables(gpu, case, dtype):
    sizes = CASES[case]
    parts, keys, o = make_batch(sizes, dtype, 1000)
    queries, qo = queries_for(parts, [max(0, s + (s % 7) - 3) for s in sizes], 2000)
    check_batch(gpu, keys, o, queries, qo)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64], ids=["u32", "u64"])
def test_batched_heavy_key_in_the_16bit_subbin(gpu, dtype):
    """The capped_last_subbin table (8390000 keys; its last sub-bin of 9584
    buckets takes 16-bit counters) with 5000 copies of one key whose bucket
    lies in that sub-bin: the sub-bin then holds about 14600 keys, more than
    the registers take, so the loop path counts and scatters it on packed
    counters, with the copies' counter adds grouped."""
    V = 8390000
    gen = inputs.uniform_u32 if dtype == np.uint32 else inputs.uniform_u64
    cand = gen(200000, 91)
    _, b = oracle.hash_bucket(cand, V)
    heavy = cand[b >= 1023 * 8192][0]
    table = np.concatenate([gen(V - 5000, 92), np.full(5000, heavy, dtype)])
    table = table[inputs.uniform_u32(V, 93).argsort(kind="stable")]
    small = gen(1000, 94)
    keys = np.concatenate([table, small])
    o = np.array([0, V, V + 1000], np.uint32)
    q0 = np.concatenate([np.full(10, heavy, dtype), table[::50]])
    queries = np.concatenate([q0, small])
    qo = np.array([0, q0.size, queries.size], np.uint32)
    check_batch(gpu, keys, o, queries, qo)


@pytest.mark.parametrize("num, den", [(1, 2), (3, 2), (4, 1)])
def test_batched_ratios_and_duplicates(gpu, num, den):
    sizes = [3000, 0, 12000, 500, 1]
    parts, keys, o = make_batch(sizes, np.uint32, 77, dup=True)
    queries, qo = queries_for(parts, [100, 5, 20000, 0, 9], 78)
    check_batch(gpu, keys, o, queries, qo, num, den)


def test_batched_offsets_are_clamped(gpu):
    """Offsets that go backwards or past n: the library clamps them to a
    non-decreasing sequence from 0 to n, as documented, and the result is
    the oracle's batch for the clamped offsets."""
    keys = inputs.uniform_u32(9000, 12)
    o = np.array([3, 4000, 2500, 8000, 12000, 9000], np.uint32)
    queries = inputs.queries_hit50(keys, 7000, 13)
    qo = np.array([0, 100, 50, 7000, 6999, 99999], np.uint32)
    check_batch(gpu, keys, o, queries, qo)


def test_batched_table_rejects_plain_probe(gpu):
    keys = to_dev(inputs.uniform_u32(100, 1))
    t = gpu.hg_build_batched(keys, to_dev(np.array([0, 50, 100], np.uint32)))
    with pytest.raises(gpu.HGError):
        gpu.hg_count(t, keys)
    plain = gpu.hg_build(keys)
    with pytest.raises(gpu.HGError):
        gpu.hg_count_batched(plain, keys, to_dev(np.array([0, 100], np.uint32)))
    t.free()
    plain.free()
