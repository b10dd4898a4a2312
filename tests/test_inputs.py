"""The seeded workload generators (no hash table arithmetic in them)."""

import os

import numpy as np

from paper_2104_00792_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_splitmix64_published_sequence():
    with open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) as f:
        want = [int(x) for x in f if x.strip() and not x.startswith("#")]
    assert [int(x) for x in inputs.splitmix64(1234567, 0, len(want))] == want


def test_counter_based_slices():
    full = inputs.splitmix64(99, 0, 10000)
    assert np.array_equal(inputs.splitmix64(99, 1234, 777), full[1234:1234 + 777])
    q = inputs.queries_hit50(inputs.uniform_u32(5000, 1), 9000, 5)
    assert q.size == 9000


def test_uniform_u32_spread():
    k = inputs.uniform_u32(1 << 20, 3)
    assert k.dtype == np.uint32
    # top nibble close to uniform
    c = np.bincount(k >> np.uint32(28), minlength=16)
    assert np.all(np.abs(c - (1 << 16)) < 6 * 256)


def test_hit_rate_about_half():
    keys = inputs.uniform_u32(1 << 20, 4)
    q = inputs.queries_hit50(keys, 1 << 20, 8)
    hit = np.isin(q, keys).mean()
    assert 0.49 < hit < 0.51


def test_zipf_rank_one_frequency():
    K, n = 1 << 20, 1 << 21
    r = inputs.zipf_ranks(n, K, 6)
    H = np.sum(1.0 / np.arange(1, K + 1))
    f1 = np.count_nonzero(r == 1) / n
    assert abs(f1 - 1.0 / H) < 0.005
    assert r.min() >= 1 and r.max() <= K
    v = inputs.zipf_u64(1 << 16, K, 6)
    assert v.dtype == np.uint64


def test_zipf_u32_is_the_high_half_of_zipf_u64():
    K = 1 << 20
    v64 = inputs.zipf_u64(1 << 16, K, 9)
    v32 = inputs.zipf_u32(1 << 16, K, 9)
    assert v32.dtype == np.uint32
    assert np.array_equal(v32, (v64 >> np.uint64(32)).astype(np.uint32))
    # the rank structure survives: as many distinct values, up to a rare merge
    assert abs(np.unique(v32).size - np.unique(v64).size) <= 2


def test_sequential_and_sample_with_replacement():
    assert inputs.sequential(5).tolist() == [1, 2, 3, 4, 5]
    s = inputs.sample_with_replacement(1 << 16, 2)
    assert s.min() >= 1 and s.max() <= 1 << 16


def test_named_workloads_shapes():
    for name in inputs.WORKLOADS:
        keys, queries, opts = inputs.make_workload(name, n=1000)
        assert keys.size == 1000 and queries.size == 1000
        assert keys.dtype == queries.dtype
        assert set(opts) == {"P", "num", "den"}


def test_torch_twin_equals_numpy():
    import torch

    for name in inputs.WORKLOADS:
        k, q, _ = inputs.make_workload(name, n=30011, q=20011)
        kt, qt, _ = inputs.make_workload(name, n=30011, q=20011, device=torch.device("cpu"))
        assert np.array_equal(kt.numpy(), k), name
        assert np.array_equal(qt.numpy(), q), name


def test_batch_generators_match_their_torch_twins():
    import torch

    sizes = inputs.batch_sizes(40, 0, 9, seed=77)
    sizes[3] = 0
    keys = inputs.batch_keys(sizes)
    qsizes = sizes + 3
    queries = inputs.batch_queries(keys, sizes, qsizes)
    kt = inputs.batch_keys_t(sizes, "cpu", chunk=1000)
    qt = inputs.batch_queries_t(kt, sizes, qsizes, "cpu", chunk=777)
    assert np.array_equal(kt.numpy(), keys)
    assert np.array_equal(qt.numpy(), queries)
    o = inputs.segment_offsets(sizes)
    for t in (0, 5, 39):
        assert np.array_equal(keys[o[t]:o[t + 1]], inputs.uniform_u32(int(sizes[t]), inputs.BATCH_KEY_SEED + t))


def test_batch_sizes_are_log_uniform():
    s = inputs.batch_sizes(4096)
    assert s.min() >= 1 << 10 and s.max() <= 1 << 20
    lg = np.log2(s)
    assert abs(lg.mean() - 15) < 0.2 and abs((lg < 12.5).mean() - 0.25) < 0.03
