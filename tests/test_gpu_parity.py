"""GPU parity: the HIP path against the CPU oracle, element by element.

Sizes span several 4096-key tiles with ragged tails; key sets cover the
paper's workloads (uniform, sequential {1..n}, sampling with replacement,
Sec. 4.3) and the degenerate ones (empty, one key, all keys equal, Zipf
duplicates, the extreme values 0 and 2^w - 1).  Everything here is integer,
so the bar is bit-exact: part_offsets, bucket_base and offsets raw; keys after
sorting each bucket (the order inside a bucket is left to the atomics of
Algorithm 1); counts raw; found == (count > 0).
"""

import numpy as np
import pytest

import oracle
from paper_2104_00792_amd import inputs

pytestmark = pytest.mark.gpu


def make_keys(kind: str, n: int, dtype, seed: int) -> np.ndarray:
    if kind == "uniform":
        return inputs.uniform_u32(n, seed) if dtype == np.uint32 else inputs.uniform_u64(n, seed)
    if kind == "equal":
        return np.full(n, 0xDEADBEEF, dtype=dtype)
    if kind == "seq":
        return inputs.sequential(n, dtype)
    if kind == "swr":
        return inputs.sample_with_replacement(n, seed, dtype)
    if kind == "zipf":
        v = inputs.zipf_u64(n, max(1, n // 8), seed)
        return v if dtype == np.uint64 else (v >> np.uint64(32)).astype(np.uint32)
    if kind == "extremes":
        top = np.iinfo(dtype).max
        base = np.array([0, top, 1, top - 1, top // 2, top // 2 + 1], dtype=dtype)
        return np.resize(base, n)
    raise ValueError(kind)


def to_dev(a: np.ndarray):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


BUILDS = {"atomic": 1, "sorted": 2}
PROBES = {"direct": 1, "sorted": 2}


def check_table(hg, keys, P=1, num=1, den=1, V=0, queries=None, build="sorted"):
    """Build with one strategy, probe with both, compare everything."""
    import torch

    t = hg.hg_build(to_dev(keys), P=P, ratio=(num, den), num_buckets=V, flags=BUILDS[build])
    ref = oracle.build_table(keys, P=P, num=num, den=den, V=V)
    po, bb, offs, tk = t.export()
    if queries is None:
        queries = inputs.queries_hit50(keys, max(keys.size, 97), 0xC0FFEE)
    qd = to_dev(queries)
    probes = {name: (hg.hg_count(t, qd, flags=f), hg.hg_query(t, qd, flags=f)) for name, f in PROBES.items()}
    torch.cuda.synchronize()
    assert np.array_equal(po.cpu().numpy(), ref["part_offsets"]), "part_offsets"
    assert np.array_equal(bb.cpu().numpy(), ref["bucket_base"]), "bucket_base"
    got_offs = offs.cpu().numpy()
    assert np.array_equal(got_offs, ref["offsets"]), "offsets"
    got_keys = oracle.canonicalize(got_offs, tk.cpu().numpy())
    assert np.array_equal(got_keys, ref["keys"]), "bucket contents"
    want = oracle.count(keys, queries)
    for name, (counts, found) in probes.items():
        got_c = counts.cpu().numpy()
        assert np.array_equal(got_c, want), f"{name} counts: {np.count_nonzero(got_c != want)} of {want.size} differ"
        assert np.array_equal(found.cpu().numpy(), (want > 0).astype(np.uint8)), f"{name} found"
    t.free()


SIZES = [0, 1, 2, 63, 64, 65, 4095, 4096, 4097, 3 * 4096 + 17, 65536 + 3]


@pytest.mark.parametrize("build", sorted(BUILDS))
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("P", [1, 16])
def test_uniform_u32_sizes(gpu, n, P, build):
    check_table(gpu, make_keys("uniform", n, np.uint32, 11 + n), P=P, build=build)


@pytest.mark.parametrize("build", sorted(BUILDS))
@pytest.mark.parametrize("kind", ["uniform", "equal", "seq", "swr", "zipf", "extremes"])
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64], ids=["u32", "u64"])
@pytest.mark.parametrize("P", [1, 2, 16])
def test_distributions(gpu, kind, dtype, P, build):
    n = 20000 + 7
    check_table(gpu, make_keys(kind, n, dtype, 5), P=P, build=build)


@pytest.mark.parametrize("build", sorted(BUILDS))
@pytest.mark.parametrize("ratio", [(1, 2), (3, 2), (1, 7), (5, 1)])
@pytest.mark.parametrize("P", [1, 4, 256])
def test_ratios(gpu, ratio, P, build):
    n = 50000 + 1
    check_table(gpu, make_keys("uniform", n, np.uint32, 3), P=P, num=ratio[0], den=ratio[1], build=build)


@pytest.mark.parametrize("build", sorted(BUILDS))
@pytest.mark.parametrize("occ", [16, 64, 256, 1024, 4096])
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64], ids=["u32", "u64"])
@pytest.mark.parametrize("P", [1, 16])
def test_high_occupancy(gpu, occ, dtype, P, build):
    """The duplicate study of Sec. 5.4 in small: the hash range shrunk so
    that about `occ` keys share a bucket (V_p = n_p / occ).  Sorted builds
    then take sub-bins of fewer buckets (about 2^13 keys each), nearly every
    bucket is long and sorted in place, and sorted probes take windows of
    fewer buckets."""
    n = (1 << 20) + 333
    check_table(gpu, make_keys("uniform", n, dtype, 23 + occ), P=P, num=1, den=occ, build=build)


@pytest.mark.parametrize("build", sorted(BUILDS))
@pytest.mark.parametrize("V", [1, 2, 3, 1000, (1 << 20) + 1, 1 << 22])
def test_explicit_bucket_count(gpu, V, build):
    n = 30000
    check_table(gpu, make_keys("uniform", n, np.uint32, 17), V=V, build=build)
    check_table(gpu, make_keys("zipf", n, np.uint64, 17), V=V, build=build)


@pytest.mark.parametrize("build", sorted(BUILDS))
@pytest.mark.parametrize("P", [1, 2, 16, 256])
def test_plain_2p20(gpu, P, build):
    keys, queries, _ = inputs.make_workload("plain_u32_2^20")
    check_table(gpu, keys, P=P, queries=queries, build=build)


@pytest.mark.parametrize("build", sorted(BUILDS))
def test_zipf_u64_small(gpu, build):
    keys, queries, opts = inputs.make_workload("zipf_u64_2^27", n=1 << 18)
    check_table(gpu, keys, P=opts["P"], num=opts["num"], den=opts["den"], queries=queries, build=build)


@pytest.mark.parametrize("build", sorted(BUILDS))
@pytest.mark.parametrize("P, num, den", [(1, 1, 1), (16, 1, 1), (2, 1, 1), (1, 1, 2), (16, 3, 1)])
def test_multi_subbin_tables(gpu, P, num, den, build):
    """Tables of several 2^15-bucket sub-bins per level-1 segment, with ragged
    last sub-bins, so the sorted path's two splits and LDS stages all work."""
    n = (1 << 21) + 12345
    check_table(gpu, make_keys("uniform", n, np.uint32, 77), P=P, num=num, den=den, build=build)


def test_wide_segment_uses_global_counters(gpu):
    """All keys equal with P = 16 and table ratio 24: the average partition
    is small enough for partition segments, but the one non-empty partition
    gets 24 * 2^20 buckets, more than 1024 sub-bins of 2^14, so the sorted
    build folds its tail into one wide sub-bin that counts in global memory.
    Checked against the oracle like every other case."""
    n = 1 << 20
    check_table(gpu, make_keys("equal", n, np.uint32, 0), P=16, num=24, den=1, build="sorted")


def test_repeat_is_deterministic(gpu):
    import torch

    keys = make_keys("swr", 100003, np.uint32, 9)
    kd = to_dev(keys)
    outs = []
    for _ in range(3):
        t = gpu.hg_build(kd, P=16, flags=2)
        po, bb, offs, tk = t.export()
        torch.cuda.synchronize()
        o = offs.cpu().numpy()
        outs.append((po.cpu().numpy(), o, oracle.canonicalize(o, tk.cpu().numpy())))
        t.free()
    for a in outs[1:]:
        for x, y in zip(outs[0], a):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64], ids=["u32", "u64"])
def test_hash_bucket(gpu, dtype):
    import torch

    top = int(np.iinfo(dtype).max)
    edge = np.array([0, 1, 2, top, top - 1, top // 2, top // 2 + 1, 0x80000000, 0x7FFFFFFF], dtype=dtype)
    keys = np.concatenate([edge, make_keys("uniform", 100000, dtype, 23)])
    kd = to_dev(keys)
    divisors = [1, 2, 3, 5, 7, 641, 65535, 65536, 65537, (1 << 24) - 3, (1 << 31) - 1, 1 << 31,
                (1 << 31) + 1, 3 << 30, (1 << 32) - 2, (1 << 32) - 1, 2654435761, 4294967291]
    for V in divisors:
        h, b = gpu.hg_hash_bucket(kd, V)
        torch.cuda.synchronize()
        rh, rb = oracle.hash_bucket(keys, V)
        assert np.array_equal(h.cpu().numpy(), rh), f"hash, V={V}"
        assert np.array_equal(b.cpu().numpy(), rb), f"bucket, V={V}"


@pytest.mark.parametrize("n", [0, 1, 4095, 4097, 100003])
@pytest.mark.parametrize("P", [1, 2, 16, 256])
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64], ids=["u32", "u64"])
def test_bin_partition(gpu, n, P, dtype):
    import torch

    keys = make_keys("uniform", n, dtype, 31 + n)
    out, po = gpu.hg_bin_partition(to_dev(keys), P)
    torch.cuda.synchronize()
    rpo, rkeys = oracle.bin_partition(keys, P)
    got_po = po.cpu().numpy()
    assert np.array_equal(got_po, rpo)
    assert np.array_equal(oracle.canonicalize(got_po, out.cpu().numpy()), rkeys)


def test_empty_table_counts_zero(gpu):
    import torch

    keys = np.empty(0, np.uint32)
    queries = make_keys("uniform", 5000, np.uint32, 1)
    check_table(gpu, keys, P=1, queries=queries)
    check_table(gpu, keys, P=16, queries=queries)
    t = gpu.hg_build(to_dev(keys))
    c = gpu.hg_count(t, to_dev(np.empty(0, np.uint32)))
    torch.cuda.synchronize()
    assert c.numel() == 0
    t.free()


@pytest.mark.parametrize("P", [1, 16])
def test_subbin_with_more_than_u16_keys(gpu, P):
    """One bucket holding 70000 copies of a key: its sub-bin has more keys than
    16-bit LDS counters can hold, so the sorted build counts it in global
    memory.  The probe still answers every query exactly."""
    keys = np.concatenate([np.full(70000, 12345, np.uint32), make_keys("uniform", 30000, np.uint32, 3)])
    check_table(gpu, keys, P=P, build="sorted")


LONG_CASES = {
    # few distinct keys per long bucket: rewritten as ascending runs
    "zipf_runs": lambda: (inputs.zipf_u64(1 << 18, 1000, 41), 0),
    "one_key_100k": lambda: (np.full(100000, 7, np.uint64), 0),
    # many distinct keys, at most 4096 per bucket: bitonic sort in LDS
    "bitonic_V8": lambda: (make_keys("uniform", 20000, np.uint64, 8), 8),
    # many distinct keys, about 6700 per bucket: bitonic sort in LDS by a
    # workgroup
    "unsorted_V3": lambda: (make_keys("uniform", 20000, np.uint64, 9), 3),
    # many distinct keys, sorted by a workgroup in registers: about 3100
    # keys per bucket (four per thread) and about 12000 (sixteen per thread
    # for 32-bit keys; more than 64 KiB of 64-bit keys: unsorted)
    "wg_sort_V8": lambda: (make_keys("uniform", 25000, np.uint64, 15), 8),
    "wg_sort_V3": lambda: (make_keys("uniform", 36000, np.uint64, 16), 3),
    # many distinct keys in buckets of about 20000 (more than the LDS sort
    # holds, fewer than a chunked bucket): left unsorted, scanned
    "unsorted_V2": lambda: (make_keys("uniform", 40000, np.uint64, 11), 2),
    # many distinct keys, sorted by one wave in registers: about 105, 700
    # and 1750 keys per bucket (1750: 32 keys per lane for 32-bit keys, a
    # workgroup's LDS sort for 64-bit ones)
    "wave_sort_V10000": lambda: (make_keys("uniform", 1 << 20, np.uint64, 12), 10000),
    "wave_sort_V1500": lambda: (make_keys("uniform", 1 << 20, np.uint64, 13), 1500),
    "wave_sort_V600": lambda: (make_keys("uniform", 1 << 20, np.uint64, 14), 600),
    "mixed_70x100_V2": lambda: (np.repeat(np.arange(70, dtype=np.uint64) * 977, 100), 2),
    # 4096 buckets of about 256 distinct keys: every one overflows the
    # wave's set and moves to the back of the shared long-bucket list, which
    # then holds as many entries as the front
    "many_bitonic_V4096": lambda: (make_keys("uniform", 1 << 20, np.uint64, 10), 4096),
    # 2^14 buckets of about 120 keys with about 3 distinct values each, dealt
    # to the waves of the wave-per-bucket pass (two buckets per wave)
    "many_runs_V16384": lambda: ((np.arange(3 * 16384, dtype=np.uint64) * 2654435761)[
        inputs.uniform_u32(2 * 1000000, 47) % (3 * 16384)], 16384),
    # buckets longer than 2^16 keys, shared by many workgroups in chunks:
    # 12 values in shuffled order over 4 buckets (a few runs per bucket), one
    # value 200000 times, 300 values over 2 buckets (too many to rewrite), and
    # a bucket of exactly 2^16 + 1 keys with two values
    "big_runs_V4": lambda: ((np.arange(12, dtype=np.uint64) * 7919)[inputs.uniform_u32(300000, 44) % 12], 4),
    "big_one_key": lambda: (np.full(200000, 99, np.uint64), 0),
    "big_unsorted_V2": lambda: ((np.arange(300, dtype=np.uint64) * 31)[inputs.uniform_u32(150000, 45) % 300], 2),
    "big_two_chunks_V1": lambda: (np.array([5, 3], np.uint64)[inputs.uniform_u32((1 << 16) + 1, 46) % 2], 1),
}


@pytest.mark.parametrize("build", sorted(BUILDS))
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64], ids=["u32", "u64"])
@pytest.mark.parametrize("case", sorted(LONG_CASES))
def test_long_buckets(gpu, case, dtype, build):
    """Buckets longer than 64 keys: exact counts through both probes, and in
    the raw table every long bucket the build could sort (at most 64 distinct
    keys, or at most 64 KiB of keys) is ascending."""
    import torch

    keys, V = LONG_CASES[case]()
    keys = keys.astype(dtype)
    queries = np.concatenate([keys[:: max(1, keys.size // 5000)], make_keys("uniform", 3000, dtype, 5)])
    check_table(gpu, keys, V=V, queries=queries, build=build)
    t = gpu.hg_build(to_dev(keys), num_buckets=V, flags=BUILDS[build])
    _, _, offs, tk = t.export()
    torch.cuda.synchronize()
    offs, tk = offs.cpu().numpy().astype(np.int64), tk.cpu().numpy()
    for g in np.nonzero(np.diff(offs) > 64)[0]:
        seg = tk[offs[g]:offs[g + 1]]
        if np.unique(seg).size <= 64 or seg.size <= 65536 // np.dtype(dtype).itemsize:
            assert np.all(seg[1:] >= seg[:-1]), f"long bucket {g} of {seg.size} keys is not sorted"
    t.free()


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64], ids=["u32", "u64"])
@pytest.mark.parametrize("P", [1, 16])
def test_probe_windows_around_the_lds_key_capacity(gpu, dtype, P):
    """Two keys per bucket (V = n/2) and twelve heavy keys of 500 to 15000
    copies each: a probe window sized for about 4096 (u64) or 8192 (u32)
    keys then holds up to several times that, so windows fall on both sides
    of what fits LDS beside their offsets (up to 8192 u64 or 14340 u32 keys
    when the window has fewer buckets than the largest), and their counts
    come from LDS, from global memory and from the run tables."""
    base = make_keys("uniform", 1 << 20, dtype, 61)
    heavy = make_keys("uniform", 12, dtype, 62)
    copies = np.linspace(500, 15000, 12).astype(np.int64)
    keys = np.concatenate([base, np.repeat(heavy, copies)])
    keys = keys[inputs.uniform_u32(keys.size, 63).argsort(kind="stable")]
    queries = np.concatenate([np.repeat(heavy, 50), base[::40], make_keys("uniform", 20000, dtype, 64)])
    check_table(gpu, keys, P=P, num=1, den=2, queries=queries)


def keys_in_buckets(dtype, V, buckets, per_bucket, seed):
    """per_bucket distinct keys for each of the given buckets of a plain
    table with V buckets (chosen from seeded candidates by the oracle's
    hash), as one array per bucket."""
    gen = inputs.uniform_u32 if dtype == np.uint32 else inputs.uniform_u64
    cand = np.unique(gen(max(2 * per_bucket, 20) * V, seed))
    _, b = oracle.hash_bucket(cand, V)
    out = [cand[b == g][:per_bucket] for g in buckets]
    assert all(x.size == per_bucket for x in out)
    return out


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64], ids=["u32", "u64"])
@pytest.mark.parametrize("case", ["over_32_long", "staged_with_unsorted"])
def test_probe_window_with_many_or_unsorted_long_buckets(gpu, dtype, case):
    """Plain table, V = 2^17 buckets for 2^18 uniform keys, plus heavy keys
    placed in the first probe window (buckets below 1024).  over_32_long: 40
    long buckets there (more than the window's list holds), so the window
    counts its short buckets from global memory and 8 long buckets have no
    runs.  staged_with_unsorted: a bucket of 100 distinct keys x 50 (left
    unsorted), one of 80 x 20 (sorted, too many keys for runs) and one of
    3 x 3000 (runs); the short buckets are staged in LDS beside them."""
    V = 1 << 17
    base = make_keys("uniform", 1 << 18, dtype, 71)
    if case == "over_32_long":
        heavy = np.concatenate(keys_in_buckets(dtype, V, list(range(3, 1000, 24))[:40], 1, 72))
        extra = np.repeat(heavy, 300)
    else:
        a, b, c = keys_in_buckets(dtype, V, [7, 300, 600], 100, 73)
        heavy = np.concatenate([a, b[:80], c[:3]])
        extra = np.concatenate([np.repeat(a, 50), np.repeat(b[:80], 20), np.repeat(c[:3], 3000)])
    keys = np.concatenate([base, extra])
    keys = keys[inputs.uniform_u32(keys.size, 74).argsort(kind="stable")]
    queries = np.concatenate([np.repeat(heavy, 20), base[::10], make_keys("uniform", 20000, dtype, 75)])
    check_table(gpu, keys, V=V, queries=queries)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64], ids=["u32", "u64"])
@pytest.mark.parametrize("values, copies", [
    ([100, 200, 300], [3000, 2000, 1000]),  # three runs: first, middle and last value
    ([100, 300], [2500, 2500]),             # two runs: either end equals the query
    ([100], [5000]),                        # one run: both ends equal
])
def test_sorted_long_bucket_counts_from_its_ends(gpu, dtype, values, copies):
    """One bucket (V = 1) of a few values, rewritten as ascending runs.
    Queries equal to its first, last and middle values, below, above and
    between them: the count in a sorted bucket looks at both ends first and
    searches only when it must, in LDS (sorted probe) and in global memory
    (direct probe)."""
    keys = np.repeat(np.array(values, dtype), copies)
    keys = keys[inputs.uniform_u32(keys.size, 81).argsort(kind="stable")]
    queries = np.repeat(np.array([100, 200, 300, 50, 400, 150, 250, 0], dtype), 7)
    check_table(gpu, keys, V=1, queries=queries)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64], ids=["u32", "u64"])
@pytest.mark.parametrize("shift", [0, 1, 3])
def test_sorted_probe_output_alignment(gpu, dtype, shift):
    """The last gather of the sorted probe stores whole vectors when the
    output allows it; an output that starts `shift` u32 elements into an
    allocation (not 16-byte aligned) takes the element-wise stores.  Both
    give the oracle's counts."""
    import torch

    keys = make_keys("uniform", 50000, dtype, 21)
    queries = inputs.queries_hit50(keys, 3 * 4096 * 4 + 1234, 0xA11)
    t = gpu.hg_build(to_dev(keys), P=16)
    buf = torch.full((queries.size + shift,), 0xFFFFFFFF, dtype=torch.uint32, device="cuda")
    out = buf[shift:]
    gpu.hg_count(t, to_dev(queries), out=out, flags=PROBES["sorted"])
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle.count(keys, queries))
    assert np.all(buf[:shift].cpu().numpy() == 0xFFFFFFFF)
    t.free()


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64], ids=["u32", "u64"])
@pytest.mark.parametrize("P", [1, 16])
def test_heavy_subbins_shared_by_workgroups(gpu, dtype, P):
    """Three keys with 300000, 150000 and 70000 copies among 400000 uniform
    keys: their sub-bins hold more than 65535 keys, so they are built by
    many workgroups (chunk histograms, reserved ranges), and their queries
    are probed by many workgroups too.  Checked against the oracle."""
    heavy = np.array([0xABCDEF01, 17, 0xFFFFFFFF], dtype=dtype)
    keys = np.concatenate([np.repeat(heavy, [300000, 150000, 70000]), make_keys("uniform", 400000, dtype, 61)])
    keys = keys[np.argsort(inputs.uniform_u32(keys.size, 62), kind="stable")]  # interleave
    queries = np.concatenate([np.repeat(heavy, 50000), make_keys("uniform", 20000, dtype, 63), keys[:30000]])
    check_table(gpu, keys, P=P, queries=queries, build="sorted")


@pytest.mark.parametrize("copies, width", [(64, 1), (65, 4)])
def test_probe_count_width_at_the_long_bucket_threshold(gpu, copies, width):
    """A key repeated `copies` times in a table whose other keys avoid its
    bucket: with 64 copies no bucket is long, the table reports 1-byte probe
    counts and the count 64 passes through them exactly; with 65 the bucket
    is long and the counts are 4 bytes wide.  Both probes give the oracle's
    counts."""
    n = 1 << 20
    x = np.uint32(0x1234567)
    _, bx = oracle.hash_bucket(np.array([x], np.uint32), n)
    base = make_keys("uniform", n + 4096, np.uint32, 91)
    _, b = oracle.hash_bucket(base, n)
    base = base[(b != bx[0]) & (base != x)][: n - copies]
    keys = np.concatenate([base, np.full(copies, x, np.uint32)])
    keys = keys[inputs.uniform_u32(keys.size, 92).argsort(kind="stable")]
    ref = oracle.build_table(keys, V=n)
    assert int(np.diff(ref["offsets"].astype(np.int64)).max()) == copies
    t = gpu.hg_build(to_dev(keys), num_buckets=n, flags=BUILDS["sorted"])
    assert t.info()["probe_count_bytes"] == width
    t.free()
    queries = np.concatenate([np.full(100, x, np.uint32), inputs.queries_hit50(keys, 1 << 20, 93)])
    check_table(gpu, keys, V=n, queries=queries)


def test_trim_pool_keeps_tables_valid(gpu):
    """Trimming the library's pool hands back only memory no table holds."""
    import torch

    keys = make_keys("uniform", 1 << 20, np.uint32, 71)
    a = gpu.hg_build(to_dev(keys))
    b = gpu.hg_build(to_dev(keys[: 1 << 19]))
    b.free()
    torch.cuda.synchronize()
    gpu.hg_trim_pool(0)
    q = inputs.queries_hit50(keys, 5000, 72)
    got = gpu.hg_count(a, to_dev(q)).cpu().numpy()
    assert np.array_equal(got, oracle.count(keys, q))
    a.free()
