"""Count-balanced split (Algorithm 2, Phases 1 and 2) on the GPU against the
oracle, bit-exact: part_offsets and bin_splits raw, each partition's keys as
a sorted multiset.  Uniform, duplicate-heavy and Zipf keys; 32- and 64-bit;
P from 1 to 256 (not only powers of two); hash ranges from 1 to 2^31; empty
and one-key inputs.  Also: the ranges cut the plain table over the same hash
range at bucket boundaries."""

import numpy as np
import pytest

import oracle
from paper_2104_00792_amd import inputs

pytestmark = pytest.mark.gpu


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def keys_of(kind, n, seed):
    if kind == "uniform32":
        return inputs.uniform_u32(n, seed)
    if kind == "uniform64":
        return inputs.uniform_u64(n, seed)
    if kind == "dup32":
        return inputs.sample_with_replacement(n, seed)
    if kind == "zipf64":
        return inputs.zipf_u64(n, 1 << 12, seed)
    raise ValueError(kind)


CASES = [
    ("uniform32", 0, 4, 1000, 0),
    ("uniform32", 1, 3, 100, 0),
    ("uniform32", 5000, 7, 1 << 16, 0),
    ("uniform32", (1 << 20) + 17, 16, 1 << 20, 0),
    ("uniform32", (1 << 20) + 5, 256, 1 << 28, 0),
    ("uniform32", 300001, 1, 1 << 20, 0),
    ("uniform32", 10000, 4, 1, 0),
    ("uniform32", 77777, 5, (1 << 31) + 3, 16384),
    ("uniform64", 100000, 5, 12345, 100),
    ("dup32", 200000, 3, 1 << 20, 1),
    ("zipf64", 300000, 8, 1 << 18, 0),
]


@pytest.mark.parametrize("kind, n, P, HR, bins", CASES)
def test_balanced_split_matches_oracle(gpu, kind, n, P, HR, bins):
    import torch

    hg = gpu
    keys = keys_of(kind, n, 0xBA1 + n % 97)
    out, po, splits = hg.hg_bin_partition_balanced(to_dev(keys), P, HR, bins)
    torch.cuda.synchronize()
    want_po, want_splits, want_out = oracle.bin_partition_balanced(keys, P, HR, bins)
    got_po, got_splits = po.cpu().numpy(), splits.cpu().numpy()
    assert np.array_equal(got_splits, want_splits), "bin splits"
    assert np.array_equal(got_po, want_po), "partition offsets"
    assert np.array_equal(oracle.canonicalize(got_po, out.cpu().numpy()), want_out), "partition contents"


def test_balanced_ranges_cut_the_plain_table_at_bucket_boundaries(gpu):
    """With hash range HR = V, the partitions are bucket ranges of the plain
    table with V buckets: part_offsets[d] = offsets[min(splits[d] * BinSize, V)]."""
    import torch

    hg = gpu
    n = (1 << 21) + 99
    V = 1 << 21
    bins = 1000
    keys = to_dev(inputs.uniform_u32(n, 0xBA7))
    out, po, splits = hg.hg_bin_partition_balanced(keys, 9, V, bins)
    t = hg.hg_build(keys, P=1, num_buckets=V)
    _, _, offs, tk = t.export()
    torch.cuda.synchronize()
    bs = -(-V // bins)
    cut = np.minimum(splits.cpu().numpy().astype(np.int64) * bs, V)
    offs = offs.cpu().numpy()
    assert np.array_equal(po.cpu().numpy(), offs[cut])
    po_np = po.cpu().numpy()
    tk = tk.cpu().numpy()
    out = out.cpu().numpy()
    for d in range(9):
        assert np.array_equal(np.sort(out[po_np[d]:po_np[d + 1]]), np.sort(tk[offs[cut[d]]:offs[cut[d + 1]]]))
    t.free()
