"""CPU checks of the full-size digests (tests/golden/fullsize.py).

The digests stand in for the oracle's outputs at 2^28 and 2^27 keys, so
they must (a) ignore the order of keys inside a bucket, which the method
leaves open, (b) change when any key moves to another bucket or changes
value, when an offset or a count changes, and (c) have been written for
the inputs the workloads draw today.
"""

import importlib.util
import os

import numpy as np

import oracle
from paper_2104_00792_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def _fullsize():
    spec = importlib.util.spec_from_file_location("fullsize", os.path.join(HERE, "golden", "fullsize.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _table(n=20000, V=997):
    keys = inputs.uniform_u32(n, 0xD1)
    ref = oracle.build_table(keys, V=V)
    q = inputs.queries_hit50(keys, n, 0xD2)
    return ref, oracle.count(keys, q)


def test_digest_ignores_order_inside_buckets():
    fs = _fullsize()
    ref, counts = _table()
    d0 = fs.digest(ref["part_offsets"], ref["bucket_base"], ref["offsets"], ref["keys"], counts)
    offs = ref["offsets"].astype(np.int64)
    shuffled = ref["keys"].copy()
    rng = np.random.default_rng(3)
    for g in range(offs.size - 1):
        seg = shuffled[offs[g]:offs[g + 1]]
        rng.shuffle(seg)
    d1 = fs.digest(ref["part_offsets"], ref["bucket_base"], ref["offsets"], shuffled, counts)
    assert d0 == d1


def test_digest_sees_every_kind_of_change():
    fs = _fullsize()
    ref, counts = _table()
    d0 = fs.digest(ref["part_offsets"], ref["bucket_base"], ref["offsets"], ref["keys"], counts)
    offs = ref["offsets"].astype(np.int64)
    # two keys of different buckets swapped (offsets unchanged)
    a = int(offs[10])
    b = int(offs[500])
    assert ref["keys"][a] != ref["keys"][b]
    swapped = ref["keys"].copy()
    swapped[[a, b]] = swapped[[b, a]]
    d = fs.digest(ref["part_offsets"], ref["bucket_base"], ref["offsets"], swapped, counts)
    assert d["bucket_keys_multiset"][0] != d0["bucket_keys_multiset"][0]
    assert d["bucket_keys_multiset"][1] != d0["bucket_keys_multiset"][1]
    # one key value changed
    changed = ref["keys"].copy()
    changed[7] ^= np.uint32(1)
    d = fs.digest(ref["part_offsets"], ref["bucket_base"], ref["offsets"], changed, counts)
    assert d["bucket_keys_multiset"] != d0["bucket_keys_multiset"]
    # a key moved across a bucket boundary by an offset change
    moved = ref["offsets"].copy()
    moved[11] += 1
    d = fs.digest(ref["part_offsets"], ref["bucket_base"], moved, ref["keys"], counts)
    assert d["offsets_blake2b"] != d0["offsets_blake2b"]
    assert d["bucket_keys_multiset"] != d0["bucket_keys_multiset"]
    # one count off by one
    c = counts.copy()
    c[123] += 1
    d = fs.digest(ref["part_offsets"], ref["bucket_base"], ref["offsets"], ref["keys"], c)
    assert d["counts_blake2b"] != d0["counts_blake2b"]
    assert fs.compare(d, d0) == {**{k: True for k in d0}, "counts_blake2b": False}


def test_committed_digests_match_todays_workloads():
    fs = _fullsize()
    stored = fs.load()
    for name in fs.WORKLOADS:
        w = inputs.WORKLOADS[name]
        assert stored[name]["inputs"] == fs.inputs_id(name, w["n"], w["n"]), name
        assert len(stored[name]["part_offsets"]) == w["P"] + 1
        assert stored[name]["part_offsets"][-1] == w["n"]
        assert stored[name]["num_buckets"] == stored[name]["bucket_base"][-1]
