"""Pins of the CPU oracle to things other than itself.

* fmix32: the published MurmurHash3_x86_32 vectors (golden file) and a library
  MurmurHash3 (scikit-learn's murmurhash3_32, called, never read), both through
  a MurmurHash3_x86_32 built here around the oracle's finalizer; plus a round
  trip through an inverse derived from the mathematics.
* fmix64: the published SMHasher verification value of MurmurHash3_x64_128,
  computed through a MurmurHash3_x64_128 built here around the oracle's 64-bit
  finalizer (the x86_32 verification value checks the procedure); plus the
  inverse round trip.
* Bucket map (Algorithm 1, first loop): every bucket equals the hash modulo V
  in Python integers, for 32- and 64-bit hashes and divisors at the edges of
  the 32-bit range.
* CSR build (Algorithm 1, CSR of Sec. 3.1, Algorithm 2 Phase 2): brute force
  from the definition on tiny inputs, invariants at moderate size, the V = 1
  special case (the table is sort(A)).
* Counts (Sec. 3.3 querying, Sec. 5.4 duplicate counting): brute force,
  all-equal keys, the paper's sequential keys {1..n}, and the identity
  sum over A of count(A_i) = sum of squared multiplicities.
* Planted mistakes: each test in the last block compiles a copy of the
  oracle with one plausible error and checks that some pin above fails.
"""

import json
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2104_00792_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
M32 = (1 << 32) - 1
M64 = (1 << 64) - 1


# ----------------------------------------------------------- helpers
def rotl32(x, r):
    return ((x << r) | (x >> (32 - r))) & M32


def murmur3_x86_32(data: bytes, seed: int) -> int:
    """MurmurHash3_x86_32 (Appleby), body and tail written here, finalizer
    taken from the oracle."""
    c1, c2 = 0xCC9E2D51, 0x1B873593
    h = seed & M32
    nblocks = len(data) // 4
    for i in range(nblocks):
        k = int.from_bytes(data[4 * i:4 * i + 4], "little")
        k = (k * c1) & M32
        k = rotl32(k, 15)
        k = (k * c2) & M32
        h ^= k
        h = rotl32(h, 13)
        h = (h * 5 + 0xE6546B64) & M32
    tail = data[4 * nblocks:]
    k = 0
    for j in reversed(range(len(tail))):
        k = (k << 8) | tail[j]
    if tail:
        k = (k * c1) & M32
        k = rotl32(k, 15)
        k = (k * c2) & M32
        h ^= k
    h ^= len(data)
    return oracle.fmix32(h)


def rotl64(x, r):
    return ((x << r) | (x >> (64 - r))) & M64


def murmur3_x64_128(data: bytes, seed: int) -> bytes:
    """MurmurHash3_x64_128 (Appleby): body, tail and the final mixing of the
    two halves written here, the 64-bit finalizer taken from the oracle.
    Returns the 16-byte digest (h1 then h2, little-endian)."""
    c1, c2 = 0x87C37B91114253D5, 0x4CF5AD432745937F
    h1 = h2 = seed & M32
    nblocks = len(data) // 16
    for i in range(nblocks):
        k1 = int.from_bytes(data[16 * i:16 * i + 8], "little")
        k2 = int.from_bytes(data[16 * i + 8:16 * i + 16], "little")
        k1 = rotl64((k1 * c1) & M64, 31)
        h1 ^= (k1 * c2) & M64
        h1 = (rotl64(h1, 27) + h2) & M64
        h1 = (h1 * 5 + 0x52DCE729) & M64
        k2 = rotl64((k2 * c2) & M64, 33)
        h2 ^= (k2 * c1) & M64
        h2 = (rotl64(h2, 31) + h1) & M64
        h2 = (h2 * 5 + 0x38495AB5) & M64
    tail = data[16 * nblocks:]
    k1 = int.from_bytes(tail[:8], "little")
    k2 = int.from_bytes(tail[8:], "little")
    if len(tail) > 8:
        h2 ^= (rotl64((k2 * c2) & M64, 33) * c1) & M64
    if tail:
        h1 ^= (rotl64((k1 * c1) & M64, 31) * c2) & M64
    h1 ^= len(data)
    h2 ^= len(data)
    h1 = (h1 + h2) & M64
    h2 = (h2 + h1) & M64
    h1 = oracle.fmix64(h1)
    h2 = oracle.fmix64(h2)
    h1 = (h1 + h2) & M64
    h2 = (h2 + h1) & M64
    return h1.to_bytes(8, "little") + h2.to_bytes(8, "little")


def smhasher_verification(digest) -> int:
    """SMHasher's verification value of a hash function `digest(data, seed)
    -> bytes`: the keys {}, {0}, {0,1}, ... of 0..255 bytes hashed with seed
    256 - length, their digests concatenated and hashed with seed 0; the
    first four bytes of that digest, little-endian."""
    key = bytes(range(256))
    cat = b"".join(digest(key[:i], 256 - i) for i in range(256))
    return int.from_bytes(digest(cat, 0)[:4], "little")


def modinv_pow2(c: int, bits: int) -> int:
    """Inverse of an odd c modulo 2^bits by Newton's iteration."""
    m = (1 << bits) - 1
    inv = c
    for _ in range(6):
        inv = (inv * (2 - c * inv)) & m
    assert (inv * c) & m == 1
    return inv


def inv_xorshift(y: np.ndarray, s: int, bits: int) -> np.ndarray:
    """Inverse of x -> x ^ (x >> s): x = y ^ (y >> s) ^ (y >> 2s) ^ ..."""
    x = y.copy()
    sh = s
    while sh < bits:
        x ^= y >> y.dtype.type(sh)
        sh += s
    return x


def fmix32_inverse(y: np.ndarray) -> np.ndarray:
    y = y.astype(np.uint32)
    y = inv_xorshift(y, 16, 32)
    y = y * np.uint32(modinv_pow2(0xC2B2AE35, 32))
    y = inv_xorshift(y, 13, 32)
    y = y * np.uint32(modinv_pow2(0x85EBCA6B, 32))
    return inv_xorshift(y, 16, 32)


def fmix64_inverse(y: np.ndarray) -> np.ndarray:
    y = y.astype(np.uint64)
    y = inv_xorshift(y, 33, 64)
    y = y * np.uint64(modinv_pow2(0xC4CEB9FE1A85EC53, 64))
    y = inv_xorshift(y, 33, 64)
    y = y * np.uint64(modinv_pow2(0xFF51AFD7ED558CCD, 64))
    return inv_xorshift(y, 33, 64)


def oracle_hash(keys: np.ndarray) -> np.ndarray:
    h, _ = oracle.hash_bucket(keys, 1)
    return h


def brute_table(keys, P=1, num=1, den=1, V=0):
    """The CSR straight from its definition, with Python integers."""
    w = 32 if keys.dtype == np.uint32 else 64
    log2P = P.bit_length() - 1
    hs = [int(x) for x in oracle_hash(keys)]
    ps = [(x >> (w - log2P)) if log2P else 0 for x in hs]
    n_p = [ps.count(i) for i in range(P)]
    Vp = [V if (P == 1 and V) else max(1, n_p[i] * num // den) for i in range(P)]
    bb = [sum(Vp[:i]) for i in range(P + 1)]
    g = [bb[p] + h % Vp[p] for h, p in zip(hs, ps)]
    B = bb[P]
    offsets = [sum(1 for x in g if x < b) for b in range(B + 1)]
    canon = []
    for b in range(B):
        canon.extend(sorted(int(k) for k, x in zip(keys, g) if x == b))
    po = [sum(n_p[:i]) for i in range(P + 1)]
    return po, bb, offsets, canon


# -------------------------------------------------------------- the pins
def pin_murmur3_published_vectors():
    with open(os.path.join(GOLDEN, "murmur3_x86_32_vectors.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            m = re.match(r'^"(.*)"\s+(0x[0-9A-Fa-f]+)\s+(0x[0-9A-Fa-f]+)\s*$', line)
            data, seed, want = m.group(1).encode(), int(m.group(2), 16), int(m.group(3), 16)
            assert murmur3_x86_32(data, seed) == want, (data, hex(seed))


def pin_murmur3_against_library():
    from sklearn.utils import murmurhash3_32

    rng = np.random.default_rng(7)
    keys = rng.integers(0, 1 << 32, size=2000, dtype=np.uint64)
    seeds = rng.integers(0, 1 << 32, size=2000, dtype=np.uint64)
    for k, s in zip(keys.tolist(), seeds.tolist()):
        # murmurhash3_32 of an int hashes its 4 little-endian bytes
        ref = murmurhash3_32(int(np.int32(np.uint32(k))), seed=int(s), positive=True)
        assert murmur3_x86_32(int(k).to_bytes(4, "little"), s) == ref, (k, s)


def pin_smhasher_verification_values():
    """fmix64's constants through the published verification value of
    MurmurHash3_x64_128; the x86_32 value checks the procedure."""
    impl = {"MurmurHash3_x86_32": lambda d, s: murmur3_x86_32(d, s).to_bytes(4, "little"),
            "MurmurHash3_x64_128": murmur3_x64_128}
    seen = set()
    with open(os.path.join(GOLDEN, "smhasher_verification.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, bits, want = line.split()
            got = smhasher_verification(impl[name])
            assert len(impl[name](b"", 0)) * 8 == int(bits), name
            assert got == int(want, 16), (name, hex(got))
            seen.add(name)
    assert seen == set(impl)


def pin_bucket_map():
    """The bucket of Algorithm 1 is the hash modulo V: each bucket the
    oracle reports equals the Python-integer remainder of the full hash
    (all 64 bits of a 64-bit hash), for divisors at the edges of the 32-bit
    range and random ones, on 32- and 64-bit keys."""
    rng = np.random.default_rng(11)
    divisors = [1, 2, 3, 7, (1 << 16) + 1, (1 << 31) - 1, 1 << 31, (1 << 31) + 1, (1 << 32) - 2, (1 << 32) - 1]
    divisors += [int(x) for x in rng.integers(1, 1 << 32, size=6, dtype=np.uint64)]
    for dt, fmix in ((np.uint32, oracle.fmix32), (np.uint64, oracle.fmix64)):
        top = (1 << 32) if dt == np.uint32 else (1 << 64)
        keys = np.concatenate([np.array([0, 1, top - 1, top // 2], dtype=np.uint64),
                               rng.integers(0, 1 << 63, size=3000, dtype=np.uint64) * np.uint64(2) +
                               rng.integers(0, 2, size=3000, dtype=np.uint64)]).astype(dt)
        want_h = [fmix(int(k)) for k in keys.tolist()]
        for V in divisors:
            h, b = oracle.hash_bucket(keys, V)
            assert h.tolist() == want_h, (dt, V)
            assert b.tolist() == [x % V for x in want_h], (dt, V)


def pin_fmix32_inverse_round_trip():
    rng = np.random.default_rng(1)
    x = np.concatenate([np.arange(1 << 16, dtype=np.uint32),
                        np.array([M32, M32 - 1, 1 << 31], dtype=np.uint32),
                        rng.integers(0, 1 << 32, size=1 << 18, dtype=np.uint64).astype(np.uint32)])
    h = oracle_hash(x).astype(np.uint32)
    assert np.array_equal(fmix32_inverse(h), x)


def pin_fmix64_inverse_round_trip():
    rng = np.random.default_rng(2)
    x = np.concatenate([np.arange(1 << 12, dtype=np.uint64), np.array([M64, M64 - 1, 1 << 63], dtype=np.uint64),
                        rng.integers(0, 1 << 63, size=1 << 16, dtype=np.uint64) * np.uint64(2) + np.uint64(1)])
    h = oracle_hash(x)
    assert np.array_equal(fmix64_inverse(h), x)


def pin_csr_brute_force():
    rng = np.random.default_rng(3)
    cases = [(0, 1, 1, 1, 0), (1, 1, 1, 1, 0), (7, 1, 1, 1, 0), (40, 1, 1, 1, 5), (120, 1, 1, 2, 0),
             (120, 2, 1, 1, 0), (150, 4, 3, 2, 0), (200, 8, 1, 3, 0), (90, 16, 1, 1, 0), (64, 1, 1, 1, 1)]
    for n, P, num, den, V in cases:
        for dt in (np.uint32, np.uint64):
            keys = rng.integers(0, 40, size=n).astype(dt) * dt(2654435761)  # duplicates included
            po, bb, offs, canon = brute_table(keys, P, num, den, V)
            t = oracle.build_table(keys, P=P, num=num, den=den, V=V)
            assert t["part_offsets"].tolist() == po, (n, P)
            assert t["bucket_base"].tolist() == bb, (n, P)
            assert t["offsets"].tolist() == offs, (n, P)
            assert [int(k) for k in t["keys"]] == canon, (n, P)


def pin_csr_invariants():
    rng = np.random.default_rng(4)
    for P, num, den in [(1, 1, 1), (16, 1, 1), (4, 1, 2), (2, 5, 3)]:
        n = 1 << 14
        keys = inputs.uniform_u32(n, 100 + P)
        keys[: n // 8] = keys[n // 8: n // 4]  # some duplicates
        t = oracle.build_table(keys, P=P, num=num, den=den)
        offs, out, po, bb = t["offsets"].astype(np.int64), t["keys"], t["part_offsets"], t["bucket_base"]
        h = oracle_hash(keys)
        log2P = P.bit_length() - 1
        p = (h >> np.uint64(32 - log2P)).astype(np.int64) if log2P else np.zeros(n, np.int64)
        n_p = np.bincount(p, minlength=P)
        Vp = np.maximum(1, n_p * num // den)
        assert np.array_equal(po, np.concatenate([[0], np.cumsum(n_p)]))
        assert np.array_equal(bb, np.concatenate([[0], np.cumsum(Vp)]))
        g = bb[p].astype(np.int64) + (h % Vp[p].astype(np.uint64)).astype(np.int64)
        B = int(bb[-1])
        assert offs[0] == 0 and offs[-1] == n and np.all(np.diff(offs) >= 0)
        assert np.array_equal(np.diff(offs), np.bincount(g, minlength=B))
        assert np.array_equal(np.sort(out), np.sort(keys))
        # every key sits in the segment of its own bucket, ascending inside it
        hout = oracle_hash(out)
        pout = (hout >> np.uint64(32 - log2P)).astype(np.int64) if log2P else np.zeros(n, np.int64)
        gout = bb[pout].astype(np.int64) + (hout % Vp[pout].astype(np.uint64)).astype(np.int64)
        assert np.array_equal(gout, np.repeat(np.arange(B), np.diff(offs)))
        same = gout[1:] == gout[:-1]
        assert np.all(out[1:][same] >= out[:-1][same])
    # V = 1: the one bucket is sort(A)
    keys = rng.integers(0, 1 << 32, size=5000, dtype=np.uint64).astype(np.uint32)
    t = oracle.build_table(keys, V=1)
    assert t["offsets"].tolist() == [0, 5000]
    assert np.array_equal(t["keys"], np.sort(keys))


def pin_counts():
    rng = np.random.default_rng(5)
    keys = rng.integers(0, 50, size=300).astype(np.uint32)
    qs = np.arange(0, 60, dtype=np.uint32)
    want = [sum(1 for k in keys.tolist() if k == q) for q in qs.tolist()]
    assert oracle.count(keys, qs).tolist() == want
    # probing A with itself: sum of counts is the sum of squared multiplicities
    big = inputs.sample_with_replacement(1 << 15, 9)
    _, mult = np.unique(big, return_counts=True)
    assert int(oracle.count(big, big).astype(np.int64).sum()) == int((mult.astype(np.int64) ** 2).sum())
    # all keys equal
    eq = np.full(1000, 77, np.uint64)
    assert oracle.count(eq, np.array([77, 78], np.uint64)).tolist() == [1000, 0]
    # the paper's sequential keys {1..n}: 1 inside, 0 outside
    seq = inputs.sequential(4096)
    q = np.array([0, 1, 2, 4096, 4097, 0xFFFFFFFF], np.uint32)
    assert oracle.count(seq, q).tolist() == [0, 1, 1, 1, 0, 0]
    # the CSR answers the same: scan the query's bucket segment
    t = oracle.build_table(big, P=16)
    h = oracle_hash(qs)
    p = (h >> np.uint64(28)).astype(np.int64)
    Vp = np.diff(t["bucket_base"]).astype(np.uint64)
    g = t["bucket_base"][p].astype(np.int64) + (h % Vp[p]).astype(np.int64)
    via_csr = [int(np.count_nonzero(t["keys"][t["offsets"][x]:t["offsets"][x + 1]] == q)) for x, q in zip(g, qs)]
    assert via_csr == oracle.count(big, qs).tolist()


def pin_partition():
    for P in (1, 2, 16, 256):
        for dt in (np.uint32, np.uint64):
            keys = inputs.uniform_u64(20000, P).astype(dt)
            po, out = oracle.bin_partition(keys, P)
            log2P = P.bit_length() - 1
            w = 32 if dt == np.uint32 else 64
            h = oracle_hash(keys)
            p = (h >> np.uint64(w - log2P)).astype(np.int64) if log2P else np.zeros(keys.size, np.int64)
            assert np.array_equal(po, np.concatenate([[0], np.cumsum(np.bincount(p, minlength=P))]))
            assert po[-1] == keys.size
            hout = oracle_hash(out)
            pout = (hout >> np.uint64(w - log2P)).astype(np.int64) if log2P else np.zeros(keys.size, np.int64)
            assert np.array_equal(pout, np.repeat(np.arange(P), np.diff(po.astype(np.int64))))
            if P == 1:
                assert np.array_equal(out, np.sort(keys))


def pin_balanced_worked_example():
    """The hand-worked example of tests/golden/balanced_split_example.txt."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "balanced_split_example.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    HR = int(rows[0][1])
    bins = int(rows[1][1])
    H = np.array([int(x) for x in rows[2][1:]], dtype=np.uint32)
    keys = fmix32_inverse(H)  # hash(key) = H < HR, so hash mod HR = H
    for r in rows[3:]:
        P = int(r[1])
        i = r.index("part_offsets")
        want_splits = [int(x) for x in r[3:i]]
        want_po = [int(x) for x in r[i + 1:]]
        po, splits, out = oracle.bin_partition_balanced(keys, P, HR, bins)
        assert splits.tolist() == want_splits, (P, splits)
        assert po.tolist() == want_po, (P, po)
        hout = oracle_hash(out)
        for d in range(P):
            assert sorted(hout[po[d]:po[d + 1]].tolist()) == sorted(
                int(h) for h in H if want_splits[d] <= int(h) // 10 < want_splits[d + 1])


def pin_balanced_split_definition():
    """Splits, grouping and balance checked against the definition by brute
    force: every boundary by a linear scan of the prefix sums, every key's
    partition from its own bin."""
    rng_keys = [inputs.uniform_u32(30000, 41), inputs.sample_with_replacement(30000, 42),
                inputs.zipf_u64(30000, 1 << 10, 43)]
    for keys in rng_keys:
        for P, HR, nb in [(1, 1 << 16, 0), (2, 1000, 0), (7, 1 << 20, 0), (16, 12345, 100), (256, 1 << 31, 0),
                          (5, 1, 0), (3, 50000, 1)]:
            po, splits, out = oracle.bin_partition_balanced(keys, P, HR, nb)
            want_bins = nb or min(1 << 14, int(np.ceil(np.sqrt(HR))))
            while want_bins * want_bins < HR and not nb and want_bins < (1 << 14):
                want_bins += 1
            bs = -(-HR // want_bins)
            nbins = -(-HR // bs)
            b = (oracle_hash(keys) % np.uint64(HR)).astype(np.int64) // bs
            cnt = np.bincount(b, minlength=nbins)
            off = np.concatenate([[0], np.cumsum(cnt)])
            n = keys.size
            assert splits[0] == 0 and splits[P] == nbins
            for d in range(1, P):
                target = n * d // P
                first = next(x for x in range(nbins + 1) if off[x] >= target)
                assert splits[d] == first, (P, HR, d)
            bo = (oracle_hash(out) % np.uint64(HR)).astype(np.int64) // bs
            for d in range(P):
                seg = bo[po[d]:po[d + 1]]
                assert np.all((seg >= splits[d]) & (seg < max(splits[d + 1], splits[d]))) or seg.size == 0
                assert po[d + 1] - po[d] == cnt[splits[d]:splits[d + 1]].sum()
            assert po[P] == n
            assert np.array_equal(np.sort(out), np.sort(keys))
            # Balance: the first d partitions hold at least their share and
            # at most one bin more.
            for d in range(1, P):
                assert n * d // P <= po[d] <= n * d // P + cnt.max()


def pin_build_like():
    """The query set's HashGraph (Sec. 3.3) against the table build: built
    from the table's own keys it is that table; for other queries, every
    query that is a table key sits in the bucket where the table holds it."""
    for dt in (np.uint32, np.uint64):
        keys = inputs.uniform_u64(6000, 71).astype(dt)
        for P, num, den, V in [(1, 1, 1, 0), (4, 1, 1, 0), (16, 1, 2, 0), (1, 1, 1, 777)]:
            t = oracle.build_table(keys, P, num, den, V)
            same = oracle.build_like(keys, keys, P, num, den, V)
            for f in ("part_offsets", "bucket_base", "offsets", "keys"):
                assert np.array_equal(same[f], t[f]), (P, f)
            queries = inputs.queries_hit50(keys, 4000, 72)
            q = oracle.build_like(keys, queries, P, num, den, V)
            assert np.array_equal(q["bucket_base"], t["bucket_base"]) and q["offsets"].size == t["offsets"].size
            assert np.array_equal(np.sort(q["keys"]), np.sort(queries))
            qb = np.repeat(np.arange(q["offsets"].size - 1), np.diff(q["offsets"].astype(np.int64)))
            tb = np.repeat(np.arange(t["offsets"].size - 1), np.diff(t["offsets"].astype(np.int64)))
            where = dict(zip(t["keys"].tolist(), tb.tolist()))
            for key, b in zip(q["keys"].tolist(), qb.tolist()):
                if key in where:
                    assert where[key] == b


PINS = [pin_murmur3_published_vectors, pin_murmur3_against_library, pin_smhasher_verification_values,
        pin_bucket_map, pin_fmix32_inverse_round_trip,
        pin_fmix64_inverse_round_trip, pin_csr_brute_force, pin_csr_invariants, pin_counts, pin_partition,
        pin_balanced_worked_example, pin_balanced_split_definition, pin_build_like]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin()


# ------------------------------------------------------- planted mistakes
ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "hg_oracle.cpp")

MUTANTS = {
    "fmix32_shift": ("h ^= h >> 13;", "h ^= h >> 12;"),
    "fmix32_constant": ("h *= 0x85ebca6bu;", "h *= 0x85ebca6cu;"),
    "fmix64_shift": ("  k ^= k >> 33;\n  k *= 0xff51afd7ed558ccdull;", "  k ^= k >> 31;\n  k *= 0xff51afd7ed558ccdull;"),
    "fmix64_constant": ("k *= 0xc4ceb9fe1a85ec53ull;", "k *= 0xc4ceb9fe1a85ec55ull;"),
    "fmix64_first_constant": ("k *= 0xff51afd7ed558ccdull;", "k *= 0xff51afd7ed558ccfull;"),
    "bucket_map_truncated_hash": ("bucket_out[i] = static_cast<uint32_t>(h % V);",
                                  "bucket_out[i] = static_cast<uint32_t>(h) % static_cast<uint32_t>(V);"),
    "partition_low_bits": ("return static_cast<uint32_t>(h >> (w - log2P));",
                           "return static_cast<uint32_t>(h & ((1ull << log2P) - 1));"),
    "bucket_dropped_hash_bit": ("h[i] % V[p_of[i]]", "(h[i] >> 1) % V[p_of[i]]"),
    "table_size_off_by_one": ("v = n_p[p] * static_cast<uint64_t>(num) / den;",
                              "v = (n_p[p] + 1) * static_cast<uint64_t>(num) / den;"),
    "offsets_inclusive": ("    offsets[g] = static_cast<uint32_t>(run);\n    run += bucket_count[g];",
                          "    run += bucket_count[g];\n    offsets[g] = static_cast<uint32_t>(run);"),
    "count_existence_only": ("counts[j] = static_cast<uint32_t>(r.second - r.first);",
                             "counts[j] = r.second != r.first ? 1u : 0u;"),
    "balanced_search_upper": ("split[d] = static_cast<uint64_t>(std::lower_bound(bin_offset.begin(), ",
                              "split[d] = static_cast<uint64_t>(std::upper_bound(bin_offset.begin(), "),
    "balanced_target_shifted": ("const uint64_t target = n * d / P;", "const uint64_t target = n * (d + 1) / P;"),
    "balanced_bin_size_floor": ("const uint64_t bin_size = (HR + bins_asked - 1) / bins_asked;",
                                "const uint64_t bin_size = HR / bins_asked > 0 ? HR / bins_asked : 1;"),
}


def run_pins_against(lib_path: str) -> list:
    """Names of the pins that fail when the oracle is the build at lib_path."""
    caught = []
    oracle.use_library(lib_path)
    try:
        for pin in PINS:
            try:
                pin()
            except (AssertionError, ValueError):
                caught.append(pin.__name__)
    finally:
        oracle.use_library(None)
    return caught


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(ORACLE_SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mut_src = tmp_path / "hg_oracle_mutant.cpp"
    mut_src.write_text(src.replace(old, new))
    lib = oracle.compile_oracle(str(mut_src), str(tmp_path / "liboracle_mutant.so"))
    # A separate process, so that a mutant that corrupts memory cannot take
    # the test session down with it.
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, PYTHONPATH=root + os.pathsep + os.environ.get("PYTHONPATH", ""))
    res = subprocess.run([sys.executable, os.path.abspath(__file__), lib], capture_output=True, text=True,
                         cwd=root, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    caught = json.loads(res.stdout.strip().splitlines()[-1])
    assert caught, f"no pin catches the planted mistake {name}"


if __name__ == "__main__":
    print(json.dumps(run_pins_against(sys.argv[1])))
