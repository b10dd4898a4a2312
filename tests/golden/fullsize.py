"""Digests of the oracle's outputs at the full workload sizes.

The two large workloads (2^28 uint32 keys split into 16 hash-range
partitions; 2^27 uint64 Zipf keys with V = n/2) are too big to keep the
oracle's outputs beside the tests, and too slow to recompute on every GPU
run.  This module reduces a table and its counts to a few hashes that a
GPU run can compare without sorting anything:

  * part_offsets and bucket_base are kept whole (P + 1 values each);
  * offsets and counts: BLAKE2b of their raw little-endian bytes, so they
    must match bit for bit;
  * keys: an order-free multiset hash of the pairs (bucket, key), the sum
    modulo 2^64 of a 64-bit mix of each pair, under two different mixes.
    The order of keys inside a bucket is left open by the method (the
    atomics of Algorithm 1), so the digest must not depend on it; with equal
    offsets, equal sums mean equal bucket contents up to a chance of about
    2^-64 per mix for any accidental difference.

The mixes are the avalanche step of xxHash64 and a second xor-shift-multiply
mix with other odd constants; they are checksum arithmetic only, unrelated to
the table's hash function.

Run as a script, it computes the digests from the CPU oracle (``oracle/``,
all-core build) on the seeded inputs of ``paper_2104_00792_amd.inputs`` and
writes ``fullsize_digests.json`` next to this file:

    python tests/golden/fullsize.py [workload ...]

Nothing else here calls the oracle.
"""

from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DIGESTS = os.path.join(HERE, "fullsize_digests.json")
WORKLOADS = ("p16_u32_2^28", "zipf_u64_2^27", "zipf_u32_2^28")
_CHUNK = 1 << 24

_XXH_P2 = np.uint64(0xC2B2AE3D27D4EB4F)
_XXH_P3 = np.uint64(0x165667B19E3779F9)
_MX_A = np.uint64(0x7FB5D329728EA185)
_MX_B = np.uint64(0x81DADEF4BC2DD44D)
_GOLD = np.uint64(0x9E3779B97F4A7C15)


def _xxh_avalanche(z: np.ndarray) -> np.ndarray:
    z ^= z >> np.uint64(33)
    z *= _XXH_P2
    z ^= z >> np.uint64(29)
    z *= _XXH_P3
    z ^= z >> np.uint64(32)
    return z


def _mix2(z: np.ndarray) -> np.ndarray:
    z ^= z >> np.uint64(27)
    z *= _MX_A
    z ^= z >> np.uint64(33)
    z *= _MX_B
    z ^= z >> np.uint64(27)
    return z


def blake(a: np.ndarray) -> str:
    return hashlib.blake2b(np.ascontiguousarray(a).view(np.uint8), digest_size=16).hexdigest()


def bucket_key_multiset(offsets: np.ndarray, keys: np.ndarray) -> list[str]:
    """Two order-free hashes of the multiset {(g, key)}: key at position i
    lies in bucket g with offsets[g] <= i < offsets[g+1]."""
    offsets = np.asarray(offsets, dtype=np.int64)
    B = offsets.size - 1
    s1 = np.uint64(0)
    s2 = np.uint64(0)
    with np.errstate(over="ignore"):
        for b0 in range(0, B, _CHUNK):
            b1 = min(B, b0 + _CHUNK)
            lo, hi = int(offsets[b0]), int(offsets[b1])
            g = np.repeat(np.arange(b0, b1, dtype=np.uint64), np.diff(offsets[b0:b1 + 1]))
            k = keys[lo:hi].astype(np.uint64)
            z = k ^ (g * _GOLD)
            s1 += _xxh_avalanche(z.copy()).sum(dtype=np.uint64)
            s2 += _mix2(z + g).sum(dtype=np.uint64)
    return [f"{int(s1):016x}", f"{int(s2):016x}"]


def digest(part_offsets, bucket_base, offsets, keys, counts) -> dict:
    """Digest of one built table and the counts of its workload's queries."""
    offsets = np.ascontiguousarray(offsets, dtype=np.uint32)
    return {
        "part_offsets": [int(x) for x in np.asarray(part_offsets)],
        "bucket_base": [int(x) for x in np.asarray(bucket_base)],
        "num_buckets": int(offsets.size - 1),
        "offsets_blake2b": blake(offsets),
        "bucket_keys_multiset": bucket_key_multiset(offsets, np.asarray(keys)),
        "counts_blake2b": blake(np.ascontiguousarray(counts, dtype=np.uint32)),
    }


def compare(got: dict, want: dict) -> dict:
    """Field-by-field equality of two digests (True where equal)."""
    return {k: got.get(k) == v for k, v in want.items() if k != "inputs"}


def load() -> dict:
    with open(DIGESTS) as f:
        return json.load(f)


def inputs_id(name: str, n: int, q: int) -> dict:
    from paper_2104_00792_amd import inputs

    w = inputs.WORKLOADS[name]
    return {"n": n, "q": q, "key_seed": inputs.KEY_SEED + w["idx"], "query_seed": inputs.QUERY_SEED + w["idx"],
            "P": w["P"], "num": w["num"], "den": w["den"]}


def oracle_digest(name: str) -> dict:
    """The oracle's table and counts of workload `name` at its full size."""
    root = os.path.dirname(os.path.dirname(HERE))
    if root not in sys.path:
        sys.path.insert(0, root)
    import oracle
    from paper_2104_00792_amd import inputs

    t0 = time.time()
    keys, queries, opts = inputs.make_workload(name)
    print(f"[{name}] inputs {time.time() - t0:.0f} s", flush=True)
    with oracle.all_cores():
        ref = oracle.build_table(keys, P=opts["P"], num=opts["num"], den=opts["den"])
        print(f"[{name}] oracle build {time.time() - t0:.0f} s", flush=True)
        counts = oracle.count(keys, queries)
        print(f"[{name}] oracle count {time.time() - t0:.0f} s", flush=True)
    d = digest(ref["part_offsets"], ref["bucket_base"], ref["offsets"], ref["keys"], counts)
    d["inputs"] = inputs_id(name, keys.size, queries.size)
    print(f"[{name}] digest {time.time() - t0:.0f} s", flush=True)
    return d


def main(names):
    out = load() if os.path.exists(DIGESTS) else {}
    for name in names:
        out[name] = oracle_digest(name)
        with open(DIGESTS, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or list(WORKLOADS))
