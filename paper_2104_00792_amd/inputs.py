"""Seeded synthetic workloads for the HashGraph build and probe.

This module holds no hashing, bucketing, partitioning or counting: it only
draws keys and queries.  Both the GPU path and the CPU oracle read the arrays
it returns, so nothing here can make the two agree by sharing arithmetic.

Generator: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), used counter-style: output i of stream
``seed`` is mix(seed + (i + 1) * GAMMA), so any slice can be drawn on its own.

Workload shapes follow the paper's experiment section (Sec. 4.3): keys drawn
uniformly or sequential {1..2^k}, as many queries as keys, table size equal
to the key count (C = 1).  Queries hit an inserted key with probability 1/2.
"""

from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 22

# Seeds of the named workloads: keys and queries of workload c use
# KEY_SEED + c and QUERY_SEED + c.
KEY_SEED = 0x5EED0000
QUERY_SEED = 0x5EED0100


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output mixer (in place on a uint64 array)."""
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs start .. start+count-1 of the SplitMix64 stream ``seed``."""
    out = np.empty(count, np.uint64)
    seed = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    for c0 in range(0, count, _CHUNK):
        c1 = min(count, c0 + _CHUNK)
        idx = np.arange(start + c0 + 1, start + c1 + 1, dtype=np.uint64)
        z = idx * GAMMA
        z += seed
        out[c0:c1] = _mix(z)
    return out


def uniform_u32(n: int, seed: int) -> np.ndarray:
    """n keys uniform over [0, 2^32): the high half of each draw."""
    return (splitmix64(seed, 0, n) >> np.uint64(32)).astype(np.uint32)


def uniform_u64(n: int, seed: int) -> np.ndarray:
    return splitmix64(seed, 0, n)


def sequential(n: int, dtype=np.uint32) -> np.ndarray:
    """The paper's sequential key set {1, ..., n} (Sec. 4.3)."""
    return np.arange(1, n + 1, dtype=dtype)


def sample_with_replacement(n: int, seed: int, dtype=np.uint32) -> np.ndarray:
    """The paper's random key set: n draws with replacement from {1..n}."""
    w = splitmix64(seed, 0, n) >> np.uint64(32)
    return ((w * np.uint64(n)) >> np.uint64(32)).astype(dtype) + dtype(1)


def queries_hit50(keys: np.ndarray, q: int, seed: int) -> np.ndarray:
    """q queries; each is, with probability 1/2, an inserted key chosen
    uniformly by position, else a uniform value of the key width (which can
    hit by chance).  Two draws per query: bit 63 of the first picks hit or
    miss, its low 32 bits pick the position; the second gives the miss value.
    """
    n = keys.size
    dt = keys.dtype
    out = np.empty(q, dt)
    for c0 in range(0, q, _CHUNK):
        c1 = min(q, c0 + _CHUNK)
        w = splitmix64(seed, 2 * c0, 2 * (c1 - c0))
        wa, wb = w[0::2], w[1::2]
        if dt == np.uint32:
            miss = (wb >> np.uint64(32)).astype(np.uint32)
        else:
            miss = wb.copy()
        if n == 0:
            out[c0:c1] = miss
            continue
        hit = (wa >> np.uint64(63)).astype(bool)
        pos = ((wa & np.uint64(0xFFFFFFFF)) * np.uint64(n)) >> np.uint64(32)
        out[c0:c1] = np.where(hit, keys[pos.astype(np.int64)], miss)
    return out


def zipf_ranks(n: int, K: int, seed: int, s: float = 1.0) -> np.ndarray:
    """n ranks in 1..K with P(r) proportional to r^-s (inverse CDF on a
    sequentially summed table; the sampler decides inputs only)."""
    cdf = np.cumsum(1.0 / np.arange(1, K + 1, dtype=np.float64) ** s)
    out = np.empty(n, np.uint64)
    for c0 in range(0, n, _CHUNK):
        c1 = min(n, c0 + _CHUNK)
        w = splitmix64(seed, c0, c1 - c0)
        u = (w >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * cdf[-1]
        r = np.searchsorted(cdf, u, side="right") + 1
        out[c0:c1] = np.minimum(r, K).astype(np.uint64)
    return out


def zipf_u64(n: int, K: int, seed: int, s: float = 1.0) -> np.ndarray:
    """n 64-bit keys, Zipf(s) over K distinct values.  The value of rank r is
    the SplitMix64 mixer of r: a bijection on 64-bit words, so the K ranks give
    K distinct, well spread values."""
    return _mix(zipf_ranks(n, K, seed, s))


def zipf_u32(n: int, K: int, seed: int, s: float = 1.0) -> np.ndarray:
    """n 32-bit keys, Zipf(s) over K ranks: the high half of zipf_u64's value
    of each rank (ranks whose halves coincide merge, which at K = 2^20 draws
    out of 2^32 happens for about a hundred pairs)."""
    return (zipf_u64(n, K, seed, s) >> np.uint64(32)).astype(np.uint32)


# --------------------------------------------------------------------------
# The same streams drawn with torch (CPU or device), bit for bit equal to the
# numpy functions above.  64-bit words are carried as int64 bit patterns:
# products wrap modulo 2^64 and right shifts are made logical by masking.
# --------------------------------------------------------------------------

def _s64(c: int) -> int:
    c &= 0xFFFFFFFFFFFFFFFF
    return c - (1 << 64) if c >= (1 << 63) else c


def _lsr(z, s: int):
    return (z >> s) & ((1 << (64 - s)) - 1)


def _mix_t(z):
    z = z ^ _lsr(z, 30)
    z = z * _s64(0xBF58476D1CE4E5B9)
    z = z ^ _lsr(z, 27)
    z = z * _s64(0x94D049BB133111EB)
    return z ^ _lsr(z, 31)


def splitmix64_t(seed: int, start: int, count: int, device, step: int = 1, offset: int = 0):
    """Outputs start + step*j + offset (j < count) of stream ``seed`` as an
    int64 tensor holding the 64-bit patterns."""
    import torch

    idx = torch.arange(count, dtype=torch.int64, device=device) * step + (start + offset + 1)
    return _mix_t(idx * _s64(int(GAMMA)) + _s64(seed))


def _to_u32(z):
    import torch

    return (_lsr(z, 32)).to(torch.int32).view(torch.uint32)


def uniform_u32_t(n: int, seed: int, device):
    return _to_u32(splitmix64_t(seed, 0, n, device))


def queries_hit50_t(keys, q: int, seed: int, device):
    """Device twin of queries_hit50 (keys: a device tensor)."""
    import torch

    n = keys.numel()
    wa = splitmix64_t(seed, 0, q, device, step=2, offset=0)
    wb = splitmix64_t(seed, 0, q, device, step=2, offset=1)
    if keys.dtype == torch.uint32:
        miss = _to_u32(wb)
    else:
        miss = wb.view(torch.uint64)
    if n == 0:
        return miss
    pos = _lsr((wa & 0xFFFFFFFF) * n, 32)
    hit = wa < 0
    if keys.dtype == torch.uint32:
        picked = keys.view(torch.int32)[pos]
        return torch.where(hit, picked, miss.view(torch.int32)).view(torch.uint32)
    picked = keys.view(torch.int64)[pos]
    return torch.where(hit, picked, miss.view(torch.int64)).view(torch.uint64)


def table_queries_t(table_n: int, table_seed: int, q: int, seed: int, device):
    """queries_hit50_t over the keys uniform_u32_t(table_n, table_seed),
    without drawing that key array: a hit at position p takes key p of the
    table's stream directly (the streams are counter-based)."""
    import torch

    wa = splitmix64_t(seed, 0, q, device, step=2, offset=0)
    wb = splitmix64_t(seed, 0, q, device, step=2, offset=1)
    miss = _to_u32(wb)
    if table_n == 0:
        return miss
    pos = _lsr((wa & 0xFFFFFFFF) * table_n, 32)
    picked = _to_u32(_mix_t((pos + 1) * _s64(int(GAMMA)) + _s64(table_seed)))
    return torch.where(wa < 0, picked.view(torch.int32), miss.view(torch.int32)).view(torch.uint32)


def table_queries(table_n: int, table_seed: int, q: int, seed: int) -> np.ndarray:
    """numpy twin of table_queries_t: queries_hit50(uniform_u32(table_n,
    table_seed), q, seed) without the key array."""
    out = np.empty(q, np.uint32)
    for c0 in range(0, q, _CHUNK):
        c1 = min(q, c0 + _CHUNK)
        w = splitmix64(seed, 2 * c0, 2 * (c1 - c0))
        wa, wb = w[0::2], w[1::2]
        miss = (wb >> np.uint64(32)).astype(np.uint32)
        if table_n == 0:
            out[c0:c1] = miss
            continue
        hit = (wa >> np.uint64(63)).astype(bool)
        pos = ((wa & np.uint64(0xFFFFFFFF)) * np.uint64(table_n)) >> np.uint64(32)
        z = (pos + np.uint64(1)) * GAMMA
        z += np.uint64(table_seed & 0xFFFFFFFFFFFFFFFF)
        picked = (_mix(z) >> np.uint64(32)).astype(np.uint32)
        out[c0:c1] = np.where(hit, picked, miss)
    return out


def zipf_u64_t(n: int, K: int, seed: int, device, s: float = 1.0):
    import torch

    cdf = torch.from_numpy(np.cumsum(1.0 / np.arange(1, K + 1, dtype=np.float64) ** s)).to(device)
    w = splitmix64_t(seed, 0, n, device)
    u = _lsr(w, 11).to(torch.float64) * (2.0 ** -53) * cdf[-1]
    r = torch.clamp(torch.searchsorted(cdf, u, right=True) + 1, max=K)
    return _mix_t(r).view(torch.uint64)


def zipf_u32_t(n: int, K: int, seed: int, device, s: float = 1.0):
    """Device twin of zipf_u32."""
    import torch

    z = zipf_u64_t(n, K, seed, device, s).view(torch.int64)
    return _lsr(z, 32).to(torch.int32).view(torch.uint32)


# --------------------------------------------------------------------------
# Named workloads.  Each returns (keys, queries, build options).
# --------------------------------------------------------------------------

WORKLOADS = {
    # Plain single table, n = 2^20 uint32 uniform, V = n, 2^20 queries.
    "plain_u32_2^20": dict(idx=1, n=1 << 20, kind="u32", P=1, num=1, den=1),
    # One GPU's share of the multi-GPU build: n = 2^28, P = 16, V_p = n_p.
    "p16_u32_2^28": dict(idx=2, n=1 << 28, kind="u32", P=16, num=1, den=1),
    # Duplicate-heavy: 2^27 uint64 Zipf(1.0) over 2^20 values, V = n / 2.
    "zipf_u64_2^27": dict(idx=3, n=1 << 27, kind="zipf64", P=1, num=1, den=2),
    # Plain reference point at the headline size: P = 1, V = n = 2^28.
    "plain_u32_2^28": dict(idx=2, n=1 << 28, kind="u32", P=1, num=1, den=1),
    # Duplicate-heavy 32-bit keys: 2^28 uint32 Zipf(1.0) over 2^20 ranks, V = n / 2.
    "zipf_u32_2^28": dict(idx=4, n=1 << 28, kind="zipf32", P=1, num=1, den=2),
}


def make_workload(name: str, n: int | None = None, q: int | None = None, device=None):
    """Keys, queries and build options of a named workload, optionally at a
    smaller n (same recipe, same seeds).  With ``device`` (a torch device)
    the arrays are drawn there as torch tensors, equal to the numpy ones."""
    w = WORKLOADS[name]
    n = w["n"] if n is None else n
    q = n if q is None else q
    ks, qs = KEY_SEED + w["idx"], QUERY_SEED + w["idx"]
    opts = dict(P=w["P"], num=w["num"], den=w["den"])
    if device is not None:
        if w["kind"] == "u32":
            keys = uniform_u32_t(n, ks, device)
            queries = queries_hit50_t(keys, q, qs, device)
        elif w["kind"] == "zipf32":
            keys = zipf_u32_t(n, 1 << 20, ks, device)
            queries = zipf_u32_t(q, 1 << 20, qs, device)
        else:
            keys = zipf_u64_t(n, 1 << 20, ks, device)
            queries = zipf_u64_t(q, 1 << 20, qs, device)
        return keys, queries, opts
    if w["kind"] == "u32":
        keys = uniform_u32(n, ks)
        queries = queries_hit50(keys, q, qs)
    elif w["kind"] == "zipf32":
        keys = zipf_u32(n, 1 << 20, ks)
        queries = zipf_u32(q, 1 << 20, qs)
    else:
        keys = zipf_u64(n, 1 << 20, ks)
        queries = zipf_u64(q, 1 << 20, qs)
    return keys, queries, opts


# --------------------------------------------------------------------------
# Batched tables: T tables with sizes log-uniform in [2^lo, 2^hi]; table t
# draws its keys from stream BATCH_KEY_SEED + t and its queries (as many as
# keys, 50% hits, as queries_hit50) from stream BATCH_QUERY_SEED + t.
# --------------------------------------------------------------------------

BATCH_SIZE_SEED = 0x5EED0300
BATCH_KEY_SEED = 0x5EED0400
BATCH_QUERY_SEED = 0x5EED0600


def batch_sizes(T: int, lo_log2: float = 10, hi_log2: float = 20, seed: int = BATCH_SIZE_SEED) -> np.ndarray:
    """T table sizes, round(2^(lo + (hi - lo) u)) with u uniform in [0, 1)."""
    u = (splitmix64(seed, 0, T) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.round(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)


def segment_offsets(sizes) -> np.ndarray:
    return np.concatenate([[0], np.cumsum(np.asarray(sizes, np.int64))]).astype(np.uint32)


def batch_keys(sizes, seed: int = BATCH_KEY_SEED) -> np.ndarray:
    """Concatenated uint32 keys of the tables (table t: uniform_u32(n_t, seed + t))."""
    parts = [uniform_u32(int(s), seed + t) for t, s in enumerate(sizes)]
    return np.concatenate(parts) if parts else np.empty(0, np.uint32)


def batch_queries(keys: np.ndarray, sizes, qsizes, seed: int = BATCH_QUERY_SEED) -> np.ndarray:
    """Concatenated queries: segment t is queries_hit50(keys of table t,
    qsizes[t], seed + t)."""
    o = segment_offsets(sizes)
    parts = [queries_hit50(keys[int(o[t]):int(o[t + 1])], int(q), seed + t) for t, q in enumerate(qsizes)]
    return np.concatenate(parts) if parts else np.empty(0, keys.dtype)


def _segments_t(offsets, start: int, count: int, device):
    """(segment id, index inside the segment) of elements start .. start+count-1."""
    import torch

    idx = torch.arange(start, start + count, dtype=torch.int64, device=device)
    seg = torch.searchsorted(offsets[1:], idx, right=True)
    return seg, idx - offsets[seg]


def batch_keys_t(sizes, device, seed: int = BATCH_KEY_SEED, chunk: int = 1 << 26):
    """Device twin of batch_keys, drawn in chunks of ``chunk`` keys."""
    import torch

    offsets = torch.from_numpy(segment_offsets(sizes).astype(np.int64)).to(device)
    total = int(offsets[-1])
    out = torch.empty(total, dtype=torch.uint32, device=device)
    for c0 in range(0, total, chunk):
        c = min(chunk, total - c0)
        seg, local = _segments_t(offsets, c0, c, device)
        z = _mix_t((local + 1) * _s64(int(GAMMA)) + (seg + seed))
        out[c0:c0 + c] = _to_u32(z)
    return out


def batch_queries_t(keys, sizes, qsizes, device, seed: int = BATCH_QUERY_SEED, chunk: int = 1 << 26):
    """Device twin of batch_queries (keys: the device tensor of batch_keys_t)."""
    import torch

    koff = torch.from_numpy(segment_offsets(sizes).astype(np.int64)).to(device)
    qoff = torch.from_numpy(segment_offsets(qsizes).astype(np.int64)).to(device)
    total = int(qoff[-1])
    out = torch.empty(total, dtype=torch.uint32, device=device)
    kv = keys.view(torch.int32)
    for c0 in range(0, total, chunk):
        c = min(chunk, total - c0)
        seg, local = _segments_t(qoff, c0, c, device)
        sd = seg + seed
        wa = _mix_t((2 * local + 1) * _s64(int(GAMMA)) + sd)
        wb = _mix_t((2 * local + 2) * _s64(int(GAMMA)) + sd)
        n_t = koff[seg + 1] - koff[seg]
        pos = koff[seg] + _lsr((wa & 0xFFFFFFFF) * n_t, 32)
        hit = (wa < 0) & (n_t > 0)
        picked = kv[torch.clamp(pos, max=max(kv.numel() - 1, 0))] if kv.numel() else torch.zeros_like(pos, dtype=torch.int32)
        miss = _to_u32(wb).view(torch.int32)
        out[c0:c0 + c] = torch.where(hit, picked, miss).view(torch.uint32)
    return out
