"""HashGraph CPU oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library and its Python binding
never import it.  The arithmetic lives in ``hg_oracle.cpp`` (plain C++17:
std::sort of tuples plus run-length counting); this module only builds that
file with g++ and marshals numpy arrays through ctypes.

Every function follows a passage of the paper (Tripathy & Green, arXiv
2104.00792): Algorithm 1 and the CSR paragraph of Sec. 3.1 for the build,
Algorithm 2 Phase 2 for the partition split, Sec. 3.3 "Querying" and Sec. 5.4
(duplicate counting) for the probe.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hg_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle_hg.so")
# The same source built for all host cores (OpenMP, GNU parallel-mode sort).
_LIB_PAR = os.path.join(_HERE, "liboracle_hg_par.so")

KT_U32 = 0
KT_U64 = 1

_lib = None


def compile_oracle(src: str, out: str, parallel: bool = False) -> str:
    """Compile an oracle source file with g++ (no HIP, no GPU headers).
    ``parallel``: the all-core build of the same source (OpenMP loops and the
    GNU parallel-mode std::sort)."""
    tmp = out + ".tmp"
    extra = ["-fopenmp", "-D_GLIBCXX_PARALLEL"] if parallel else []
    cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", *extra, src, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        compile_oracle(_SRC, _LIB)
    if force or not os.path.exists(_LIB_PAR):
        compile_oracle(_SRC, _LIB_PAR, parallel=True)
    return _LIB


def load_library(path: str):
    """ctypes handle with typed entry points for an oracle build at `path`."""
    lib = ctypes.CDLL(path)
    u32, u64, i32, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
    lib.orc_fmix32.argtypes = [u32]
    lib.orc_fmix32.restype = u32
    lib.orc_fmix64.argtypes = [u64]
    lib.orc_fmix64.restype = u64
    lib.orc_hash_bucket.argtypes = [vp, u64, i32, u64, vp, vp]
    lib.orc_hash_bucket.restype = i32
    lib.orc_layout.argtypes = [vp, u64, i32, u32, u32, u32, u64, vp, vp]
    lib.orc_layout.restype = i32
    lib.orc_build.argtypes = [vp, u64, i32, u32, u32, u32, u64, vp, vp, vp, u64, vp]
    lib.orc_build.restype = i32
    lib.orc_count.argtypes = [vp, u64, i32, vp, u64, vp]
    lib.orc_count.restype = i32
    lib.orc_bin_partition.argtypes = [vp, u64, i32, u32, vp, vp]
    lib.orc_bin_partition.restype = i32
    lib.orc_bin_partition_balanced.argtypes = [vp, u64, i32, u32, u64, u32, vp, vp, vp]
    lib.orc_bin_partition_balanced.restype = i32
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = load_library(_LIB)
    return _lib


def use_library(path: str | None):
    """Point this module at another oracle build (None: the default one).
    Used only by the planted-mistake tests."""
    global _lib
    _lib = None if path is None else load_library(path)


class all_cores:
    """``with oracle.all_cores(): ...`` runs the oracle calls inside on the
    all-core build of the same source (``threads`` OpenMP threads; None: the
    OpenMP default), then returns to the single-threaded build."""

    def __init__(self, threads: int | None = None):
        self.threads = threads

    def __enter__(self):
        global _lib
        if not os.path.exists(_LIB_PAR):
            compile_oracle(_SRC, _LIB_PAR, parallel=True)
        self._saved = _lib
        if self.threads is not None:
            os.environ["OMP_NUM_THREADS"] = str(self.threads)
        _lib = load_library(_LIB_PAR)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False


def _kt(a: np.ndarray) -> int:
    if a.dtype == np.uint32:
        return KT_U32
    if a.dtype == np.uint64:
        return KT_U64
    raise TypeError(f"keys must be uint32 or uint64, got {a.dtype}")


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (code {rc})")


def fmix32(x: int) -> int:
    """MurmurHash3 32-bit finalizer of one value."""
    return int(_load().orc_fmix32(int(x) & 0xFFFFFFFF))


def fmix64(x: int) -> int:
    """MurmurHash3 64-bit finalizer of one value."""
    return int(_load().orc_fmix64(int(x) & 0xFFFFFFFFFFFFFFFF))


def hash_bucket(keys: np.ndarray, V: int):
    """hash(A[i]) (uint64) and hash(A[i]) mod V (uint32) for every key."""
    keys = np.ascontiguousarray(keys)
    n = keys.size
    h = np.empty(n, np.uint64)
    b = np.empty(n, np.uint32)
    _check(_load().orc_hash_bucket(_ptr(keys), n, _kt(keys), V, _ptr(h), _ptr(b)), "hash_bucket")
    return h, b


def layout(keys: np.ndarray, P: int = 1, num: int = 1, den: int = 1, V: int = 0):
    """part_offsets[P+1] and bucket_base[P+1] of the table the build makes."""
    keys = np.ascontiguousarray(keys)
    po = np.empty(P + 1, np.uint32)
    bb = np.empty(P + 1, np.uint32)
    _check(_load().orc_layout(_ptr(keys), keys.size, _kt(keys), P, num, den, V, _ptr(po), _ptr(bb)), "layout")
    return po, bb


def build_table(keys: np.ndarray, P: int = 1, num: int = 1, den: int = 1, V: int = 0):
    """Whole build (steps O1-O3).

    Returns dict(part_offsets, bucket_base, offsets, keys) with ``keys`` in
    canonical form (each bucket ascending).  ``V`` (nonzero, P == 1 only)
    fixes the bucket count; otherwise V_p = max(1, n_p * num // den).
    """
    keys = np.ascontiguousarray(keys)
    po, bb = layout(keys, P, num, den, V)
    total = int(bb[P])
    offsets = np.empty(total + 1, np.uint32)
    out = np.empty_like(keys)
    rc = _load().orc_build(_ptr(keys), keys.size, _kt(keys), P, num, den, V,
                           _ptr(po), _ptr(bb), _ptr(offsets), offsets.size, _ptr(out))
    _check(rc, "build")
    return {"part_offsets": po, "bucket_base": bb, "offsets": offsets, "keys": out}


def count(keys: np.ndarray, queries: np.ndarray) -> np.ndarray:
    """Exact multiplicity of every query in ``keys`` (step O4)."""
    keys = np.ascontiguousarray(keys)
    queries = np.ascontiguousarray(queries)
    if keys.dtype != queries.dtype:
        raise TypeError("keys and queries must share a dtype")
    out = np.empty(queries.size, np.uint32)
    _check(_load().orc_count(_ptr(keys), keys.size, _kt(keys), _ptr(queries), queries.size, _ptr(out)), "count")
    return out


def bin_partition(keys: np.ndarray, P: int):
    """Partition split alone (step O5): part_offsets[P+1] and the keys,
    each partition ascending."""
    keys = np.ascontiguousarray(keys)
    po = np.empty(P + 1, np.uint32)
    out = np.empty_like(keys)
    _check(_load().orc_bin_partition(_ptr(keys), keys.size, _kt(keys), P, _ptr(po), _ptr(out)), "bin_partition")
    return po, out


def bin_partition_balanced(keys: np.ndarray, P: int, HR: int, num_bins: int = 0):
    """Count-balanced split (step O6, Algorithm 2 Phases 1 and 2):
    (part_offsets[P+1], bin_splits[P+1], keys grouped by partition, each
    group ascending)."""
    keys = np.ascontiguousarray(keys)
    po = np.empty(P + 1, np.uint32)
    splits = np.empty(P + 1, np.uint32)
    out = np.empty_like(keys)
    _check(_load().orc_bin_partition_balanced(_ptr(keys), keys.size, _kt(keys), P, HR, num_bins, _ptr(po),
                                              _ptr(splits), _ptr(out)), "bin_partition_balanced")
    return po, splits, out


def build_like(table_keys: np.ndarray, queries: np.ndarray, P: int = 1, num: int = 1, den: int = 1, V: int = 0):
    """The query set's HashGraph over the buckets of the table built from
    table_keys (Sec. 3.3, "Querying"): the table's V_p and bucket bases, the
    queries' own partition offsets; each query in bucket bucket_base[p] +
    hash mod V_p, where p is the partition of its hash.  Returns
    dict(part_offsets, bucket_base, offsets, keys), keys canonical (each
    bucket ascending)."""
    queries = np.ascontiguousarray(queries)
    _, bb = layout(table_keys, P, num, den, V)
    B = int(bb[P])
    w = 32 if queries.dtype == np.uint32 else 64
    h, _ = hash_bucket(queries, 1)
    h = h.astype(np.uint64)
    log2P = P.bit_length() - 1
    p = (h >> np.uint64(w - log2P)).astype(np.int64) if log2P else np.zeros(queries.size, np.int64)
    Vp = np.diff(bb.astype(np.int64)).astype(np.uint64)
    g = bb[p].astype(np.int64) + (h % Vp[p]).astype(np.int64) if queries.size else np.zeros(0, np.int64)
    order = np.lexsort((queries, g))
    offsets = np.concatenate([[0], np.cumsum(np.bincount(g, minlength=B))]).astype(np.uint32)
    po = np.concatenate([[0], np.cumsum(np.bincount(p, minlength=P))]).astype(np.uint32)
    return {"part_offsets": po, "bucket_base": bb, "offsets": offsets, "keys": queries[order]}


def canonicalize(offsets: np.ndarray, keys: np.ndarray) -> np.ndarray:
    """Sort every bucket segment keys[offsets[g]:offsets[g+1]] ascending.

    The comparison form shared by every parity test: the order inside a
    bucket is left open by the paper (atomics of Algorithm 1)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    keys = np.asarray(keys)
    n = keys.size
    lengths = np.diff(offsets)
    if lengths.size == 0 or n == 0:
        return keys.copy()
    seg = np.repeat(np.arange(lengths.size, dtype=np.int64), lengths)
    order = np.lexsort((keys, seg))
    return keys[order]


def clamp_offsets(offsets: np.ndarray, n: int) -> np.ndarray:
    """Segment offsets as the batched calls read them: entry 0 is 0, entry T
    is n, every other entry min(o[x], n), then the running maximum (a
    non-decreasing sequence from 0 to n)."""
    o = np.asarray(offsets, dtype=np.int64).copy()
    o[0] = 0
    o[-1] = n
    o = np.minimum(o, n)
    return np.maximum.accumulate(o).astype(np.uint32)


def build_batched(keys: np.ndarray, table_offsets: np.ndarray, num: int = 1, den: int = 1):
    """A batch of tables: table t is build_table(keys[o[t]:o[t+1]]) with P = 1,
    its buckets placed after those of tables 0..t-1 (one CSR over all
    buckets).  Returns dict(part_offsets = o, bucket_base, offsets, keys)."""
    keys = np.ascontiguousarray(keys)
    o = clamp_offsets(table_offsets, keys.size)
    bb = [0]
    offs = []
    out = []
    for t in range(o.size - 1):
        r = build_table(keys[int(o[t]):int(o[t + 1])], P=1, num=num, den=den)
        offs.append(r["offsets"][:-1].astype(np.int64) + int(o[t]))
        out.append(r["keys"])
        bb.append(bb[-1] + int(r["bucket_base"][1]))
    offsets = np.concatenate(offs + [np.array([keys.size], np.int64)]).astype(np.uint32)
    kk = np.concatenate(out) if out else keys[:0].copy()
    return {"part_offsets": o, "bucket_base": np.array(bb, np.uint32), "offsets": offsets, "keys": kk}


def count_batched(keys: np.ndarray, table_offsets: np.ndarray, queries: np.ndarray,
                  query_offsets: np.ndarray) -> np.ndarray:
    """Multiplicity of every query of segment t among the keys of table t."""
    o = clamp_offsets(table_offsets, keys.size)
    qo = clamp_offsets(query_offsets, queries.size)
    out = np.empty(queries.size, np.uint32)
    for t in range(o.size - 1):
        a, b = int(qo[t]), int(qo[t + 1])
        out[a:b] = count(keys[int(o[t]):int(o[t + 1])], queries[a:b])
    return out
