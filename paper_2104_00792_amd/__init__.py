"""HashGraph build and probe on MI355X: Python binding of ``libhg.so``.

The binding only marshals arguments: device pointers and the HIP stream come
from torch tensors and ``torch.cuda.current_stream()``; every step of the
build and the probe runs in the library's HIP kernels.  If ``libhg.so`` has
not been built the first call raises; there is no fallback path.

Entry points mirror ``include/hg.h``: :func:`hg_build`, :func:`hg_count`,
:func:`hg_query`, :func:`hg_bin_partition`, :func:`hg_hash_bucket`, and the
batched forms :func:`hg_build_batched`, :func:`hg_count_batched`,
:func:`hg_query_batched`.
"""

from __future__ import annotations

import ctypes
import os

__all__ = [
    "HGError", "Table", "hg_build", "hg_build_like", "hg_intersect", "hg_count", "hg_query", "hg_bin_partition",
    "hg_bin_partition_noalloc",
    "hg_hash_bucket", "hg_bin_partition_balanced", "hg_build_batched", "hg_count_batched", "hg_query_batched", "hg_trim_pool",
    "hg_set_allocator", "hg_workspace_size", "torch_allocator", "lib", "lib_path", "profile",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libhg.so")

HG_KEY_U32 = 0
HG_KEY_U64 = 1

# Build strategies (include/hg.h): global atomics as in Algorithm 1, or two
# stable splits down to LDS-sized sub-bins.  0 lets the library choose.
HG_BUILD_ATOMIC = 1
HG_BUILD_SORTED = 2
# Probe strategies: each query reads its bucket in place, or queries are split
# like the table, counted against LDS windows and gathered back.
HG_PROBE_DIRECT = 1
HG_PROBE_SORTED = 2
# Operations sized by hg_workspace_size.
HG_OP_BUILD = 0
HG_OP_COUNT = 1
HG_OP_QUERY = 2
HG_OP_BUILD_BATCHED = 3
HG_OP_COUNT_BATCHED = 4
HG_OP_QUERY_BATCHED = 5
HG_OP_BIN_PARTITION = 6

# Allocator hook signatures of include/hg.h.
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_hooks = None  # the installed callbacks, kept alive while the library may call them

_lib = None


class HGError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {detail} (status {status})")


class _BuildOpts(ctypes.Structure):
    _fields_ = [
        ("P", ctypes.c_uint32),
        ("ratio_num", ctypes.c_uint32),
        ("ratio_den", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("num_buckets", ctypes.c_uint64),
        ("log2_subbin", ctypes.c_uint32),
        ("split_bits", ctypes.c_uint32),
    ]


class _TableDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint64),
        ("num_buckets", ctypes.c_uint64),
        ("P", ctypes.c_uint32),
        ("key_type", ctypes.c_uint32),
        ("d_keys", ctypes.c_void_p),
        ("d_offsets", ctypes.c_void_p),
        ("d_part_offsets", ctypes.c_void_p),
        ("d_bucket_base", ctypes.c_void_p),
        ("probe_count_bytes", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


def lib_path() -> str:
    return _LIB_PATH


def lib() -> ctypes.CDLL:
    """Load libhg.so (built in-tree by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch first: its HIP runtime (same soname) is then the one libhg.so
    # binds to, so streams and pointers from torch are valid in the library.
    _torch()
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(
            f"{_LIB_PATH} is missing: build it with __graft_entry__.build() "
            "(there is no fallback path)")
    L = ctypes.CDLL(_LIB_PATH)
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    L.hg_build.argtypes = [vp, u64, i32, ctypes.POINTER(_BuildOpts), vp, ctypes.POINTER(vp)]
    L.hg_build.restype = i32
    L.hg_build_like.argtypes = [vp, vp, u64, vp, ctypes.POINTER(vp)]
    L.hg_build_like.restype = i32
    L.hg_intersect.argtypes = [vp, vp, vp, vp]
    L.hg_intersect.restype = i32
    L.hg_count.argtypes = [vp, vp, u64, vp, vp]
    L.hg_count.restype = i32
    L.hg_query.argtypes = [vp, vp, u64, vp, vp]
    L.hg_query.restype = i32
    L.hg_count_ex.argtypes = [vp, vp, u64, vp, u32, vp]
    L.hg_count_ex.restype = i32
    L.hg_query_ex.argtypes = [vp, vp, u64, vp, u32, vp]
    L.hg_query_ex.restype = i32
    L.hg_build_batched.argtypes = [vp, u64, i32, u32, vp, ctypes.POINTER(_BuildOpts), vp, ctypes.POINTER(vp)]
    L.hg_build_batched.restype = i32
    L.hg_count_batched.argtypes = [vp, vp, u64, vp, vp, vp]
    L.hg_count_batched.restype = i32
    L.hg_query_batched.argtypes = [vp, vp, u64, vp, vp, vp]
    L.hg_query_batched.restype = i32
    L.hg_bin_partition.argtypes = [vp, u64, i32, u32, vp, vp, vp]
    L.hg_bin_partition.restype = i32
    L.hg_bin_partition_noalloc.argtypes = [vp, u64, i32, u32, vp, vp, vp]
    L.hg_bin_partition_noalloc.restype = i32
    L.hg_bin_partition_balanced.argtypes = [vp, u64, i32, u32, u64, u32, vp, vp, vp, vp]
    L.hg_bin_partition_balanced.restype = i32
    L.hg_hash_bucket.argtypes = [vp, u64, i32, u64, vp, vp, vp]
    L.hg_hash_bucket.restype = i32
    L.hg_table_info.argtypes = [vp, ctypes.POINTER(_TableDesc)]
    L.hg_table_info.restype = i32
    L.hg_table_export.argtypes = [vp, vp, vp, vp, vp, vp]
    L.hg_table_export.restype = i32
    L.hg_table_free.argtypes = [vp]
    L.hg_table_free.restype = None
    L.hg_trim_pool.argtypes = [u64]
    L.hg_trim_pool.restype = i32
    L.hg_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, vp]
    L.hg_set_allocator.restype = i32
    L.hg_workspace_size.argtypes = [i32, vp, u64, i32, ctypes.POINTER(_BuildOpts), u32,
                                    ctypes.POINTER(u64), ctypes.POINTER(u64)]
    L.hg_workspace_size.restype = i32
    L.hg_status_string.argtypes = [i32]
    L.hg_status_string.restype = ctypes.c_char_p
    L.hg_last_error.argtypes = []
    L.hg_last_error.restype = ctypes.c_char_p
    L.hg_profile_enable.argtypes = [i32]
    L.hg_profile_enable.restype = i32
    L.hg_profile_only.argtypes = [ctypes.c_char_p]
    L.hg_profile_only.restype = i32
    L.hg_profile_collect.argtypes = []
    L.hg_profile_collect.restype = i32
    L.hg_profile_read.argtypes = [ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(u64),
                                  ctypes.POINTER(ctypes.c_double), i32]
    L.hg_profile_read.restype = i32
    L.hg_profile_reset.argtypes = []
    L.hg_profile_reset.restype = None
    _lib = L
    return L


def _check(status: int, where: str):
    if status != 0:
        L = lib()
        raise HGError(status, where, L.hg_last_error().decode() or L.hg_status_string(status).decode())


def _torch():
    import torch
    return torch


def _key_type(t) -> int:
    torch = _torch()
    if t.dtype in (torch.uint32, torch.int32):
        return HG_KEY_U32
    if t.dtype in (torch.uint64, torch.int64):
        return HG_KEY_U64
    raise TypeError(f"keys must be 32- or 64-bit integers, got {t.dtype}")


def _dev_ptr(t) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr() if t.numel() > 0 else None


def _stream(stream) -> int | None:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream or None


class Table:
    """A built table (owns device memory until :meth:`free`)."""

    def __init__(self, handle: int, key_type: int, n: int, P: int):
        self._h = handle
        self.key_type = key_type
        self.n = n
        self.P = P

    @property
    def handle(self) -> int:
        if not self._h:
            raise ValueError("table already freed")
        return self._h

    def count(self, queries, out=None, stream=None, flags=0):
        return hg_count(self, queries, out, stream, flags)

    def query(self, queries, out=None, stream=None, flags=0):
        return hg_query(self, queries, out, stream, flags)

    def info(self) -> dict:
        d = _TableDesc()
        _check(lib().hg_table_info(self.handle, ctypes.byref(d)), "hg_table_info")
        return {"n": d.n, "num_buckets": d.num_buckets, "P": d.P, "key_type": d.key_type,
                "d_keys": d.d_keys, "d_offsets": d.d_offsets,
                "d_part_offsets": d.d_part_offsets, "d_bucket_base": d.d_bucket_base,
                "probe_count_bytes": d.probe_count_bytes}

    def export(self, stream=None):
        """Device copies of (part_offsets, bucket_base, offsets, keys)."""
        torch = _torch()
        d = self.info()
        kdt = torch.uint32 if self.key_type == HG_KEY_U32 else torch.uint64
        po = torch.empty(self.P + 1, dtype=torch.uint32, device="cuda")
        bb = torch.empty(self.P + 1, dtype=torch.uint32, device="cuda")
        offs = torch.empty(d["num_buckets"] + 1, dtype=torch.uint32, device="cuda")
        keys = torch.empty(self.n, dtype=kdt, device="cuda")
        _check(lib().hg_table_export(self.handle, _dev_ptr(po), _dev_ptr(bb), _dev_ptr(offs), _dev_ptr(keys),
                                     _stream(stream)), "hg_table_export")
        return po, bb, offs, keys

    def free(self):
        if self._h:
            lib().hg_table_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def hg_build(keys, P: int = 1, ratio=(1, 1), num_buckets: int = 0, stream=None, flags: int = 0,
             log2_subbin: int = 0, split_bits: int = 0) -> Table:
    """Build a table from a device tensor of 32- or 64-bit keys.

    V_p = max(1, n_p * ratio[0] // ratio[1]); with P == 1 a nonzero
    ``num_buckets`` fixes V instead.  ``flags``: HG_BUILD_ATOMIC or
    HG_BUILD_SORTED to pin the strategy (the table is the same).
    ``log2_subbin`` (10..13) and ``split_bits`` (7..10) tune the sorted build
    (0: the library's choice); they never change the table."""
    kt = _key_type(keys)
    opts = _BuildOpts(P, ratio[0], ratio[1], flags, num_buckets, log2_subbin, split_bits)
    h = ctypes.c_void_p()
    _check(lib().hg_build(_dev_ptr(keys), keys.numel(), kt, ctypes.byref(opts), _stream(stream),
                          ctypes.byref(h)), "hg_build")
    return Table(h.value, kt, keys.numel(), P)


def hg_build_like(table: Table, keys, stream=None) -> Table:
    """A HashGraph of `keys` (the query set) over the same buckets as
    `table` (Sec. 3.3): bucket g of both holds the keys hashing to g."""
    if _key_type(keys) != table.key_type:
        raise TypeError("keys and table keys differ in width")
    h = ctypes.c_void_p()
    _check(lib().hg_build_like(table.handle, _dev_ptr(keys), keys.numel(), _stream(stream), ctypes.byref(h)),
           "hg_build_like")
    return Table(h.value, table.key_type, keys.numel(), table.P)


def hg_intersect(table: Table, queries: Table, out=None, stream=None):
    """Per-bucket intersections (Sec. 3.3): for each key of the query table
    in its bucket order, the number of equal keys in `table` (uint32)."""
    torch = _torch()
    if out is None:
        out = torch.empty(queries.n, dtype=torch.uint32, device="cuda")
    _check(lib().hg_intersect(table.handle, queries.handle, _dev_ptr(out), _stream(stream)), "hg_intersect")
    return out


def hg_count(table: Table, queries, out=None, stream=None, flags: int = 0):
    """Exact multiplicity of each query (uint32 device tensor).  ``flags``:
    HG_PROBE_DIRECT or HG_PROBE_SORTED to pin the strategy."""
    torch = _torch()
    if _key_type(queries) != table.key_type:
        raise TypeError("queries and table keys differ in width")
    if out is None:
        out = torch.empty(queries.numel(), dtype=torch.uint32, device=queries.device)
    _check(lib().hg_count_ex(table.handle, _dev_ptr(queries), queries.numel(), _dev_ptr(out), flags,
                             _stream(stream)), "hg_count")
    return out


def hg_query(table: Table, queries, out=None, stream=None, flags: int = 0):
    """Existence of each query (uint8 device tensor of 0/1)."""
    torch = _torch()
    if _key_type(queries) != table.key_type:
        raise TypeError("queries and table keys differ in width")
    if out is None:
        out = torch.empty(queries.numel(), dtype=torch.uint8, device=queries.device)
    _check(lib().hg_query_ex(table.handle, _dev_ptr(queries), queries.numel(), _dev_ptr(out), flags,
                             _stream(stream)), "hg_query")
    return out


def hg_build_batched(keys, table_offsets, ratio=(1, 1), stream=None, log2_subbin: int = 0) -> Table:
    """Build T tables at once: table t holds keys[table_offsets[t] ..
    table_offsets[t+1]) (``table_offsets``: uint32 device tensor of T + 1
    entries from 0 to n) with V_t = max(1, n_t * ratio[0] // ratio[1]).
    ``log2_subbin`` (10..13, 0: the library's choice) tunes the build."""
    kt = _key_type(keys)
    T = table_offsets.numel() - 1
    if table_offsets.dtype not in (_torch().uint32, _torch().int32):
        raise TypeError("table_offsets must be 32-bit")
    opts = _BuildOpts(1, ratio[0], ratio[1], 0, 0, log2_subbin, 0)
    h = ctypes.c_void_p()
    _check(lib().hg_build_batched(_dev_ptr(keys), keys.numel(), kt, max(T, 0), _dev_ptr(table_offsets),
                                  ctypes.byref(opts), _stream(stream), ctypes.byref(h)), "hg_build_batched")
    return Table(h.value, kt, keys.numel(), T)


def hg_count_batched(table: Table, queries, query_offsets, out=None, stream=None):
    """Exact multiplicity of each query in its own table: queries[qo[t] ..
    qo[t+1]) go to table t (``query_offsets`` = qo, uint32 device tensor)."""
    torch = _torch()
    if _key_type(queries) != table.key_type:
        raise TypeError("queries and table keys differ in width")
    if out is None:
        out = torch.empty(queries.numel(), dtype=torch.uint32, device=queries.device)
    _check(lib().hg_count_batched(table.handle, _dev_ptr(queries), queries.numel(), _dev_ptr(query_offsets),
                                  _dev_ptr(out), _stream(stream)), "hg_count_batched")
    return out


def hg_query_batched(table: Table, queries, query_offsets, out=None, stream=None):
    """Existence of each query in its own table (uint8 0/1)."""
    torch = _torch()
    if _key_type(queries) != table.key_type:
        raise TypeError("queries and table keys differ in width")
    if out is None:
        out = torch.empty(queries.numel(), dtype=torch.uint8, device=queries.device)
    _check(lib().hg_query_batched(table.handle, _dev_ptr(queries), queries.numel(), _dev_ptr(query_offsets),
                                  _dev_ptr(out), _stream(stream)), "hg_query_batched")
    return out


def hg_trim_pool(keep_bytes: int = 0):
    """Hand the library's cached device memory (freed tables and workspace)
    back to the system, keeping at most ``keep_bytes``."""
    _check(lib().hg_trim_pool(keep_bytes), "hg_trim_pool")


def hg_workspace_size(op: int, n: int = 0, key_type: int = HG_KEY_U32, P: int = 1, ratio=(1, 1),
                      num_buckets: int = 0, flags: int = 0, table: Table | None = None, aux: int = 0,
                      log2_subbin: int = 0, split_bits: int = 0):
    """(workspace bytes, table bytes) that one call of ``op`` allocates,
    computed on the host without touching the device.  Builds take n,
    key_type, P, ratio, num_buckets and flags (and ``aux`` = number of tables
    for HG_OP_BUILD_BATCHED); probes take ``table``, n = number of queries and
    ``aux`` = probe flags."""
    opts = _BuildOpts(P, ratio[0], ratio[1], flags, num_buckets, log2_subbin, split_bits)
    ws, tb = ctypes.c_uint64(), ctypes.c_uint64()
    h = table.handle if table is not None else None
    _check(lib().hg_workspace_size(op, h, n, key_type, ctypes.byref(opts), aux, ctypes.byref(ws), ctypes.byref(tb)),
           "hg_workspace_size")
    return ws.value, tb.value


def hg_set_allocator(alloc=None, free=None):
    """Route the library's device allocations through Python callables:
    ``alloc(nbytes, stream_handle) -> device address (int) or 0`` and
    ``free(address, nbytes, stream_handle)``, with the stream-ordered contract
    of include/hg.h.  No arguments restores the library's own pool.  Tables
    built under an allocator return their memory to it when freed, so keep the
    callables usable until those tables are freed."""
    global _hooks
    if (alloc is None) != (free is None):
        raise ValueError("hg_set_allocator takes both callables or neither")
    if alloc is None:
        _check(lib().hg_set_allocator(_ALLOC_FN(), _FREE_FN(), None), "hg_set_allocator")
        return

    def _alloc(nbytes, stream, ctx):
        return alloc(nbytes, stream or 0) or None

    def _free(ptr, nbytes, stream, ctx):
        free(ptr, nbytes, stream or 0)

    hooks = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    _check(lib().hg_set_allocator(hooks[0], hooks[1], None), "hg_set_allocator")
    # Older hooks stay referenced: tables built under them still free through them.
    _hooks = (hooks, _hooks)


class torch_allocator:
    """``with torch_allocator(): ...`` serves the library's device memory from
    torch's caching allocator (the stream passed by the library is the one the
    block is used on), then restores the library's pool."""

    def __enter__(self):
        torch = _torch()
        dev = torch.cuda.current_device()

        def alloc(nbytes, stream):
            return torch.cuda.caching_allocator_alloc(nbytes, dev, stream)

        def free(ptr, nbytes, stream):
            torch.cuda.caching_allocator_delete(ptr)

        hg_set_allocator(alloc, free)
        return self

    def __exit__(self, *exc):
        hg_set_allocator()
        return False


def hg_bin_partition(keys, P: int, out=None, part_offsets=None, stream=None):
    """Hash-range split into P partitions: (keys grouped by partition,
    part_offsets[P+1])."""
    torch = _torch()
    kt = _key_type(keys)
    if out is None:
        out = torch.empty_like(keys)
    if part_offsets is None:
        part_offsets = torch.empty(P + 1, dtype=torch.uint32, device=keys.device)
    _check(lib().hg_bin_partition(_dev_ptr(keys), keys.numel(), kt, P, _dev_ptr(out), _dev_ptr(part_offsets),
                                  _stream(stream)), "hg_bin_partition")
    return out, part_offsets


def hg_bin_partition_noalloc(keys, P: int, out, part_offsets, stream=None):
    """hg_bin_partition into caller-given outputs with no device allocation
    by the library (its scratch is a fixed array of 2^20 + 1024 words per
    device, so P * ceil(n / 4096) <= 2^20).  Returns (out, part_offsets)."""
    kt = _key_type(keys)
    _check(lib().hg_bin_partition_noalloc(_dev_ptr(keys), keys.numel(), kt, P, _dev_ptr(out), _dev_ptr(part_offsets),
                                          _stream(stream)), "hg_bin_partition_noalloc")
    return out, part_offsets


def hg_bin_partition_balanced(keys, P: int, hash_range: int, num_bins: int = 0, out=None, part_offsets=None,
                              bin_splits=None, stream=None):
    """Count-balanced hash-range split into P partitions (Algorithm 2,
    Phases 1 and 2): (keys grouped by partition, part_offsets[P+1],
    bin_splits[P+1]).  num_bins 0 takes ceil(sqrt(hash_range))."""
    torch = _torch()
    kt = _key_type(keys)
    if out is None:
        out = torch.empty_like(keys)
    if part_offsets is None:
        part_offsets = torch.empty(P + 1, dtype=torch.uint32, device=keys.device)
    if bin_splits is None:
        bin_splits = torch.empty(P + 1, dtype=torch.uint32, device=keys.device)
    _check(lib().hg_bin_partition_balanced(_dev_ptr(keys), keys.numel(), kt, P, hash_range, num_bins, _dev_ptr(out),
                                           _dev_ptr(part_offsets), _dev_ptr(bin_splits), _stream(stream)),
           "hg_bin_partition_balanced")
    return out, part_offsets, bin_splits


def hg_hash_bucket(keys, V: int, want_hash: bool = True, stream=None):
    """(hash(k) as uint64, hash(k) mod V as uint32) for every key."""
    torch = _torch()
    kt = _key_type(keys)
    n = keys.numel()
    h = torch.empty(n, dtype=torch.uint64, device=keys.device) if want_hash else None
    b = torch.empty(n, dtype=torch.uint32, device=keys.device)
    _check(lib().hg_hash_bucket(_dev_ptr(keys), n, kt, V, _dev_ptr(h), _dev_ptr(b), _stream(stream)),
           "hg_hash_bucket")
    return h, b


class profile:
    """Per-kernel HIP-event timing of the library's launches.

    ``with profile() as p: ...`` then ``p.results`` maps kernel name to
    (launches, total milliseconds).  ``profile(only="lds_probe")`` brackets
    the launches of that name only."""

    def __init__(self, only: str | None = None):
        self.only = only

    def __enter__(self):
        L = lib()
        L.hg_profile_reset()
        _check(L.hg_profile_only(self.only.encode() if self.only else None), "hg_profile_only")
        _check(L.hg_profile_enable(1), "hg_profile_enable")
        self.results = {}
        return self

    def __exit__(self, *exc):
        L = lib()
        L.hg_profile_enable(0)
        L.hg_profile_only(None)
        _check(L.hg_profile_collect(), "hg_profile_collect")
        cap = 64
        names = (ctypes.c_char_p * cap)()
        launches = (ctypes.c_uint64 * cap)()
        ms = (ctypes.c_double * cap)()
        k = L.hg_profile_read(names, launches, ms, cap)
        self.results = {names[i].decode(): (int(launches[i]), float(ms[i])) for i in range(min(k, cap))}
        return False
