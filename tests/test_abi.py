"""The C ABI without a GPU: the library loads, exports every entry point that
include/hg.h declares, and rejects bad arguments before any HIP call."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hg.h")
LIB = os.path.join(ROOT, "paper_2104_00792_amd", "libhg.so")

HG_OK, HG_ERR_INVALID_ARG, HG_ERR_OUT_OF_MEMORY, HG_ERR_HIP, HG_ERR_UNSUPPORTED = range(5)


class Opts(ctypes.Structure):
    _fields_ = [("P", ctypes.c_uint32), ("ratio_num", ctypes.c_uint32), ("ratio_den", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("num_buckets", ctypes.c_uint64), ("log2_subbin", ctypes.c_uint32),
                ("split_bits", ctypes.c_uint32)]


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hg_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libhg.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB)
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    L.hg_build.argtypes = [vp, u64, i32, ctypes.POINTER(Opts), vp, ctypes.POINTER(vp)]
    L.hg_count.argtypes = [vp, vp, u64, vp, vp]
    L.hg_query.argtypes = [vp, vp, u64, vp, vp]
    L.hg_bin_partition.argtypes = [vp, u64, i32, u32, vp, vp, vp]
    L.hg_hash_bucket.argtypes = [vp, u64, i32, u64, vp, vp, vp]
    L.hg_table_info.argtypes = [vp, vp]
    L.hg_table_export.argtypes = [vp, vp, vp, vp, vp, vp]
    L.hg_status_string.argtypes = [i32]
    L.hg_status_string.restype = ctypes.c_char_p
    L.hg_last_error.restype = ctypes.c_char_p
    L.hg_table_free.argtypes = [vp]
    L.hg_table_free.restype = None
    L.hg_build_batched.argtypes = [vp, u64, i32, u32, vp, ctypes.POINTER(Opts), vp, ctypes.POINTER(vp)]
    L.hg_count_batched.argtypes = [vp, vp, u64, vp, vp, vp]
    L.hg_query_batched.argtypes = [vp, vp, u64, vp, vp, vp]
    return L


def test_header_declares_the_core_calls():
    fns = declared_functions()
    for name in ["hg_build", "hg_count", "hg_query", "hg_bin_partition", "hg_hash_bucket", "hg_table_info",
                 "hg_table_export", "hg_table_free", "hg_status_string", "hg_last_error", "hg_build_batched",
                 "hg_count_batched", "hg_query_batched", "hg_set_allocator", "hg_workspace_size",
                 "hg_bin_partition_balanced", "hg_build_like", "hg_intersect"]:
        assert name in fns


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in hg.h but not exported"


def test_status_strings(lib):
    for code, name in enumerate(["HG_OK", "HG_ERR_INVALID_ARG", "HG_ERR_OUT_OF_MEMORY", "HG_ERR_HIP",
                                 "HG_ERR_UNSUPPORTED"]):
        assert lib.hg_status_string(code).decode() == name


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


def build(lib, keys, n, kt=0, P=1, num=1, den=1, V=0, flags=0, out=True, sub=0, bits=0):
    opts = Opts(P, num, den, flags, V, sub, bits)
    h = ctypes.c_void_p()
    return lib.hg_build(keys, n, kt, ctypes.byref(opts), None, ctypes.byref(h) if out else None)


@pytest.mark.parametrize("case, expected", [
    (dict(keys=None, n=10), HG_ERR_INVALID_ARG),             # null keys
    (dict(keys=FAKE, n=1 << 32), HG_ERR_INVALID_ARG),        # n >= 2^32
    (dict(keys=FAKE, n=10, kt=7), HG_ERR_INVALID_ARG),       # key type
    (dict(keys=FAKE, n=10, P=0), HG_ERR_INVALID_ARG),        # P = 0
    (dict(keys=FAKE, n=10, P=12), HG_ERR_INVALID_ARG),       # P not a power of two
    (dict(keys=FAKE, n=10, P=512), HG_ERR_UNSUPPORTED),      # P above 256
    (dict(keys=FAKE, n=10, num=0), HG_ERR_INVALID_ARG),      # zero ratio
    (dict(keys=FAKE, n=10, den=0), HG_ERR_INVALID_ARG),
    (dict(keys=FAKE, n=10, V=(1 << 32) - 1), HG_ERR_INVALID_ARG),  # V too large
    (dict(keys=FAKE, n=(1 << 32) - 1, num=2), HG_ERR_INVALID_ARG),  # too many buckets
    (dict(keys=FAKE, n=10, flags=4), HG_ERR_INVALID_ARG),    # unknown build flag
    (dict(keys=FAKE, n=10, flags=3), HG_ERR_INVALID_ARG),    # both strategies
    (dict(keys=FAKE, n=10, out=False), HG_ERR_INVALID_ARG),  # null out
    (dict(keys=FAKE, n=10, sub=9), HG_ERR_INVALID_ARG),      # sub-bins below 2^10 buckets
    (dict(keys=FAKE, n=10, sub=14), HG_ERR_INVALID_ARG),     # sub-bins above LDS size
    (dict(keys=FAKE, n=10, bits=6), HG_ERR_INVALID_ARG),     # level-2 digits
    (dict(keys=FAKE, n=10, bits=11), HG_ERR_INVALID_ARG),
])
def test_build_rejects(lib, case, expected):
    assert build(lib, **case) == expected
    assert lib.hg_last_error().decode() != ""


def test_build_null_opts(lib):
    h = ctypes.c_void_p()
    assert lib.hg_build(FAKE, 10, 0, None, None, ctypes.byref(h)) == HG_ERR_INVALID_ARG


def test_probe_rejects(lib):
    assert lib.hg_count(None, FAKE, 10, FAKE, None) == HG_ERR_INVALID_ARG
    assert lib.hg_query(None, FAKE, 10, FAKE, None) == HG_ERR_INVALID_ARG
    lib.hg_count_ex.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                ctypes.c_uint32, ctypes.c_void_p]
    assert lib.hg_count_ex(None, FAKE, 10, FAKE, 0, None) == HG_ERR_INVALID_ARG


def test_bin_partition_rejects(lib):
    assert lib.hg_bin_partition(FAKE, 10, 0, 3, FAKE, FAKE, None) == HG_ERR_INVALID_ARG
    assert lib.hg_bin_partition(FAKE, 10, 0, 16, FAKE, None, None) == HG_ERR_INVALID_ARG
    assert lib.hg_bin_partition(None, 10, 0, 16, FAKE, FAKE, None) == HG_ERR_INVALID_ARG
    assert lib.hg_bin_partition(FAKE, 1 << 32, 0, 16, FAKE, FAKE, None) == HG_ERR_INVALID_ARG
    assert lib.hg_bin_partition(FAKE, 10, 0, 1024, FAKE, FAKE, None) == HG_ERR_UNSUPPORTED


def test_bin_partition_noalloc_rejects(lib):
    """Argument errors, including a request larger than the fixed scratch
    (P * ceil(n / 4096) above 2^20), come back before any HIP call."""
    f = lib.hg_bin_partition_noalloc
    f.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_void_p]
    assert f(FAKE, 10, 0, 3, FAKE, FAKE, None) == HG_ERR_INVALID_ARG
    assert f(FAKE, 10, 0, 16, FAKE, None, None) == HG_ERR_INVALID_ARG
    assert f(None, 10, 0, 16, FAKE, FAKE, None) == HG_ERR_INVALID_ARG
    assert f(FAKE, 1 << 32, 0, 16, FAKE, FAKE, None) == HG_ERR_INVALID_ARG
    assert f(FAKE, 10, 0, 1024, FAKE, FAKE, None) == HG_ERR_UNSUPPORTED
    assert f(FAKE, (1 << 28) + 1, 0, 16, FAKE, FAKE, None) == HG_ERR_INVALID_ARG
    assert "scratch" in lib.hg_last_error().decode()
    assert f(FAKE, (1 << 24) + 1, 1, 256, FAKE, FAKE, None) == HG_ERR_INVALID_ARG


def test_hash_bucket_rejects(lib):
    assert lib.hg_hash_bucket(FAKE, 10, 0, 0, FAKE, FAKE, None) == HG_ERR_INVALID_ARG
    assert lib.hg_hash_bucket(FAKE, 10, 0, 1 << 32, FAKE, FAKE, None) == HG_ERR_INVALID_ARG
    assert lib.hg_hash_bucket(None, 10, 0, 5, FAKE, FAKE, None) == HG_ERR_INVALID_ARG
    # nothing to do: no outputs requested, or no keys
    assert lib.hg_hash_bucket(FAKE, 10, 0, 5, None, None, None) == HG_OK
    assert lib.hg_hash_bucket(None, 0, 0, 5, FAKE, FAKE, None) == HG_OK


def test_table_calls_reject_null(lib):
    assert lib.hg_table_info(None, FAKE) == HG_ERR_INVALID_ARG
    assert lib.hg_table_export(None, None, None, None, None, None) == HG_ERR_INVALID_ARG
    lib.hg_table_free(None)  # no-op


def build_batched(lib, keys=FAKE, n=10, kt=0, T=3, offs=FAKE, P=1, num=1, den=1, V=0, flags=0, out=True,
                  opts=True, sub=0):
    o = Opts(P, num, den, flags, V, sub, 0)
    h = ctypes.c_void_p()
    return lib.hg_build_batched(keys, n, kt, T, offs, ctypes.byref(o) if opts else None, None,
                                ctypes.byref(h) if out else None)


@pytest.mark.parametrize("case, expected", [
    (dict(T=0), HG_ERR_INVALID_ARG),                        # no tables
    (dict(T=(1 << 22) + 1), HG_ERR_INVALID_ARG),            # too many tables
    (dict(offs=None), HG_ERR_INVALID_ARG),                  # null offsets
    (dict(keys=None), HG_ERR_INVALID_ARG),                  # null keys
    (dict(n=1 << 32), HG_ERR_INVALID_ARG),
    (dict(kt=5), HG_ERR_INVALID_ARG),
    (dict(P=16), HG_ERR_INVALID_ARG),                       # partitions are the tables
    (dict(V=100), HG_ERR_INVALID_ARG),                      # sizes come from the ratio
    (dict(num=0), HG_ERR_INVALID_ARG),
    (dict(flags=1), HG_ERR_UNSUPPORTED),                    # atomic build
    (dict(flags=8), HG_ERR_INVALID_ARG),
    (dict(n=(1 << 32) - 1, num=2), HG_ERR_INVALID_ARG),     # too many buckets
    (dict(out=False), HG_ERR_INVALID_ARG),
    (dict(opts=False), HG_ERR_INVALID_ARG),
    (dict(sub=15), HG_ERR_INVALID_ARG),
])
def test_build_batched_rejects(lib, case, expected):
    assert build_batched(lib, **case) == expected
    assert lib.hg_last_error().decode() != ""


def test_batched_probe_rejects(lib):
    assert lib.hg_count_batched(None, FAKE, 10, FAKE, FAKE, None) == HG_ERR_INVALID_ARG
    assert lib.hg_query_batched(None, FAKE, 10, FAKE, FAKE, None) == HG_ERR_INVALID_ARG


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
HG_OP_BUILD, HG_OP_COUNT, HG_OP_QUERY, HG_OP_BUILD_BATCHED, HG_OP_COUNT_BATCHED, HG_OP_QUERY_BATCHED = range(6)


def workspace(lib, op, n=0, kt=0, P=1, num=1, den=1, flags=0, V=0, aux=0, table=None):
    lib.hg_workspace_size.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                      ctypes.POINTER(Opts), ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64),
                                      ctypes.POINTER(ctypes.c_uint64)]
    o = Opts(P, num, den, flags, V)
    ws, tb = ctypes.c_uint64(7), ctypes.c_uint64(7)
    st = lib.hg_workspace_size(op, table, n, kt, ctypes.byref(o), aux, ctypes.byref(ws), ctypes.byref(tb))
    return st, ws.value, tb.value


def test_set_allocator_takes_both_functions_or_neither(lib):
    lib.hg_set_allocator.argtypes = [ALLOC_FN, FREE_FN, ctypes.c_void_p]
    assert lib.hg_set_allocator(ALLOC_FN(lambda n, s, c: None), FREE_FN(), None) == HG_ERR_INVALID_ARG
    assert lib.hg_set_allocator(ALLOC_FN(), FREE_FN(lambda p, n, s, c: None), None) == HG_ERR_INVALID_ARG
    assert lib.hg_set_allocator(ALLOC_FN(), FREE_FN(), None) == HG_OK  # the library's pool


@pytest.mark.parametrize("n, kt, P, num, den, V", [
    (0, 0, 1, 1, 1, 0), (1, 0, 16, 1, 1, 0), (5000, 1, 1, 1, 2, 0), (1 << 20, 0, 1, 0, 0, 1 << 20),
    (1 << 22, 0, 16, 1, 1, 0), (1 << 28, 0, 16, 1, 1, 0), (1 << 27, 1, 1, 1, 2, 0)])
def test_workspace_size_of_a_build_needs_no_device(lib, n, kt, P, num, den, V):
    """The dry run makes no HIP call.  The table keeps its keys, its offsets
    over floor(n * num / den) + P buckets (or V + 1) and a small metadata
    block, each rounded up to 256 bytes."""
    st, ws, tb = workspace(lib, HG_OP_BUILD, n=n, kt=kt, P=P, num=num, den=den, V=V)
    assert st == HG_OK, lib.hg_last_error()
    ks = 4 if kt == 0 else 8
    bound = V if V else n * num // den + P
    floor = n * ks + (bound + 1) * 4
    assert floor <= tb <= floor + 3 * 256 + (1 << 16)
    assert tb % 256 == 0 and ws % 256 == 0
    if n >= (1 << 22):  # sorted build: two split buffers of n keys at least
        assert ws >= 2 * n * ks


def test_workspace_size_grows_with_n(lib):
    prev = (0, 0)
    for n in [0, 1, 100, 4096, 1 << 16, 1 << 20, 1 << 24]:
        st, ws, tb = workspace(lib, HG_OP_BUILD, n=n, P=16)
        assert st == HG_OK
        assert tb >= prev[1]
        prev = (ws, tb)


def test_workspace_size_mirrors_the_calls_errors(lib):
    assert workspace(lib, HG_OP_BUILD, n=10, P=3)[0] == HG_ERR_INVALID_ARG
    assert workspace(lib, HG_OP_BUILD, n=10, P=512)[0] == HG_ERR_UNSUPPORTED
    assert workspace(lib, HG_OP_BUILD, n=1 << 32)[0] == HG_ERR_INVALID_ARG
    assert workspace(lib, HG_OP_BUILD, n=10, num=0)[0] == HG_ERR_INVALID_ARG
    assert workspace(lib, HG_OP_COUNT, n=10)[0] == HG_ERR_INVALID_ARG          # no table
    assert workspace(lib, HG_OP_QUERY_BATCHED, n=10)[0] == HG_ERR_INVALID_ARG  # no table
    assert workspace(lib, HG_OP_BUILD_BATCHED, n=10, aux=0)[0] == HG_ERR_INVALID_ARG  # no tables
    assert workspace(lib, 17)[0] == HG_ERR_INVALID_ARG
    st, ws, tb = workspace(lib, HG_OP_BUILD_BATCHED, n=1 << 20, aux=4096)
    assert st == HG_OK and tb >= (1 << 20) * 4 + ((1 << 20) + 4096 + 1) * 4


def test_bin_partition_balanced_rejects(lib):
    f = lib.hg_bin_partition_balanced
    f.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    ok = dict(keys=FAKE, n=10, kt=0, P=3, HR=1000, bins=0, out=FAKE, po=FAKE, sp=FAKE)

    def call(**kw):
        a = dict(ok, **kw)
        return f(a["keys"], a["n"], a["kt"], a["P"], a["HR"], a["bins"], a["out"], a["po"], a["sp"], None)

    assert call(P=0) == HG_ERR_INVALID_ARG
    assert call(P=257) == HG_ERR_INVALID_ARG
    assert call(HR=0) == HG_ERR_INVALID_ARG
    assert call(HR=1 << 32) == HG_ERR_INVALID_ARG
    assert call(bins=(1 << 14) + 1) == HG_ERR_INVALID_ARG
    assert call(n=1 << 32) == HG_ERR_INVALID_ARG
    assert call(kt=4) == HG_ERR_INVALID_ARG
    assert call(po=None) == HG_ERR_INVALID_ARG
    assert call(sp=None) == HG_ERR_INVALID_ARG
    assert call(keys=None) == HG_ERR_INVALID_ARG
    assert call(out=None) == HG_ERR_INVALID_ARG


def test_build_like_and_intersect_reject_null(lib):
    lib.hg_build_like.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                  ctypes.c_void_p]
    lib.hg_intersect.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    h = ctypes.c_void_p()
    assert lib.hg_build_like(None, FAKE, 10, None, ctypes.byref(h)) == HG_ERR_INVALID_ARG
    assert lib.hg_intersect(None, None, FAKE, None) == HG_ERR_INVALID_ARG
