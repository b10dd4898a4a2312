"""hg_bin_partition_noalloc against hg_bin_partition, through the C ABI.

The no-allocation variant keeps its tile counts in a fixed scratch array
of the library instead of allocated workspace.  Two calls in a row (the
second with fewer keys, so scratch left by the first lies beyond what the
second writes) must each give exactly what hg_bin_partition gives on the
same keys: part_offsets raw and the keys of every partition as a multiset
(the order inside a partition is open), and both must equal the oracle's
split.  Neither call may allocate: the library's allocator hook counts
every block it is asked for.
"""

import numpy as np
import pytest

import oracle
from paper_2104_00792_amd import inputs

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("dtype, P, sizes", [
    (np.uint32, 16, [(1 << 22) + 1234, 70001]),
    (np.uint64, 256, [300007, 4097]),
    (np.uint32, 1, [100000, 0]),
])
def test_noalloc_matches_bin_partition(gpu, dtype, P, sizes):
    import torch

    hg = gpu
    gen = inputs.uniform_u32 if dtype == np.uint32 else inputs.uniform_u64
    asked = []

    def alloc(nbytes, stream):
        asked.append(nbytes)
        return 0  # any allocation would fail the call

    def free(ptr, nbytes, stream):
        pass

    for k, n in enumerate(sizes):
        keys_np = gen(n, 0xA110C + k)
        keys = _dev(keys_np)
        ref_out, ref_po = hg.hg_bin_partition(keys, P)
        out = torch.full_like(keys, 7) if n else torch.empty_like(keys)
        po = torch.full((P + 1,), 0xFFFFFFFF, dtype=torch.uint32, device="cuda")
        hg.hg_set_allocator(alloc, free)
        try:
            hg.hg_bin_partition_noalloc(keys, P, out, po)
        finally:
            hg.hg_set_allocator()
        torch.cuda.synchronize()
        assert asked == [], f"call {k} asked the allocator for {asked}"
        got_po = po.cpu().numpy()
        assert np.array_equal(got_po, ref_po.cpu().numpy()), f"call {k}: part_offsets"
        canon = oracle.canonicalize(got_po, out.cpu().numpy())
        assert np.array_equal(canon, oracle.canonicalize(got_po, ref_out.cpu().numpy())), f"call {k}: keys"
        opo, okeys = oracle.bin_partition(keys_np, P)
        assert np.array_equal(got_po, opo) and np.array_equal(canon, okeys), f"call {k}: oracle"
