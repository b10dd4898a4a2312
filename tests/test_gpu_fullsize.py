"""GPU parity at the full workload sizes, against the oracle's digests.

The 2^28-key, 16-partition workload and the 2^27-key Zipf workload are
built and probed exactly as the benchmark times them (device-drawn inputs
of the same seeds, default knobs).  Their outputs are then compared with
the oracle's outputs at the same sizes through the digests of
``tests/golden/fullsize_digests.json``, written by
``tests/golden/fullsize.py`` from the oracle alone: partition offsets and
bucket bases raw, offsets and counts bit for bit (BLAKE2b), and bucket
contents as an order-free multiset hash of (bucket, key) pairs.  A sample
of 2^16 queries is also counted by the oracle one by one, on the spot.
"""

import importlib.util
import os

import numpy as np
import pytest

import oracle
from paper_2104_00792_amd import inputs

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _fullsize():
    spec = importlib.util.spec_from_file_location("fullsize", os.path.join(HERE, "golden", "fullsize.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name", ["p16_u32_2^28", "zipf_u64_2^27", "zipf_u32_2^28"])
def test_full_size_against_oracle_digest(gpu, name):
    import torch

    fs = _fullsize()
    want = fs.load()[name]
    dev = torch.device("cuda:0")
    keys, queries, opts = inputs.make_workload(name, device=dev)
    assert want["inputs"] == fs.inputs_id(name, keys.numel(), queries.numel())
    t = gpu.hg_build(keys, P=opts["P"], ratio=(opts["num"], opts["den"]))
    counts = gpu.hg_count(t, queries)
    po, bb, offs, tk = t.export()
    torch.cuda.synchronize()
    t.free()
    counts_h = counts.cpu().numpy()
    got = fs.digest(po.cpu().numpy(), bb.cpu().numpy(), offs.cpu().numpy(), tk.cpu().numpy(), counts_h)
    del offs, tk
    assert fs.compare(got, want) == {k: True for k in want if k != "inputs"}, (got, want)

    pick = (inputs.splitmix64(0xF055, 0, 1 << 16) % np.uint64(queries.numel())).astype(np.int64)
    keys_h = keys.cpu().numpy()
    with oracle.all_cores():
        ref = oracle.count(keys_h, queries.cpu().numpy()[pick])
    assert np.array_equal(counts_h[pick], ref)
