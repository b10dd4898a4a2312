"""The library's per-launch event timing: every launch bracketed, or only
the launches of one name (what the bench times its steps with)."""

import numpy as np
import pytest

from paper_2104_00792_amd import inputs

pytestmark = pytest.mark.gpu


def test_profile_only_brackets_the_named_launches(gpu):
    import torch

    hg = gpu
    n = (1 << 22) + 5  # sorted build and sorted probe
    raw = inputs.uniform_u32(n, 0x51)
    keys = torch.from_numpy(raw).to("cuda")
    queries = torch.from_numpy(inputs.queries_hit50(raw, n, 0x52)).to("cuda")

    def step():
        t = hg.hg_build(keys, P=16)
        c = hg.hg_count(t, queries)
        t.free()
        return c

    with hg.profile() as every:
        want = step()
        torch.cuda.synchronize()
    assert "lds_probe" in every.results and "lds_build" in every.results
    assert len(every.results) > 5
    with hg.profile(only="lds_probe") as one:
        got = step()
        torch.cuda.synchronize()
    assert set(one.results) == {"lds_probe"}
    assert one.results["lds_probe"][0] == every.results["lds_probe"][0]
    assert one.results["lds_probe"][1] > 0.0
    assert np.array_equal(got.cpu().numpy(), want.cpu().numpy())
    # the filter ends with the context: every launch is bracketed again
    with hg.profile() as again:
        step()
        torch.cuda.synchronize()
    assert set(again.results) == set(every.results)
