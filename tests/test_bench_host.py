"""Host-side logic of bench.py, on the CPU: the one-GPU guard, the
algorithmic bytes per launch (the per-unit figures of the kernel table), and
that counter figures are reported only for the kernel sources they were
taken on."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("args, env", [(["--gpus", "2"], {}), (["--gpus", "1"], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(args, env):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                       timeout=120, env=dict(os.environ, **env))
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_bytes_per_unit_of_each_launch():
    n = q = B = 1 << 20
    per = lambda k, ks=4: bench.algorithmic_bytes(k, n, q, B, ks, 16) / n  # noqa: E731
    assert per("part_count") == 4 and per("split1_count") == 4 and per("split2_count") == 4
    assert per("split1_scatter") == 8 and per("split2_scatter") == 8
    assert per("lds_build") == 12                      # key in, key out, offset out (B == n)
    assert per("qsplit1_scatter") == 10 and per("qsplit2_scatter") == 10
    assert per("lds_probe") == 16                      # query, offset, table key, count
    assert per("qgather1") == 10 and per("qgather2") == 10
    assert per("lds_build", ks=8) == 20 and per("lds_probe", ks=8) == 24
    assert bench.algorithmic_bytes("no_such_launch", n, q, B, 4, 16) == 0.0


def test_headline_step_moves_104_bytes_per_key_and_query():
    n = q = B = 1 << 28
    launches = ["part_count", "split1_count", "split1_scatter", "split2_count", "split2_scatter", "lds_build",
                "qsplit1_count", "qsplit1_scatter", "qsplit2_count", "qsplit2_scatter", "lds_probe", "qgather2",
                "qgather1"]
    total = sum(bench.algorithmic_bytes(k, n, q, B, 4, 16) for k in launches)
    assert total == 104 * n


def test_narrow_counts_take_92_bytes_per_pair():
    """Without long buckets the probe passes its counts as bytes: the probe
    writes 1 B instead of 4, the level-2 gather moves 2 + 1 + 1, the last
    gather 2 + 1 + 4."""
    n = q = B = 1 << 28
    launches = ["part_count", "split1_count", "split1_scatter", "split2_count", "split2_scatter", "lds_build",
                "qsplit1_count", "qsplit1_scatter", "qsplit2_count", "qsplit2_scatter", "lds_probe", "qgather2",
                "qgather1"]
    assert sum(bench.algorithmic_bytes(k, n, q, B, 4, 16, cb=1) for k in launches) == 92 * n
    assert bench.algorithmic_bytes("qgather2", n, q, B, 4, 16, cb=1) == 4 * q
    assert bench.algorithmic_bytes("qgather1", n, q, B, 4, 16, cb=1) == 7 * q


@pytest.mark.parametrize("P, per_pair", [(16, 60), (1, 48)])
def test_model_bytes_per_step_and_per_kernel(P, per_pair):
    """The scope table's model: 28 B per key (partition count 4, scatter 8,
    local histogram 4, offsets 4, local scatter 8) + 32 B per query for the
    partitioned build; 16 + 32 for a plain table.  The per-kernel charges
    add up to the step's bytes, and the dominant probe pass is charged
    8 B per query."""
    n = q = B = 1 << 24
    launches = ["part_count", "split1_count", "split1_scatter", "split2_count", "split2_scatter", "lds_build",
                "qsplit1_count", "qsplit1_scatter", "qsplit2_count", "qsplit2_scatter", "lds_probe", "qgather2",
                "qgather1"]
    assert bench.survey_step_bytes(n, q, B, 4, P) == per_pair * n
    assert sum(bench.survey_bytes(k, n, q, B, 4, P) for k in launches) == per_pair * n
    assert bench.survey_bytes("lds_probe", n, q, B, 4, P) == 8 * q
    # 64-bit keys, V = n / 2 (the Zipf workload): 8 + 2 + 16 per key, 52 per query
    assert bench.survey_step_bytes(n, q, n // 2, 8, 1) == 78 * n


def test_traffic_is_read_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.read_traffic("w", "lds_probe") is None  # no summary at all
    prof = tmp_path / "profiles"
    prof.mkdir()
    f = prof / "traffic_w.txt"
    f.write_text(f"# comment\nkernel_source_sha256_16 = {bench.kernel_source_hash()}\n"
                 "hbm_bytes_per_launch.lds_probe = 4319000000\n")
    assert bench.read_traffic("w", "lds_probe") == 4319000000.0
    assert bench.read_traffic("w", "qgather1") is None  # kernel not in the summary
    f.write_text("kernel_source_sha256_16 = 0000000000000000\nhbm_bytes_per_launch.lds_probe = 4319000000\n")
    assert bench.read_traffic("w", "lds_probe") is None  # taken on other sources


def test_launch_share_is_the_step_outside_its_launch_groups():
    kernels = {"a": {"ms_per_step": 1.0, "launches_per_step": 2}, "b": {"ms_per_step": 2.5, "launches_per_step": 1}}
    share = bench.launch_share(kernels, 4.0)
    assert share["launch_groups_per_step"] == 3 and share["kernel_ms_per_step"] == 3.5
    assert share["between_launches_ms"] == 0.5 and share["between_frac"] == 0.125
    assert bench.launch_share(kernels, 3.0)["between_launches_ms"] == 0.0  # event overhead can exceed the gaps


def test_duplicate_study_workload():
    """The duplicate-study sweep runs on the headline's keys, from one key
    per bucket up to 4096, and names itself among the bench workloads."""
    assert "dup_sweep_u32_2^28" in bench.DESCRIPTIONS
    occ = bench.DUP_OCCUPANCIES
    assert occ[0] == 1 and occ[-1] == 4096 and list(occ) == sorted(set(occ))
    assert all(o & (o - 1) == 0 for o in occ)  # V_p = n_p / occ stays exact for n_p a power of two
