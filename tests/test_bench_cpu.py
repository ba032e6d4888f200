"""The benchmark's host-side contract (CPU only): one GPU only, and the calibrated HBM traffic of
the fused CG kernel is reported only for the kernel source it was measured on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_exits_with_a_message(argv, env):
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, cwd=ROOT,
                         env=dict(os.environ, **env), capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr and res.stdout == ""


def test_kernel_hash_covers_exactly_the_fused_cg_template():
    src = open(os.path.join(ROOT, "paper_2506_18867_amd", "csrc", "solve.hip")).read()
    a = src.index("template <typename T, bool FIRST>")
    assert "k_cg_fused(DevSheet S" in src[a:a + 300]
    assert len(bench.cg_kernel_sha()) == 16


def test_traffic_is_null_once_the_kernel_changes(monkeypatch):
    t = dict(bench.CG_TRAFFIC)
    monkeypatch.setattr(bench, "cg_kernel_sha", lambda: t["kernel_sha256_16"])
    expect = int(1024 * (t["fetch_kib"] / t["fetch_factor"] + t["write_kib"] / t["write_factor"]))
    assert bench.cg_traffic_bytes() == expect
    monkeypatch.setattr(bench, "cg_kernel_sha", lambda: "0" * 16)
    assert bench.cg_traffic_bytes() is None
