"""Host-side checks of bench.py (no GPU): the one-GPU contract, the algorithmic byte counts and
the committed rocprofv3 summaries it reads its traffic figure from."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_per_voxel():
    """Per pore voxel and step: 19 f read and written, 8 moment slots read and written, phi and
    N written then read, 24 neighbour entries (6 in the phase kernel, 18 in the collide)."""
    b64 = bench.launch_bytes("fp64", False, 1000, (8, 8, 8))["per_voxel"]
    b32 = bench.launch_bytes("fp32dev", False, 1000, (8, 8, 8))["per_voxel"]
    assert (b64["collide"], b64["phase"], b64["step"]) == (456, 104, 560)
    assert (b32["collide"], b32["phase"], b32["step"]) == (264, 64, 328)
    rank = bench.launch_bytes("fp64", True, 1000, (8, 8, 64))
    assert rank["per_voxel"]["step"] == 8 * 58 + 8
    assert rank["row_bytes"] == 8 * 8 * 1 * 32


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_committed_profiles_describe_the_current_kernels(precision):
    """The traffic figure bench.py reports comes from the committed summary only while it was
    measured on the current kernel source."""
    src = os.path.join(ROOT, "paper_2007_12266_amd", "csrc", "lbm_kernels.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    prof = open(os.path.join(ROOT, "profiles", "collide_phase_grf256_%s.md" % precision)).read()
    assert "kernel_source_sha256_prefix: " + digest[:16] in prof
    t = bench._profiled_traffic(precision, "table")
    assert t is not None and t > bench.launch_bytes(precision, False, 1, (1, 1, 1))[
        "per_voxel"]["collide"] * 0.9
    assert bench._profiled_traffic(precision, "rank") is None
