"""Host-side checks of bench.py (no GPU): the one-GPU contract, the algorithmic byte counts and
the committed rocprofv3 summaries it reads its traffic figure from."""
import hashlib
import os
import subprocess
import sys


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
    N written then read, 24 neighbour entries (6 in the phase kernel, 18 in the collide); f in
    the first storage width, the rest in the second (FP64 8/8, FP32-dev 4/4, FP32-mixed 4/8)."""
    per = {p: bench.launch_bytes(p, "table", 1000, (8, 8, 8))["per_voxel"]
           for p in ("fp64", "fp32dev", "mixed")}
    assert (per["fp64"]["collide"], per["fp64"]["phase"], per["fp64"]["step"]) == (456, 104, 560)
    assert (per["fp32dev"]["collide"], per["fp32dev"]["phase"], per["fp32dev"]["step"]) == \
        (264, 64, 328)
    assert (per["mixed"]["collide"], per["mixed"]["phase"], per["mixed"]["step"]) == \
        (304, 104, 408)
    rank = bench.launch_bytes("fp64", "rank", 1000, (8, 8, 64))
    assert rank["per_voxel"]["step"] == 8 * 58 + 8
    assert rank["row_bytes"] == 8 * 8 * 1 * 32
    # Compact lookup over 640 voxels (10 waves), 2 of them exception waves: records for 512
    # voxels (40 B collide, 16 B phase), int32 entries for 128 (72 / 24 B), wave bases read
    # (37 / 13 ints per wave).
    c = bench.launch_bytes("fp64", "compact", 640, (8, 8, 10), ex_waves=2)
    assert c["collide"] == 640 * 384 + 512 * 40 + 128 * 72 + 10 * 148
    assert c["phase"] == 640 * 80 + 512 * 16 + 128 * 24 + 10 * 52
    assert c["row_bytes"] == 0
    # The survey's accounting: the 14 D3Q7 populations instead of their 8 moments, the table
    # once per step.
    assert bench.survey_bytes("fp64") == {"step": 632, "collide": 504}
    assert bench.survey_bytes("fp32dev") == {"step": 352, "collide": 288}
    assert bench.survey_bytes("mixed") == {"step": 480, "collide": 352}


def test_committed_profile_describes_the_current_kernels():
    """The traffic figure of the default (512^3 displacement, FP64) line comes from the committed
    counter summary only while it was measured on the current kernel source."""
    src = os.path.join(ROOT, "paper_2007_12266_amd", "csrc", "lbm_kernels.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    prof = open(os.path.join(ROOT, "profiles", "collide_phase_disp512_fp64.md")).read()
    assert "kernel_source_sha256_prefix: " + digest[:16] in prof
    t = bench._profiled_traffic("disp512", "fp64", "compact")
    assert t is not None and t > bench.launch_bytes("fp64", "compact", 64, (1, 1, 64))[
        "per_voxel"]["collide"] * 0.9
    assert bench._profiled_traffic("disp512", "fp64", "rank") is None
    assert bench._profiled_traffic("disp512", "fp64", "table") is None
