"""Host-side checks of bench.py (no GPU needed): the committed counter
summaries it reads, the valid-window count it prices pairs with, and its
refusal of more than one GPU."""
import hashlib
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

KERNEL = os.path.join(ROOT, "paper_2112_12965_amd", "csrc", "join_fp32.hip")


def test_profiled_field_only_for_the_profiled_source(tmp_path):
    src = tmp_path / "k.hip"
    src.write_text("kernel one\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    summary = tmp_path / "s.md"
    summary.write_text(f"# t\n\nkernel_source_sha256: {sha}\ntraffic_bytes_per_launch: 1234\n")
    assert bench.profiled_field(str(src), str(summary), "traffic_bytes_per_launch") == 1234.0
    assert bench.profiled_field(str(src), str(summary), "missing_field") is None
    src.write_text("kernel two\n")  # the kernel changed since the counters were taken
    assert bench.profiled_field(str(src), str(summary), "traffic_bytes_per_launch") is None
    assert bench.profiled_field(str(src), str(tmp_path / "absent.md"), "traffic_bytes_per_launch") is None


@pytest.mark.parametrize("seed", range(5))
def test_valid_windows_brute_force(seed):
    rng = np.random.default_rng(seed)
    lens = rng.integers(1, 40, int(rng.integers(1, 8)))
    bounds = np.concatenate([[0], np.cumsum(lens)])
    m = int(rng.integers(1, 20))
    # a window [j, j + m) is valid iff it lies inside one segment (Def. 8)
    brute = sum(1 for j in range(int(bounds[-1]) - m + 1)
                if any(bounds[s] <= j and j + m <= bounds[s + 1] for s in range(len(bounds) - 1)))
    assert bench.valid_windows(bounds, m) == brute


@pytest.mark.parametrize("workload", [bench.DICT_WORKLOAD, "rw1m_m128"])
def test_committed_counters_match_the_kernel_source(workload):
    # the bench reports HBM traffic and the FMA-class issue fraction only while
    # the committed summaries were taken on the current kernel source
    kinds = ["valu_types", "hbm"]
    for kind in kinds:
        summary = os.path.join(ROOT, "profiles", f"k_join_fp32_{workload}_{kind}_counters.md")
        text = open(summary).read()
        assert "rocprofv3 " in text  # the command that made it
        field = "traffic_bytes_per_launch" if kind == "hbm" else "fma_class_lane_instructions_per_pair"
        v = bench.profiled_field(KERNEL, summary, field)
        assert v is not None and v > 0, f"{summary} was taken on another version of {KERNEL}: profile again"


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


@pytest.mark.parametrize("tier", ["bf16", "fp16"])
@pytest.mark.parametrize("workload", [bench.DICT_WORKLOAD, "rw1m_m128"])
def test_committed_matrix_core_counters_match_the_kernel_source(tier, workload):
    src = os.path.join(ROOT, "paper_2112_12965_amd", "csrc", "join_mfma.hip")
    for kind, field in (("hbm", "traffic_bytes_per_launch"), ("mfma", "mfma_busy_frac")):
        summary = bench.summary_path(tier, workload, kind)
        assert "rocprofv3 " in open(summary).read()
        v = bench.profiled_field(src, summary, field)
        assert v is not None and v > 0, f"{summary} was taken on another version of {src}: profile again"
