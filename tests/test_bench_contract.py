"""bench.py on the host: the one-GPU refusal, the kernel source digests the
traffic records are keyed on, and the algorithmic bytes of one launch."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("kernel_file", sorted(bench.KERNEL_SOURCES))
def test_kernel_source_digest(kernel_file):
    d = bench.kernel_source_digest(kernel_file)
    assert d is not None and len(d) == 64
    assert d == bench.kernel_source_digest(kernel_file)   # stable
    assert bench.kernel_source_digest("no_such_kernel.hip") is None


def test_traffic_record_needs_matching_source():
    # a workload that no record names has no counter traffic
    assert bench.traffic_for("pair_mfma.hip", "no-such-workload", "fp16", 11) is None


class _Info:
    spectrum_elem_bytes = 4


class _Plan:
    info = _Info()
    M, N, P = 16, 512, 120


def test_kernel_bytes_per_launch():
    L, T = 960000, 7497
    kb = bench.kernel_bytes(_Plan(), L, T)
    spec = T * 16 * 256 * 4
    assert kb["stft_phat"] == 16 * L * 4 + spec          # audio read once, spectra written once
    assert kb["pair"] == spec + T * 120 * 4              # spectra read once, one int32 per pair-frame


def test_busy_record_needs_matching_source():
    assert bench.busy_for("pair_mfma.hip", "no-such-workload", "fp16", 11) is None


def test_cpu_baseline_small(tmp_path):
    """The CPU oracle baseline on a short recording: every frame, stated
    cores, CPU model and a median of the passes."""
    from gen import make_recording
    rec = make_recording(1)                       # 1 s, 4 mics: 122 frames
    r = bench.cpu_baseline(rec, 4, 9, workers=2, runs=3, chunk=64)
    assert r["kind"] == "oracle" and r["cores"] == 2 and len(r["runs_s"]) == 3
    assert r["value"] > 0 and r["cpu_model"] and r["nproc"] >= 1
    assert "all 122 frames" in r["sample"]


def test_workload_option():
    """--workload high-rate selects the 48 kHz workload for profiling; the
    default stays the benchmark workload (rank chosen in main when 0)."""
    old = sys.argv
    try:
        sys.argv = ["bench.py"]
        a = bench.parse_args()
        assert a.workload == "benchmark" and a.rank == 0
        sys.argv = ["bench.py", "--workload", "high-rate", "--rank", "29"]
        a = bench.parse_args()
        assert a.workload == "high-rate" and a.rank == 29
    finally:
        sys.argv = old
