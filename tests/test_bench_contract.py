"""bench.py's host-side contract (no GPU): the one-GPU limit, and the
roofline arithmetic it reports."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_per_kernel_rate():
    import bench
    k = bench.per_kernel("k", ms=2000.0, nbytes=8e12, launches=4, steps=2)
    assert k["ms_per_step"] == 1000.0
    assert k["bytes_per_launch"] == 2_000_000_000_000
    assert abs(k["achieved"] - 4000.0) < 1e-6  # 8e12 B in 2 s = 4000 GB/s
    assert abs(k["frac"] - 0.5) < 1e-9          # of 8 TB/s


def test_counter_records_are_tied_to_the_kernel_sources():
    import bench
    # a kernel the record was not taken for never gets its figures
    assert bench.measured_traffic("plane3d_1m", "no_such_kernel") is None
    assert bench.measured_valu("pose4dof_1m", "no_such_kernel") is None
    assert bench.measured_traffic("no_such_workload", "k_compact_lin<PLANE3D>") is None


def test_valu_fraction():
    import bench
    # 39.3216e12 lane-ops/s peak: 10 lane-ops per test over 3.93216e12 tests in 1 s is the peak
    assert abs(bench.valu_frac(10.0, 3.93216e12, 1000.0) - 1.0) < 1e-9
    assert bench.valu_frac(10.0, 1e9, 0.0) is None
