"""The packed 8-byte list entries of the linear families, checked on the
host: exact round trips inside the field limits, overflow flagged outside.
(The device kernels use the same header functions.)"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_packed_entries_round_trip(tmp_path):
    exe = str(tmp_path / "pack_check")
    src = os.path.join(HERE, "host", "pack_check.cpp")
    subprocess.run([HIPCC, "-std=c++17", "-O1", "-o", exe, src], check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("OK")
