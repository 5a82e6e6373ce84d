"""PyTorch as the source of device memory and streams.

The boundary takes plain device pointers and an optional HIP stream, so
torch tensors (float64, contiguous, on the GPU) can be handed to the library
as observation columns, and torch's stream can be the one the library runs
on: the columns are written by torch on that stream and read by the search
after them, with no other synchronization.  Results equal the oracle's.

torch ships its own HIP runtime under the same soname as the system's, and
whichever is loaded first serves the process.  torch initializes only on its
own, so the check runs in a child process that imports torch before the
library is loaded.
"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
import numpy as np
import torch
if not torch.cuda.is_available():
    print("SKIP no GPU visible to torch", flush=True)
    sys.exit(0)
import oracle
from paper_2107_11810_amd import gvote, synth
for name in ("plane3d_small", "pose4dof_small"):
    g = synth.config(name)
    ro = oracle.solve(oracle.Problem(g["family"], g["cols"], g["lo"], g["hi"], g["eps"]))
    s = torch.cuda.Stream()  # default priority
    with torch.cuda.stream(s):
        cols = [torch.from_numpy(np.ascontiguousarray(c, dtype=np.float64)).to("cuda") for c in g["cols"]]
    c = gvote.Context(0, hip_stream=s.cuda_stream)
    try:
        r = c.solve(g["family"], cols, g["lo"], g["hi"], g["eps"])
    finally:
        c.close()
    torch.cuda.synchronize()
    ok = (r["count"] == ro["count"] and r["leaf_index"] == ro["leaf_index"] and r["sector"] == ro["sector"]
          and np.array_equal(r["inliers"], ro["inliers"]))
    # the columns are borrowed, not changed
    ok = ok and all(np.array_equal(t.cpu().numpy(), np.asarray(a, dtype=np.float64)) for t, a in zip(cols, g["cols"]))
    print(name, "count", r["count"], "oracle", ro["count"], "ok", ok, flush=True)
    if not ok:
        sys.exit(1)
print("DONE", flush=True)
"""


def test_torch_columns_on_a_torch_stream():
    print("torch interop child", flush=True)
    env = dict(os.environ)
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    p = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=240)
    print(p.stdout, p.stderr[-2000:], flush=True)
    if p.returncode == 0 and p.stdout.startswith("SKIP"):
        pytest.skip(p.stdout.strip())
    assert p.returncode == 0, p.stderr[-2000:]
    assert "DONE" in p.stdout
