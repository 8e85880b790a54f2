"""The library loaded before anything has imported torch: the binding imports
torch first, so that libgfo binds to the HIP runtime that torch's wheel brings
(the one that owns torch's memory and streams) rather than loading the system
copy beside it; the first entry points then launch normally."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_SCRIPT = r"""
import sys
sys.path.insert(0, {root!r})
sys.path.insert(0, {tests!r})
from paper_2202_05388_amd import _lib as L
L.lib()                                  # before any import of torch in this process
print("[case] library loaded before torch was imported", flush=True)
import numpy as np
import torch
import workloads as W
from paper_2202_05388_amd.job import Job
p = W.tiny(12, 14, n_mon=4, dtype="c64")
job = Job(p, device="cuda:0")
job.init()
job.score()
job.apply()
for t, j in enumerate((3, 40, 77)):
    job.set_pick(j, 1, slot=t)
job.apply_rank_k(3)
torch.cuda.synchronize()
assert job.status() == 0
print("ok", flush=True)
"""


def test_entry_points_after_early_load():
    script = _SCRIPT.format(root=ROOT, tests=os.path.join(ROOT, "tests"))
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    print(r.stderr[-2000:])
    assert r.returncode == 0
    assert r.stdout.strip().endswith("ok")
