"""FFST_LOG on the GPU path (a child process, since the log setting is read
once per process): level 2 logs the plan's creation with its sizes and
windows, every transform call with its schedule, the tuner's result, an
uneven batch with its size classes, and every destruction."""

import os
import re
import subprocess
import sys

import pytest

from gpu_helpers import log

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
import torch
from paper_1202_1773_amd import Plan, BatchPlan
plan = Plan(64, 64, 2)
x = torch.rand((2, 64, 64), device="cuda")
c = plan.forward(x)
y = plan.adjoint(c)
plan.tune(x)
torch.cuda.synchronize()
plan.close()
bp = BatchPlan([(64, 64), (48, 96), (64, 64)], [2, 2, 2])
bp.close()
print("child done", flush=True)
"""


def test_level_two_log(tmp_path):
    path = tmp_path / "ffst.log"
    log(f"FFST_LOG=2:{path} child process: plan, calls, tuner, batch")
    env = dict(os.environ, FFST_LOG=f"2:{path}")
    res = subprocess.run([sys.executable, "-c", CHILD, ROOT], env=env, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-3000:]
    assert "child done" in res.stdout
    text = path.read_text()
    log(text[:2000])
    m = re.search(r"plan (0x[0-9a-f]+): 64 x 64, J = 2, eta = 13, real Meyer shearlets", text)
    assert m, text[:1000]
    p = m.group(1)
    assert re.search(rf"plan {p} ffst_forward: 2 image\(s\), \d+ per unit, \d line\(s\) per column", text)
    assert re.search(rf"plan {p} ffst_adjoint: 2 image\(s\), \d+ per unit, \d line\(s\) per column", text)
    assert re.search(rf"plan {p} tuned for 2 image\(s\): nparts [1248], fwd_nparts [1248]", text)
    assert f"plan {p} destroyed" in text
    assert re.search(r"batch 0x[0-9a-f]+: 3 image\(s\) in 2 size class\(es\)", text)
    assert re.search(r"class 0: 2 image\(s\) of 64 x 64, J = 2", text)
    assert re.search(r"class 1: 1 image\(s\) of 48 x 96, J = 2", text)
    assert re.search(r"batch 0x[0-9a-f]+ destroyed", text)
    assert "error" not in text
