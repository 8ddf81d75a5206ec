"""bench.py host logic on the CPU: the committed traffic records parse and are
found for their own source hash, the multi-GPU request exits cleanly, and the
library CPU baseline computes the transform the oracle computes."""

import json
import os
import subprocess
import sys

import numpy as np

import bench
from oracle import spectra as ospec
from oracle import transform as otr
from paper_1202_1773_amd.synthetic import cartoon

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILE = os.path.join(ROOT, "profiles", "traffic_ffst_512x512_J3_B16.md")


def test_traffic_records_parse_and_match_their_hash(monkeypatch):
    recs = [json.loads(line[len("TRAFFIC "):]) for line in open(PROFILE) if line.startswith("TRAFFIC {")]
    assert recs, "no traffic records"
    for r in recs:
        assert {"kernel", "source_sha", "workload", "bytes_per_launch"} <= set(r)
        assert r["bytes_per_launch"] > 0
    rec = recs[0]
    monkeypatch.setattr(bench, "source_sha", lambda: rec["source_sha"])
    assert bench.committed_traffic(rec["kernel"], *rec["workload"]) == rec["bytes_per_launch"]
    monkeypatch.setattr(bench, "source_sha", lambda: "0" * 16)
    assert bench.committed_traffic(rec["kernel"], *rec["workload"]) is None


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr


def test_library_baseline_matches_the_oracle():
    M, N, J = 64, 48, 2
    psi = ospec.spectra(M, N, J)
    imgs = [cartoon(M, N, 8, 3, 0.1, seed=60 + b).astype(np.float64) for b in range(2)]
    c, y = bench.library_transform(np.stack(imgs), psi[:, :, : N // 2 + 1], M, N, 2)
    for b, f in enumerate(imgs):
        ref = otr.forward(f, psi)
        assert np.abs(c[b] - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.abs(y[b] - f).max() <= 1e-12 * np.abs(f).max()
    out = bench.cpu_library(psi[:, :, : N // 2 + 1].astype(np.float32), imgs, M, N, reps=1)
    assert out["f64"] > 0 and out["f32"] > 0
    assert out["f64_reconstruction_rel_l2"] < 1e-6 and out["f32_reconstruction_rel_l2"] < 1e-5
