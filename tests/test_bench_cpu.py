"""bench.py host logic on the CPU: the committed traffic records parse and are
found for their own source hash, and the multi-GPU request exits cleanly."""

import json
import os
import subprocess
import sys

import bench

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
