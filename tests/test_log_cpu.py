"""FFST_LOG, the library's text log (read once per process, so every case
runs in a child process): errors are logged at level 1 with their status and
message, a bare path means level 1 into that file, 0 turns it off. The plan,
tuning and per-call lines need a GPU (tests/test_gpu_log.py)."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import ctypes, sys
sys.path.insert(0, sys.argv[1])
from paper_1202_1773_amd import _lib
lib = _lib.load()
plan = ctypes.c_void_p()
assert lib.ffst_spectra(320, 512, 3, ctypes.byref(plan)) == _lib.FFST_EUNSUPPORTED
opt = _lib.ffst_options(0, 0, 0, 11)
assert lib.ffst_spectra_ex(64, 64, 2, ctypes.byref(opt), ctypes.byref(plan)) == _lib.FFST_EINVAL
print("child done")
"""


def _run(tmp_path, value):
    env = dict(os.environ)
    if value is None:
        env.pop("FFST_LOG", None)
    else:
        env["FFST_LOG"] = value
    res = subprocess.run([sys.executable, "-c", CHILD, ROOT], env=env, capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    assert "child done" in res.stdout
    return res


def test_errors_go_to_the_log_file(tmp_path):
    log = tmp_path / "ffst.log"
    _run(tmp_path, f"1:{log}")
    lines = log.read_text().splitlines()
    assert len(lines) == 2, lines
    assert all(line.startswith("ffst[") for line in lines)
    assert "error 2: GPU path supports sides" in lines[0] and "320 x 512" in lines[0]
    assert "error 1: aux_order" in lines[1]


def test_bare_path_is_level_one(tmp_path):
    log = tmp_path / "bare.log"
    _run(tmp_path, str(log))
    assert log.read_text().count("error ") == 2


def test_off_and_stderr(tmp_path):
    res = _run(tmp_path, "0")
    assert "ffst[" not in res.stderr
    res = _run(tmp_path, None)
    assert "ffst[" not in res.stderr
    res = _run(tmp_path, "1")
    assert res.stderr.count("ffst[") == 2 and "aux_order" in res.stderr


def test_library_links_the_roctx_ranges():
    from paper_1202_1773_amd import _lib
    out = subprocess.run(["readelf", "-d", _lib.LIB_PATH], capture_output=True, text=True).stdout
    assert "rocprofiler-sdk-roctx" in out
