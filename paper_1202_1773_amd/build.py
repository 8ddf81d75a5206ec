"""Build libffst.so (the HIP kernels and the C ABI) in-tree for gfx950.

    python -m paper_1202_1773_amd.build          # or build() from Python

Every call recompiles: each source to an object file (in parallel), then one
link. Packed FP32 instructions are disabled for all device code
(-Xclang -target-feature -Xclang -packed-fp32-ops).
"""

import hashlib
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libffst.so")
SOURCES = ["spectra.hip", "transform_rows.hip", "transform_cols.hip", "complex.hip", "api.hip", "batch.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]
NOISE = "packed-fp32-ops"


# Host code that launches no kernel of a single-size plan: the uneven-batch
# driver (it replays the plans' own launches in a graph).
NOT_KERNEL_SOURCES = ("batch.hip",)


def source_sha():
    """Short hash of the sources the kernels and their launch settings come
    from (csrc/*.hip and csrc/*.hpp but the uneven-batch driver), to tie
    measurements to the code they were taken on."""
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp")) and f not in NOT_KERNEL_SOURCES)
    for name in files:
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if NOISE not in l)
    return res.returncode, err


def build(verbose=False):
    with tempfile.TemporaryDirectory(prefix="ffst_build_") as tmpdir:
        objs, cmds = [], []
        for s in SOURCES:
            obj = os.path.join(tmpdir, s.replace(".hip", ".o"))
            objs.append(obj)
            cmds.append([HIPCC, *FLAGS, "-c", os.path.join(CSRC, s), "-o", obj])
        jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        with ThreadPoolExecutor(jobs) as pool:
            results = list(pool.map(_run, cmds))
        for cmd, (rc, err) in zip(cmds, results):
            if verbose:
                print(" ".join(cmd), flush=True)
            if rc != 0:
                raise RuntimeError("hipcc failed:\n" + err)
            if verbose and err.strip():
                print(err, file=sys.stderr)
        tmp = LIB + ".tmp"
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        rc, err = _run(link)
        if rc != 0:
            raise RuntimeError("link failed:\n" + err)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
