"""Build libffst.so (the HIP kernels and the C ABI) in-tree for gfx950.

    python -m paper_1202_1773_amd.build              # or build() from Python
    python -m paper_1202_1773_amd.build --sanitize   # libffst_asan.so

Every call recompiles: each source to an object file (in parallel), then one
link. Packed FP32 instructions are disabled for all device code
(-Xclang -target-feature -Xclang -packed-fp32-ops).

--sanitize builds the same sources into libffst_asan.so with AddressSanitizer
and UndefinedBehaviorSanitizer on the HOST code only (every -fsanitize= flag
behind -Xarch_host; the GPU code is built as usual). Load it with the ASan
runtime preloaded and FFST_LIBRARY pointing at it
(tests/test_sanitizers_cpu.py does this for the CPU tests of the C ABI).
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
LIB_ASAN = os.path.join(HERE, "libffst_asan.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ffst.h")
SOURCES = ["spectra.hip", "transform_rows.hip", "transform_cols.hip", "complex.hip", "api.hip", "batch.hip",
           "trace.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]
NOISE = "packed-fp32-ops"
LIBS = ["-lrocprofiler-sdk-roctx"]   # roctx ranges (trace.hip)
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
SANITIZE_LINK = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan"]


def asan_runtime():
    """Path of the compiler's shared ASan runtime (to preload), or None."""
    res = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = res.stdout.strip()
    if res.returncode == 0 and os.path.isabs(path) and os.path.exists(path):
        return path
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


# Host code that launches no kernel of a single-size plan: the uneven-batch
# driver (it replays the plans' own launches in a graph) and the log / roctx
# tracing.
NOT_KERNEL_SOURCES = ("batch.hip", "trace.hip")


def source_sha():
    """Short hash of the sources the kernels and their launch settings come
    from (csrc/*.hip and csrc/*.hpp but the uneven-batch driver), to tie
    measurements to the code they were taken on. Comments and blank lines
    are left out, so that editing a comment keeps a measurement valid."""
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp")) and f not in NOT_KERNEL_SOURCES)
    for name in files:
        with open(os.path.join(CSRC, name)) as fh:
            code = _strip_comments(fh.read())
        h.update(name.encode() + b"\0" + code.encode())
    return h.hexdigest()[:16]


def _strip_comments(text):
    """C++ source without // and /* */ comments and without blank lines
    (string and character literals are kept as they are)."""
    out, i, n = [], 0, len(text)
    while i < n:
        ch = text[i]
        if ch in "\"'":
            j = i + 1
            while j < n and text[j] != ch:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(ch)
            i += 1
    lines = (line.rstrip() for line in "".join(out).split("\n"))
    return "\n".join(line for line in lines if line)


def build_id():
    """Hash of everything libffst.so is compiled from: every file under csrc/,
    the public header and the compiler flags. It is compiled into the library
    (ffst_build_id) and compared with the tree by _lib.load(), so a library
    built from other sources cannot be loaded silently."""
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp", ".h")))
    paths = [os.path.join(CSRC, f) for f in files] + [HEADER]
    for path in paths:
        with open(path, "rb") as fh:
            h.update(os.path.basename(path).encode() + b"\0" + fh.read())
    h.update(" ".join(FLAGS).encode())
    return h.hexdigest()[:16]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if NOISE not in l)
    return res.returncode, err


def build(verbose=False, sanitize=False):
    extra = SANITIZE if sanitize else []
    out_lib = LIB_ASAN if sanitize else LIB
    with tempfile.TemporaryDirectory(prefix="ffst_build_") as tmpdir:
        objs, cmds = [], []
        bid = f'-DFFST_BUILD_ID="{build_id()}"'
        for s in SOURCES:
            obj = os.path.join(tmpdir, s.replace(".hip", ".o"))
            objs.append(obj)
            cmds.append([HIPCC, *FLAGS, *extra, bid, "-c", os.path.join(CSRC, s), "-o", obj])
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
        tmp = out_lib + ".tmp"
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *(SANITIZE_LINK if sanitize else []), *objs,
                *LIBS, "-o", tmp]
        rc, err = _run(link)
        if rc != 0:
            raise RuntimeError("link failed:\n" + err)
    os.replace(tmp, out_lib)
    return out_lib


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize" in sys.argv[1:]))
