"""Summaries of rocprofv3 output, as kept under profiles/.

Kernel trace (rocpd SQLite database), per kernel and launch shape:

    python -m paper_1202_1773_amd.profile_summary <run_results.db>

Vector-ALU instructions from a counter run with SQ_INSTS_VALU (CSV output),
per labelled kernel shape, with the time they take at full issue rate (a
wave64 FP32 instruction occupies a 16-lane SIMD for 4 cycles; 4 SIMDs per
compute unit, 256 compute units at 2.4 GHz; packed FP32 is not used):

    python -m paper_1202_1773_amd.profile_summary --valu <dir> --label ...

HBM traffic from two counter-collection runs (one with FETCH_SIZE, one with
WRITE_SIZE; CSV output). Both counters are scaled by what they read for the
largest plain device copy in the same runs (the benchmark's calibration copy
of a known size), then averaged per launch of each labelled kernel shape:

    python -m paper_1202_1773_amd.profile_summary --pmc <fetch_dir> <write_dir> \\
        --copy-mib 256 --workload 512 512 3 16 \\
        --label "k_r2c_rows(planes)=k_r2c_rows<256, false>@2048" ...

Each label maps a kernel name of the library's timing table to a compiled
kernel and a grid size in workgroups; one "TRAFFIC {json}" line is printed
per label, tied to the kernel sources by their hash.

Host-side roctx ranges of the library (one per C ABI call and one per kernel
launch, named as in its timing table) from a run with --marker-trace and CSV
output, by median duration:

    python -m paper_1202_1773_amd.profile_summary --markers <dir>
"""

import argparse
import collections
import csv
import glob
import json
import os
import re
import sqlite3


def short_name(name):
    m = re.search(r"(k_[a-z0-9_]+(<[^>]*>)?)", name)
    return m.group(1) if m else name[:48]


def summarize(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, grid_x, grid_y, workgroup_x, duration, lds_size, scratch_size "
                       "from kernels").fetchall()
    agg = collections.defaultdict(list)
    for name, gx, gy, wx, dur, lds, scr in rows:
        agg[(short_name(name), gx // max(wx, 1), gy, wx, lds, scr)].append(dur)
    total = sum(sum(v) for k, v in agg.items() if k[0].startswith("k_"))
    out = ["| kernel | blocks | wg | LDS B | scratch | launches | avg us | share |",
           "|---|---|---|---|---|---|---|---|"]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        if not k[0].startswith("k_"):
            continue
        out.append(f"| {k[0]} | {k[1]}x{k[2]} | {k[3]} | {k[4]} | {k[5]} | {len(v)} | "
                   f"{sum(v) / len(v) / 1000:.2f} | {100 * sum(v) / total:.1f}% |")
    return "\n".join(out)


def read_counters(run_dir, counter):
    """(kernel name, blocks) -> list of counter values (KiB per dispatch)."""
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {run_dir}")
    out = collections.defaultdict(list)
    for f in files:
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            wg = max(int(float(r.get("Workgroup_Size", 1) or 1)), 1)
            blocks = int(float(r.get("Grid_Size", 0) or 0)) // wg
            out[(r["Kernel_Name"], blocks)].append(float(r["Counter_Value"]))
    return out


def calibration(fetch, write, copy_mib):
    """Scale factors from the plain copy: the non-library dispatch that
    fetched the most, whose bytes read and written are both copy_mib MiB."""
    cands = [(max(v), k) for k, v in fetch.items() if not short_name(k[0]).startswith("k_")]
    if not cands:
        raise RuntimeError("no copy dispatch in the fetch run")
    kib = max(cands)[0]
    key = max(cands)[1]
    wkib = max(write.get(key, [0.0]))
    if wkib <= 0:
        raise RuntimeError("copy dispatch missing from the write run")
    want = copy_mib * 1024.0
    return want / kib, want / wkib, key[0]


def traffic(fetch_dir, write_dir, copy_mib, workload, labels, sha):
    fetch = read_counters(fetch_dir, "FETCH_SIZE")
    write = read_counters(write_dir, "WRITE_SIZE")
    ff, wf, copy_name = calibration(fetch, write, copy_mib)
    lines = [f"Calibration: copy of {copy_mib} MiB (`{short_name(copy_name)}`): FETCH_SIZE x{ff:.3f}, "
             f"WRITE_SIZE x{wf:.3f}", "",
             "| kernel | compiled kernel | blocks | launches | FETCH KiB | WRITE KiB | HBM bytes / launch |",
             "|---|---|---|---|---|---|---|"]
    recs = []
    for label in labels:
        api, rest = label.split("=", 1)
        kname, blocks = rest.rsplit("@", 1)
        blocks = int(blocks)
        fv = [v for (n, b), vals in fetch.items() if short_name(n) == kname and b == blocks for v in vals]
        wv = [v for (n, b), vals in write.items() if short_name(n) == kname and b == blocks for v in vals]
        if not fv or not wv:
            raise RuntimeError(f"no dispatch of {kname} with {blocks} blocks")
        f_kib = sum(fv) / len(fv)
        w_kib = sum(wv) / len(wv)
        nbytes = int(round((f_kib * ff + w_kib * wf) * 1024))
        lines.append(f"| {api} | {kname} | {blocks} | {len(fv)} | {f_kib:.0f} | {w_kib:.0f} | {nbytes} |")
        recs.append({"kernel": api, "compiled": kname, "blocks": blocks, "source_sha": sha,
                     "workload": workload, "bytes_per_launch": nbytes,
                     "fetch_bytes": int(round(f_kib * ff * 1024)), "write_bytes": int(round(w_kib * wf * 1024))})
    lines.append("")
    lines += ["TRAFFIC " + json.dumps(r) for r in recs]
    return "\n".join(lines)


VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4   # wave64 VALU instructions per second, whole device


def valu(run_dir, labels):
    counts = read_counters(run_dir, "SQ_INSTS_VALU")
    lines = ["| kernel | compiled kernel | blocks | launches | SQ_INSTS_VALU / launch | VALU issue us / launch |",
             "|---|---|---|---|---|---|"]
    for label in labels:
        api, rest = label.split("=", 1)
        kname, blocks = rest.rsplit("@", 1)
        vals = [v for (n, b), vv in counts.items() if short_name(n) == kname and b == int(blocks) for v in vv]
        if not vals:
            raise RuntimeError(f"no dispatch of {kname} with {blocks} blocks")
        avg = sum(vals) / len(vals)
        lines.append(f"| {api} | {kname} | {blocks} | {len(vals)} | {avg:.4g} | {avg / VALU_ISSUE_PER_S * 1e6:.1f} |")
    return "\n".join(lines)


def markers(run_dir):
    paths = glob.glob(os.path.join(run_dir, "**", "*marker_api_trace.csv"), recursive=True)
    if not paths:
        raise RuntimeError(f"no marker trace under {run_dir}")
    durs = collections.defaultdict(list)
    for path in paths:
        with open(path, newline="") as fh:
            for row in csv.DictReader(fh):
                name = row.get("Function") or row.get("Name") or ""
                start, end = row.get("Start_Timestamp"), row.get("End_Timestamp")
                if name and start and end:
                    durs[name].append((int(end) - int(start)) / 1e3)
    lines = ["| range | calls | median us | min us | max us |", "|---|---|---|---|---|"]
    for name, v in sorted(durs.items(), key=lambda kv: -sorted(kv[1])[len(kv[1]) // 2]):
        v = sorted(v)
        lines.append(f"| {name} | {len(v)} | {v[len(v) // 2]:.1f} | {v[0]:.1f} | {v[-1]:.1f} |")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db", nargs="?")
    ap.add_argument("--pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--valu", metavar="DIR")
    ap.add_argument("--markers", metavar="DIR")
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--workload", type=int, nargs=4, metavar=("M", "N", "J", "B"))
    ap.add_argument("--label", action="append", default=[])
    args = ap.parse_args()
    if args.markers:
        print(markers(args.markers))
    elif args.valu:
        print(valu(args.valu, args.label))
    elif args.pmc:
        from .build import source_sha
        print(traffic(args.pmc[0], args.pmc[1], args.copy_mib, args.workload, args.label, source_sha()))
    else:
        print(summarize(args.db))


if __name__ == "__main__":
    main()
