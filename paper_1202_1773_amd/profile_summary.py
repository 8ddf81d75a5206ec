"""Summarise a rocprofv3 kernel trace (rocpd SQLite database) per kernel and
launch shape: launches, average and total duration. Used to produce the
text summaries kept under profiles/.

    python -m paper_1202_1773_amd.profile_summary <run_results.db>
"""

import collections
import re
import sqlite3
import sys


def summarize(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, grid_x, grid_y, workgroup_x, duration, lds_size, scratch_size "
                       "from kernels").fetchall()
    agg = collections.defaultdict(list)
    for name, gx, gy, wx, dur, lds, scr in rows:
        m = re.search(r"(k_[a-z0-9_]+(<[^>]*>)?)", name)
        short = m.group(1) if m else name[:48]
        agg[(short, gx // max(wx, 1), gy, wx, lds, scr)].append(dur)
    total = sum(sum(v) for k, v in agg.items() if k[0].startswith("k_"))
    out = ["| kernel | blocks | wg | LDS B | scratch | launches | avg us | share |",
           "|---|---|---|---|---|---|---|---|"]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        if not k[0].startswith("k_"):
            continue
        out.append(f"| {k[0]} | {k[1]}x{k[2]} | {k[3]} | {k[4]} | {k[5]} | {len(v)} | "
                   f"{sum(v) / len(v) / 1000:.2f} | {100 * sum(v) / total:.1f}% |")
    return "\n".join(out)


if __name__ == "__main__":
    print(summarize(sys.argv[1]))
