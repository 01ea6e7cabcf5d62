"""Per-kernel summary of a rocprofv3 kernel-trace database (rocpd SQLite output).

rocprofv3 --stats writes its summary when the profiled process exits; with cooperative
launches the profiler itself can crash at that point after the trace database is
complete.  This reads the database directly and prints the same figures (calls, total,
average, min, max duration per kernel) plus the dispatch shape of each kernel.

Usage: python -m paper_2405_05213_amd.profsum <results.db> [--top N]
"""
from __future__ import annotations

import argparse
import sqlite3


def summarize(db: str, top: int = 15):
    con = sqlite3.connect(db)
    rows = con.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration), "
        "max(grid_x), max(workgroup_x), max(lds_size), max(vgpr_count), max(scratch_size) "
        "from kernels group by name order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows) or 1.0
    out = []
    out.append(f"{'kernel':<70} {'calls':>6} {'total_ms':>10} {'avg_us':>10} {'min_us':>10} {'max_us':>10} "
               f"{'%':>6} {'grid':>8} {'wg':>5} {'lds':>7} {'vgpr':>5} {'scratch':>7}")
    for r in rows[:top]:
        name = r[0] if len(r[0]) <= 70 else r[0][:67] + "..."
        out.append(f"{name:<70} {r[1]:>6d} {r[2] / 1e6:>10.3f} {r[3] / 1e3:>10.2f} {r[4] / 1e3:>10.2f} "
                   f"{r[5] / 1e3:>10.2f} {100.0 * r[2] / total:>6.2f} {r[6]:>8} {r[7]:>5} {r[8]:>7} {r[9]:>5} "
                   f"{r[10]:>7}")
    return "\n".join(out)


def counters(db: str, top: int = 15):
    """Value per dispatch of every collected counter, per kernel (rocprofv3 --pmc): the
    counter's rows of one dispatch (one per shader engine / instance for the basic SQ
    counters) are summed, then averaged over the dispatches."""
    con = sqlite3.connect(db)
    rows = con.execute(
        "select kernel_name, counter_name, count(*), avg(v), min(v), max(v) from "
        "(select kernel_name, counter_name, dispatch_id, sum(value) as v from counters_collection "
        " group by kernel_name, counter_name, dispatch_id) "
        "group by kernel_name, counter_name order by avg(v) desc").fetchall()
    out = [f"{'kernel':<70} {'counter':<28} {'dispatches':>10} {'avg':>16} {'min':>16} {'max':>16}"]
    for r in rows[: top * 4]:
        name = r[0] if len(r[0]) <= 70 else r[0][:67] + "..."
        out.append(f"{name:<70} {r[1]:<28} {r[2]:>10d} {r[3]:>16.1f} {r[4]:>16.1f} {r[5]:>16.1f}")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--top", type=int, default=15)
    ap.add_argument("--counters", action="store_true", help="summarise PMC counters instead of durations")
    a = ap.parse_args()
    print(counters(a.db, a.top) if a.counters else summarize(a.db, a.top))


if __name__ == "__main__":
    main()
