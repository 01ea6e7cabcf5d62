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


# the sources that define the persistent projection kernel (the .hip files only instantiate it)
PROJECTION_KERNEL_SOURCES = ("ep_common.hpp", "ep_device.hpp", "ep_expm.hpp", "ep_tangent.hpp", "ep_q2.hpp",
                             "ep_krylov.hpp", "ep_expv.hpp")


# ... and those of the batch kernel (lists of instances or teams per workgroup)
BATCH_KERNEL_SOURCES = PROJECTION_KERNEL_SOURCES + ("ep_batch.hip",)


def sources_sha256(files) -> str:
    import hashlib
    import os
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def projection_kernel_sha256() -> str:
    return sources_sha256(PROJECTION_KERNEL_SOURCES)


def batch_kernel_sha256() -> str:
    return sources_sha256(BATCH_KERNEL_SOURCES)


def _per_dispatch(db: str, counter: str, kernel_like: str):
    con = sqlite3.connect(db)
    return [r[1] for r in con.execute(
        "select dispatch_id, sum(value) from counters_collection where counter_name = ? and kernel_name like ? "
        "group by dispatch_id order by dispatch_id", (counter, kernel_like)).fetchall()]


def traffic(fetch_db: str, write_db: str, kernel: str, last: int, bench_json: str, copy_kib: float = 262144.0):
    """HBM bytes per launch of `kernel` from a FETCH_SIZE run and a WRITE_SIZE run of the same
    command (KiB per dispatch, averaged over its last `last` dispatches), each scaled by what the
    counter reads for the runtime's copy of copy_kib KiB (bench.py --copy-probe)."""
    import json
    f = _per_dispatch(fetch_db, "FETCH_SIZE", kernel)[-last:]
    w = _per_dispatch(write_db, "WRITE_SIZE", kernel)[-last:]
    cf = max(_per_dispatch(fetch_db, "FETCH_SIZE", "%copyBuffer%"))
    cw = max(_per_dispatch(write_db, "WRITE_SIZE", "%copyBuffer%"))
    fetch, write = sum(f) / len(f), sum(w) / len(w)
    fs, ws = copy_kib / cf, copy_kib / cw
    with open(bench_json) as fh:
        b = json.loads(fh.read().strip().splitlines()[-1])
    c = b["config"]
    batch = "k_batch" in kernel
    return {"kernel": kernel, "workload": c["workload"],
            "dispatches": f"the {last} timed launches (last {last} dispatches of the kernel in each run)",
            "fetch_kib_per_launch": fetch, "write_kib_per_launch": write, "copy_probe_kib": copy_kib,
            "copy_fetch_kib": cf, "copy_write_kib": cw, "fetch_scale": fs, "write_scale": ws,
            "traffic_bytes_per_launch": (fs * fetch + ws * write) * 1024.0,
            "kernel_sources_sha256": batch_kernel_sha256() if batch else projection_kernel_sha256(),
            "precision": c["precision"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--top", type=int, default=15)
    ap.add_argument("--counters", action="store_true", help="summarise PMC counters instead of durations")
    ap.add_argument("--traffic", nargs=3, metavar=("WRITE_DB", "KERNEL", "BENCH_JSON"),
                    help="db is the FETCH_SIZE run: print the per-launch traffic record of KERNEL")
    ap.add_argument("--last", type=int, default=3)
    a = ap.parse_args()
    if a.traffic:
        import json
        print(json.dumps(traffic(a.db, a.traffic[0], a.traffic[1], a.last, a.traffic[2]), indent=1))
    else:
        print(counters(a.db, a.top) if a.counters else summarize(a.db, a.top))


if __name__ == "__main__":
    main()
