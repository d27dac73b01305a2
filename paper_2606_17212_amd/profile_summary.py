"""Summarise a rocprofv3 kernel-trace database (``*_results.db``) per kernel:
share of GPU time, dispatch count, average / min / max duration.

    python -m paper_2606_17212_amd.profile_summary <results.db> [--top N]
"""

import argparse
import sqlite3


def summarize(db: str, top: int = 25) -> str:
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), avg(end - start), min(end - start), max(end - start), "
                       "sum(end - start) from kernels group by name order by sum(end - start) desc").fetchall()
    total = sum(r[5] for r in rows) or 1
    out = [f"{'share':>7} {'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10}  kernel"]
    for name, n, avg, mn, mx, tot in rows[:top]:
        out.append(f"{100.0 * tot / total:6.2f}% {n:6d} {avg / 1e3:10.2f} {mn / 1e3:10.2f} {mx / 1e3:10.2f}  {name}")
    out.append(f"total GPU kernel time {total / 1e6:.3f} ms over {sum(r[1] for r in rows)} dispatches")
    return "\n".join(out)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--top", type=int, default=25)
    a = ap.parse_args()
    print(summarize(a.db, a.top))


def summarize_pmc(csv_paths, match=None) -> str:
    """Per-kernel averages of rocprofv3 ``--pmc ... --output-format csv``
    counter files (``*_counter_collection.csv``)."""
    import collections
    import csv
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for p in csv_paths:
        for row in csv.DictReader(open(p)):
            name = row["Kernel_Name"]
            if match and not any(m in name for m in match):
                continue
            acc[name][row["Counter_Name"]].append(float(row["Counter_Value"]))
    lines = []
    for name, ctrs in acc.items():
        lines.append(name)
        for c, v in sorted(ctrs.items()):
            lines.append(f"    {c:24s} mean {sum(v) / len(v):16.1f}   dispatches {len(v)}")
    return "\n".join(lines)
