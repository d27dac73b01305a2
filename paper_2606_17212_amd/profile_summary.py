"""Summaries of rocprofv3 output, and the measured HBM traffic of a kernel.

    python -m paper_2606_17212_amd.profile_summary trace <results.db> [--top N]
    python -m paper_2606_17212_amd.profile_summary pmc <counter_collection.csv>... [--match NAME]
    python -m paper_2606_17212_amd.profile_summary traffic --fetch <csv> --write <csv>
        --kernel NAME --workload NAME --copy-bytes B --command "..." --out <json>

``traffic`` turns two ``rocprofv3 --pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE``
runs (KiB per dispatch) into bytes per launch of one kernel.  Each counter is
scaled by what it reads for a plain device copy of known size in the same run
(``bench.py --copy-mib``: one ``torch.neg`` over a buffer of that size, which
reads and writes it once; its dispatches summed), so the result is in true
bytes.  The JSON records a hash of the
kernel's sources; ``measured_traffic`` returns the figure only while the
sources are unchanged.
"""

from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re
import sqlite3

HERE = os.path.dirname(os.path.abspath(__file__))
# sources that define the compositing kernels (forward and backward) and the geometry backward
KERNEL_SOURCES = ("csrc/composite.hip", "csrc/geometry.hip", "csrc/common.h", "csrc/kernels.h")
COPY_KERNEL = "neg_kernel"  # the calibration pass of bench.py --copy-mib


def short_name(name: str) -> str:
    """A kernel's name without its parameter list; library (torch) kernels
    shortened to the kernel and the functor or reduction they run."""
    if name.endswith(")"):
        depth = 0
        for i in range(len(name) - 1, -1, -1):
            if name[i] == ")":
                depth += 1
            elif name[i] == "(":
                depth -= 1
                if depth == 0:
                    name = name[:i]
                    break
    if "at::native::" in name:
        base = name.split("<", 1)[0]
        red = re.search(r"ReduceOp<(\w+)", name)
        if red:
            return f"{base}<ReduceOp<{red.group(1)} ...>>"
        fn = re.search(r"(\w*Functor\w*|\w+_kernel_cuda)", name.split("<", 1)[1] if "<" in name else "")
        vec = re.match(r"[^<]*<(\d+),", name)
        parts = ([vec.group(1)] if vec else []) + ([fn.group(1) + " ..."] if fn else [])
        return f"{base}<{', '.join(parts)}>" if parts else base
    return name


def summarize(db: str, top: int = 25) -> str:
    """Per kernel: share of GPU time, dispatches, average / min / max duration."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), avg(end - start), min(end - start), max(end - start), "
                       "sum(end - start) from kernels group by name order by sum(end - start) desc").fetchall()
    total = sum(r[5] for r in rows) or 1
    out = [f"{'share':>7} {'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10}  kernel"]
    for name, n, avg, mn, mx, tot in rows[:top]:
        out.append(f"{100.0 * tot / total:6.2f}% {n:6d} {avg / 1e3:10.2f} {mn / 1e3:10.2f} {mx / 1e3:10.2f}  "
                   f"{short_name(name)}")
    out.append(f"total GPU kernel time {total / 1e6:.3f} ms over {sum(r[1] for r in rows)} dispatches")
    return "\n".join(out)


def _pmc_rows(paths, match=None):
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for p in paths:
        with open(p) as f:
            for row in csv.DictReader(f):
                name = row["Kernel_Name"]
                if match and not any(m in name for m in match):
                    continue
                acc[name][row["Counter_Name"]].append(float(row["Counter_Value"]))
    return acc


def summarize_pmc(csv_paths, match=None) -> str:
    """Per-kernel means of rocprofv3 ``--pmc ... --output-format csv`` files."""
    lines = []
    for name, ctrs in _pmc_rows(csv_paths, match).items():
        lines.append(short_name(name))
        for c, v in sorted(ctrs.items()):
            lines.append(f"    {c:24s} mean {sum(v) / len(v):16.1f}   dispatches {len(v)}")
    return "\n".join(lines)


def kernel_sources_hash(pkg_dir: str = HERE) -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(pkg_dir, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()


def traffic_path(root: str, workload: str, tag: str = "k_composite") -> str:
    return os.path.join(root, "profiles", f"traffic_{tag}_{workload}.json")


def traffic_record(fetch_csv: str, write_csv: str, kernel: str, workload: str, copy_bytes: int,
                   command: str) -> dict:
    """Calibrated HBM bytes per launch of ``kernel`` from FETCH_SIZE and
    WRITE_SIZE counter files of two runs of the same command.  ``kernel`` may
    name several kernels joined by '+' (one call that launches each once):
    their per-dispatch means are added."""
    rec = {"kernel": kernel, "workload": workload, "command": command, "copy_bytes": copy_bytes,
           "sources_sha256": kernel_sources_hash()}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = _pmc_rows([path])
        cp = [v for name, c in rows.items() if COPY_KERNEL in name for v in c.get(counter, [])]
        if not cp:
            raise ValueError(f"{counter}: no dispatches of the copy kernel in {path}")
        copy_kib = sum(cp)  # one call, possibly split over dispatches
        factor = copy_bytes / (copy_kib * 1024.0)
        key = counter.split("_")[0].lower()
        kib, ndisp = 0.0, []
        for part in kernel.split("+"):
            ks = [v for name, c in rows.items() if part in name.replace(" ", "") for v in c.get(counter, [])]
            if not ks:
                raise ValueError(f"{counter}: no dispatches of {part!r} in {path}")
            kib += sum(ks) / len(ks)
            ndisp.append(len(ks))
        rec[f"{key}_kib_per_dispatch"] = kib
        rec[f"{key}_dispatches"] = ndisp[0] if len(ndisp) == 1 else ndisp
        rec[f"{key}_copy_kib"] = copy_kib
        rec[f"{key}_factor"] = factor
        rec[f"{key}_bytes"] = kib * 1024.0 * factor
    rec["traffic_bytes"] = rec["fetch_bytes"] + rec["write_bytes"]
    return rec


def measured_traffic(kernel: str, workload: str, root: str, tag: str = "k_composite"):
    """Calibrated HBM bytes per launch of ``kernel`` on ``workload`` from the
    committed counter record, or None if there is none or the kernel's sources
    changed since it was taken."""
    path = traffic_path(root, workload, tag)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel") != kernel or rec.get("sources_sha256") != kernel_sources_hash():
        return None
    return round(float(rec["traffic_bytes"]))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--top", type=int, default=25)
    p = sub.add_parser("pmc")
    p.add_argument("csv", nargs="+")
    p.add_argument("--match", action="append")
    r = sub.add_parser("traffic")
    r.add_argument("--fetch", required=True)
    r.add_argument("--write", required=True)
    r.add_argument("--kernel", required=True)
    r.add_argument("--workload", required=True)
    r.add_argument("--copy-bytes", type=int, required=True)
    r.add_argument("--command", required=True)
    r.add_argument("--out", required=True)
    r.add_argument("--tag", default="k_composite")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(summarize(a.db, a.top))
    elif a.cmd == "pmc":
        print(summarize_pmc(a.csv, a.match))
    else:
        rec = traffic_record(a.fetch, a.write, a.kernel, a.workload, a.copy_bytes, a.command)
        with open(a.out, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
