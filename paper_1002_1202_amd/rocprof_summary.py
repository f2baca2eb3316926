"""Short text summaries of rocprofv3 output for the kernels this library runs.

Two summaries, both Markdown with the command that produced the data:

``stats``    the ``--kernel-trace --stats`` CSV as a table (calls, total,
             average, min and max duration per kernel).
``counters`` per-dispatch means of the counters of several ``--pmc`` runs for
             the kernels matching a pattern, one row per kernel.
``traffic``  HBM bytes per dispatch of one kernel from two ``--pmc`` runs
             (FETCH_SIZE, then WRITE_SIZE, in KiB per dispatch), each scaled
             by what the same counter reads for a plain copy-like kernel of
             known size run in the same process (``torch.neg`` of a 1 GiB
             tensor: 1 GiB read, 1 GiB written).  The summary records a digest
             of the kernel's source files, so a reader can tell whether the
             counters still describe the current kernel.

    python -m paper_1002_1202_amd.rocprof_summary stats STATS_CSV --title T --cmd C
    python -m paper_1002_1202_amd.rocprof_summary counters DIR [DIR ...] --kernel REGEX --title T --cmd C
    python -m paper_1002_1202_amd.rocprof_summary traffic FETCH_DIR WRITE_DIR \
        --kernel REGEX --name NAME --probe-bytes B --cmd-fetch C1 --cmd-write C2
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
# sources whose change invalidates a traffic summary of a product kernel
KERNEL_SOURCES = {
    "cheb_step": ["csrc/spmm.hip", "csrc/kernels.h"],
    "cheb_mx": ["csrc/spmm.hip", "csrc/kernels.h"],
    "shift_update": ["csrc/solver.hip", "csrc/kernels.h"],
}


def source_digest(name: str) -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[name]:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(rel.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
    return re.sub(r"\(.*", "", name).replace("void ", "").strip()


def stats_md(path: str, title: str, cmd: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = [f"# {title}", "", "Command (MI355X, from the repository root):", "", "```", cmd, "```", "",
           "| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| `{_short(r['Name'])}` | {int(r['Calls'])} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def _counter_rows(d: str):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    for f in files:
        yield from csv.DictReader(open(f))


def _per_dispatch(d: str, counter: str, pattern: str):
    """Mean counter value (KiB) per dispatch of kernels matching pattern."""
    rx = re.compile(pattern)
    vals = {}
    for r in _counter_rows(d):
        if r["Counter_Name"] != counter or not rx.search(r["Kernel_Name"]):
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id") or str(len(vals))
        vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    if not vals:
        raise SystemExit(f"{counter}: no dispatch of /{pattern}/ under {d}")
    return sum(vals.values()) / len(vals), len(vals)


def traffic_md(fetch_dir, write_dir, kernel, name, probe_bytes, cmd_fetch, cmd_write, probe="neg"):
    f_k, n_f = _per_dispatch(fetch_dir, "FETCH_SIZE", kernel)
    w_k, n_w = _per_dispatch(write_dir, "WRITE_SIZE", kernel)
    f_p, _ = _per_dispatch(fetch_dir, "FETCH_SIZE", probe)
    w_p, _ = _per_dispatch(write_dir, "WRITE_SIZE", probe)
    cf = probe_bytes / (f_p * 1024.0)
    cw = probe_bytes / (w_p * 1024.0)
    traffic = (f_k * cf + w_k * cw) * 1024.0
    out = [f"# HBM traffic per dispatch — `{name}` (kernels /{kernel}/)", "",
           "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two rocprofv3 --pmc runs, each scaled by",
           f"the same counter's reading for a copy-like probe kernel (/{probe}/, {probe_bytes} bytes read",
           "and written) in the same process.", "",
           "Commands (MI355X, from the repository root):", "", "```", cmd_fetch, cmd_write, "```", "",
           "| quantity | value |", "|---|---|",
           f"| dispatches (fetch run / write run) | {n_f} / {n_w} |",
           f"| FETCH_SIZE KiB per dispatch | {f_k:.1f} |",
           f"| WRITE_SIZE KiB per dispatch | {w_k:.1f} |",
           f"| probe FETCH_SIZE KiB | {f_p:.1f} (scale {cf:.4f}) |",
           f"| probe WRITE_SIZE KiB | {w_p:.1f} (scale {cw:.4f}) |",
           f"| fetched bytes per dispatch | {f_k * cf * 1024:.4e} |",
           f"| written bytes per dispatch | {w_k * cw * 1024:.4e} |", "",
           f"- kernel: {name}",
           f"- traffic_bytes_per_dispatch: {traffic:.6e}",
           f"- source_digest: {source_digest(name)}"]
    return "\n".join(out)


def counters_md(dirs, kernel, title, cmds):
    """Mean value per dispatch of every counter found under the run
    directories, for each kernel (short name) matching the pattern."""
    rx = re.compile(kernel)
    acc = {}
    for d in dirs:
        per = {}
        for r in _counter_rows(d):
            if not rx.search(r["Kernel_Name"]):
                continue
            key = (_short(r["Kernel_Name"]), r["Counter_Name"], r.get("Dispatch_Id") or r.get("Correlation_Id"))
            per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
        for (k, c, _), v in per.items():
            acc.setdefault(k, {}).setdefault(c, []).append(v)
    names = sorted({c for d in acc.values() for c in d})
    out = [f"# {title}", "", "Commands (MI355X, from the repository root; one --pmc run per line):", "", "```",
           *cmds, "```", "", "Mean per dispatch.", "",
           "| kernel | dispatches | " + " | ".join(names) + " |", "|---|---|" + "---|" * len(names)]
    for k in sorted(acc):
        n = max(len(v) for v in acc[k].values())
        cells = [f"{sum(acc[k][c]) / len(acc[k][c]):.4g}" if c in acc[k] else "" for c in names]
        out.append(f"| `{k}` | {n} | " + " | ".join(cells) + " |")
    return "\n".join(out)


def read_traffic(path: str, name: str):
    """traffic_bytes_per_dispatch recorded in a traffic summary, or None when
    the file is missing, names another kernel or its source digest no longer
    matches the sources (the kernel changed since the counters were taken)."""
    try:
        text = open(path).read()
    except OSError:
        return None
    kv = dict(re.findall(r"^- (\w+): (\S+)$", text, flags=re.M))
    if kv.get("kernel") != name or kv.get("source_digest") != source_digest(name):
        return None
    return float(kv["traffic_bytes_per_dispatch"])


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--title", required=True)
    s.add_argument("--cmd", required=True)
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--kernel", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--cmd", action="append", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("--kernel", required=True)
    t.add_argument("--name", required=True, choices=sorted(KERNEL_SOURCES))
    t.add_argument("--probe-bytes", type=float, default=float(1 << 30))
    t.add_argument("--probe", default="neg")
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    a = ap.parse_args(argv)
    if a.mode == "stats":
        print(stats_md(a.csv, a.title, a.cmd))
    elif a.mode == "counters":
        print(counters_md(a.dirs, a.kernel, a.title, a.cmd))
    else:
        print(traffic_md(a.fetch_dir, a.write_dir, a.kernel, a.name, a.probe_bytes, a.cmd_fetch, a.cmd_write,
                         a.probe))


if __name__ == "__main__":
    sys.exit(main())
