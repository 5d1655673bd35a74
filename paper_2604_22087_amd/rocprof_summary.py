"""Summaries of rocprofv3 CSV output (used to write the text summaries kept under profiles/).

  python -m paper_2604_22087_amd.rocprof_summary trace DIR [--min-ns NS] [--top K]
      per-kernel launch count and mean / median duration from *kernel_trace.csv,
      optionally over launches longer than NS only (the CG driver enqueues a few
      launches past convergence that return at once; they are dropped that way)
  python -m paper_2604_22087_amd.rocprof_summary pmc DIR [--kernel SUBSTR]
      per-kernel mean / median / max of each counter from *counter_collection.csv
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import os
import statistics


def _rows(root, suffix):
    for f in sorted(glob.glob(os.path.join(root, "**", "*" + suffix), recursive=True)):
        with open(f, newline="") as fh:
            yield from csv.DictReader(fh)


def trace(root, min_ns=0.0, top=12):
    dur = collections.defaultdict(list)
    for r in _rows(root, "kernel_trace.csv"):
        d = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
        dur[r["Kernel_Name"]].append(d)
    total = sum(sum(v) for v in dur.values())
    lines = ["| kernel | launches | kept (> %g ns) | mean us (kept) | median us (kept) | share of GPU time |" % min_ns,
             "|---|---|---|---|---|---|"]
    for name, v in sorted(dur.items(), key=lambda kv: -sum(kv[1]))[:top]:
        kept = [x for x in v if x > min_ns] or v
        lines.append(f"| `{name[:110]}` | {len(v)} | {len(kept)} | {statistics.fmean(kept) / 1e3:.2f} | "
                     f"{statistics.median(kept) / 1e3:.2f} | {100 * sum(v) / total:.1f}% |")
    return "\n".join(lines)


def pmc(root, kernel=""):
    vals = collections.defaultdict(list)
    for r in _rows(root, "counter_collection.csv"):
        if kernel in r["Kernel_Name"]:
            vals[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"] or 0))
    lines = ["| kernel | counter | dispatches | mean | median | max |", "|---|---|---|---|---|---|"]
    for (name, c), v in sorted(vals.items()):
        lines.append(f"| `{name[:110]}` | {c} | {len(v)} | {statistics.fmean(v):.1f} | {statistics.median(v):.1f} | "
                     f"{max(v):.1f} |")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("mode", choices=["trace", "pmc"])
    ap.add_argument("dir")
    ap.add_argument("--min-ns", type=float, default=0.0)
    ap.add_argument("--top", type=int, default=12)
    ap.add_argument("--kernel", default="")
    a = ap.parse_args(argv)
    print(trace(a.dir, a.min_ns, a.top) if a.mode == "trace" else pmc(a.dir, a.kernel))


if __name__ == "__main__":
    main()
