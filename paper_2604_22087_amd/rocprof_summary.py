"""Summaries of rocprofv3 CSV output (used to write the text summaries kept under profiles/).

  python -m paper_2604_22087_amd.rocprof_summary trace DIR [--min-ns NS] [--top K]
      per-kernel launch count and mean / median duration from *kernel_trace.csv,
      optionally over launches longer than NS only (the CG driver enqueues a few
      launches past convergence that return at once; they are dropped that way)
  python -m paper_2604_22087_amd.rocprof_summary pmc DIR [--kernel SUBSTR]
      per-kernel mean / median / max of each counter from *counter_collection.csv
  python -m paper_2604_22087_amd.rocprof_summary traffic --fetch DIR --write DIR --cal-fetch DIR
      --cal-write DIR --bench-json FILE --kernel SUBSTR --workload TEXT [--roofline KEY.PATH]
      HBM bytes per launch of one kernel from a FETCH_SIZE and a WRITE_SIZE run (KiB per dispatch),
      each scaled by what the same counter reads for a device copy of exactly 1 GiB each way
      (bench.py --copy-calib runs), next to the algorithmic bytes per launch of the benchmark line
      in FILE (its "roofline" object, or the one at the dotted KEY.PATH), with the SHA-256 of the
      kernel sources the counters belong to (JSON)
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


def _mean_counter(root, counter, kernel):
    v = [float(r["Counter_Value"] or 0) for r in _rows(root, "counter_collection.csv")
         if r["Counter_Name"].startswith(counter) and kernel in r["Kernel_Name"]]
    return statistics.fmean(v), len(v)


def traffic(fetch, write, cal_fetch, cal_write, bench_json, kernel, workload, roofline="roofline"):
    import hashlib
    import json
    f_kib, nf = _mean_counter(fetch, "FETCH_SIZE", kernel)
    w_kib, nw = _mean_counter(write, "WRITE_SIZE", kernel)
    cf, _ = _mean_counter(cal_fetch, "FETCH_SIZE", "copyBuffer")
    cw, _ = _mean_counter(cal_write, "WRITE_SIZE", "copyBuffer")
    gib_kib = float(1 << 20)
    fs, ws = gib_kib / cf, gib_kib / cw
    line = [ln for ln in open(bench_json).read().splitlines() if ln.startswith("{")][-1]
    node = json.loads(line)
    for key in roofline.split("."):
        node = node[key]
    algo = node["bytes_per_launch"]
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for f in ("fe_kernels.hip", "fe_internal.hpp", "fe_device.hpp"):
        h.update(open(os.path.join(src, f), "rb").read())
    return json.dumps({"kernel": kernel, "workload": workload, "dispatches": [nf, nw], "fetch_kib_mean": f_kib,
                       "write_kib_mean": w_kib, "fetch_scale": fs, "write_scale": ws,
                       "traffic_bytes_per_launch": 1024.0 * (f_kib * fs + w_kib * ws),
                       "algorithmic_bytes_per_launch": algo, "source_sha256": h.hexdigest()}, indent=1)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("mode", choices=["trace", "pmc", "traffic"])
    ap.add_argument("dir", nargs="?")
    ap.add_argument("--min-ns", type=float, default=0.0)
    ap.add_argument("--top", type=int, default=12)
    ap.add_argument("--kernel", default="")
    for opt in ("--fetch", "--write", "--cal-fetch", "--cal-write", "--bench-json", "--workload"):
        ap.add_argument(opt)
    ap.add_argument("--roofline", default="roofline")
    a = ap.parse_args(argv)
    if a.mode == "traffic":
        print(traffic(a.fetch, a.write, a.cal_fetch, a.cal_write, a.bench_json, a.kernel, a.workload, a.roofline))
    else:
        print(trace(a.dir, a.min_ns, a.top) if a.mode == "trace" else pmc(a.dir, a.kernel))


if __name__ == "__main__":
    main()
