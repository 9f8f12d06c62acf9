#!/usr/bin/env python3
"""Summaries of rocprofv3 output for the checker's kernels.

  python bench_profile.py stats DIR
      Markdown table of the per-kernel statistics (``*_kernel_stats.csv``) that
      ``rocprofv3 --kernel-trace --stats --output-format csv -d DIR`` wrote.

  python bench_profile.py traffic FETCH_DIR WRITE_DIR --workload W
      HBM bytes per launch of every kernel from two counter runs of
      ``bench.py --copy-probe`` (``--pmc FETCH_SIZE`` into FETCH_DIR, ``--pmc WRITE_SIZE``
      into WRITE_DIR).  Each counter is scaled by what it reads for the copy probe (one
      elementwise kernel that reads and writes a known number of bytes).  Writes the
      per-kernel figures into profiles/traffic.json under W, keyed by the kernel labels
      bench.py reports, each with the digest of the sources it was taken on (the headers
      and the files that launch a kernel under that label).
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import re
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.abspath(__file__))
PROBE_BYTES = 4 * (1 << 28)  # bench.copy_probe: 2^28 int32 read and written


def short_name(name: str) -> str:
    """kernel symbol without namespaces, return type and parameter list"""
    n = name.replace("(anonymous namespace)::", "").replace("vc::", "")
    n = n.split("(")[0]
    return n[5:] if n.startswith("void ") else n


def label_of(name: str) -> str:
    """bench.py's label for a kernel symbol: the function name without the k_ prefix
    (segscan with the pre-status output is segscan_pre); other kernels keep a short name."""
    head = short_name(name)
    m = re.search(r"k_([A-Za-z0-9_]+)(<([^>]*)>)?", head)
    if not m:
        return head[:80]
    base, targs = m.group(1), m.group(3) or ""
    if base == "segscan" and targs.strip().startswith("1"):
        return "segscan_pre"
    return base


def read_csvs(d: str, pattern: str):
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True)):
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    if not rows:
        sys.exit(f"no {pattern} under {d}")
    return rows


def cmd_stats(a):
    rows = read_csvs(a.dir, "*kernel_stats.csv")
    print("| kernel | label | calls | total µs | average µs | % |")
    print("|---|---|---|---|---|---|")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        print(f"| {short_name(r['Name'])[:90]} | {label_of(r['Name'])} | {r['Calls']} | "
              f"{float(r['TotalDurationNs']) / 1e3:.1f} | {float(r['AverageNs']) / 1e3:.1f} | "
              f"{float(r['Percentage']):.1f} |")


def per_dispatch(rows, counter):
    """kernel name -> list of counter values (KiB), one per dispatch"""
    out = defaultdict(list)
    for r in rows:
        if r.get("Counter_Name", "").startswith(counter):
            out[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return out


def cmd_traffic(a):
    sys.path.insert(0, ROOT)
    from bench import source_digest
    fetch = per_dispatch(read_csvs(a.fetch_dir, "*counter_collection.csv"), "FETCH_SIZE")
    write = per_dispatch(read_csvs(a.write_dir, "*counter_collection.csv"), "WRITE_SIZE")
    probe_f = [v for k, vs in fetch.items() if "neg" in k for v in vs]
    probe_w = [v for k, vs in write.items() if "neg" in k for v in vs]
    if not probe_f or not probe_w:
        sys.exit("copy probe kernel not found; non-checker kernels seen: " +
                 ", ".join(sorted({short_name(k)[:60] for k in fetch if 'vc::' not in k})))
    kf = PROBE_BYTES / (probe_f[0] * 1024.0)
    kw = PROBE_BYTES / (probe_w[0] * 1024.0)
    res = {}
    print(f"copy probe: FETCH_SIZE {probe_f[0]:.0f} KiB, WRITE_SIZE {probe_w[0]:.0f} KiB for "
          f"{PROBE_BYTES} bytes each way; scale factors fetch {kf:.4f}, write {kw:.4f}\n")
    print("| kernel | label | dispatches | FETCH KiB/launch | WRITE KiB/launch | HBM bytes/launch (scaled) |")
    print("|---|---|---|---|---|---|")
    agg = defaultdict(lambda: [0.0, 0.0, 0])
    for k in fetch:
        if "vc::" not in k:
            continue
        lab = label_of(k)
        f, w = fetch[k], write.get(k, [])
        n = min(len(f), len(w)) if w else len(f)
        g = agg[lab]
        g[0] += sum(f[:n])
        g[1] += sum(w[:n])
        g[2] += n
    for lab, (f, w, n) in sorted(agg.items(), key=lambda kv: -(kv[1][0] + kv[1][1])):
        fb, wb = f / n, w / n
        bytes_ = fb * 1024 * kf + wb * 1024 * kw
        res[lab] = {"bytes_per_launch": round(bytes_), "fetch_kib": round(fb, 1), "write_kib": round(wb, 1),
                    "dispatches": n, "source_digest": source_digest(lab)}
        print(f"| {lab} | {lab} | {n} | {fb:.1f} | {wb:.1f} | {bytes_:.0f} |")
    p = os.path.join(ROOT, "profiles", "traffic.json")
    t = {}
    if os.path.exists(p):
        with open(p) as fh:
            t = json.load(fh)
    t[a.workload] = {"probe": {"fetch_kib": probe_f[0], "write_kib": probe_w[0], "bytes": PROBE_BYTES,
                               "fetch_scale": kf, "write_scale": kw}, **res}
    with open(p, "w") as fh:
        json.dump(t, fh, indent=1, sort_keys=True)
        fh.write("\n")


def main():
    ap = argparse.ArgumentParser()
    sp = ap.add_subparsers(dest="cmd", required=True)
    s1 = sp.add_parser("stats")
    s1.add_argument("dir")
    s2 = sp.add_parser("traffic")
    s2.add_argument("fetch_dir")
    s2.add_argument("write_dir")
    s2.add_argument("--workload", required=True)
    a = ap.parse_args()
    {"stats": cmd_stats, "traffic": cmd_traffic}[a.cmd](a)


if __name__ == "__main__":
    main()
