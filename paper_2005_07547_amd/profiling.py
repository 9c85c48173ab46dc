"""Summaries of rocprofv3 output for the hash-path kernels.

* ``stats``: turn a ``--kernel-trace --stats`` kernel_stats.csv into a short
  Markdown table (with the command that produced it);
* ``counters-md``: any other counters (L2 hits, LDS bank conflicts, waves)
  per kernel as a Markdown table;
* ``traffic-md``: the same record as a Markdown table beside the kernels'
  algorithmic bytes;
* ``traffic``: combine two ``--pmc`` runs (FETCH_SIZE, then WRITE_SIZE, KiB
  per dispatch) with the same counters taken on a plain 1 GiB device copy,
  into per-launch HBM bytes of each kernel, scaled so that the copy reads
  and writes exactly its size.  The record carries a digest of the kernel
  sources; a consumer treats it as stale once the sources change.

Usage: python -m paper_2005_07547_amd.profiling stats|traffic ... (see --help).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ("csrc/psf_device.h", "csrc/psf_internal.h", "csrc/psf_kernels.hip",
           "csrc/psf_partition.hip")
COPY_BYTES = 1 << 30


def source_digest() -> str:
    h = hashlib.sha256()
    for rel in SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _find(d, pattern):
    hits = glob.glob(os.path.join(d, "**", pattern), recursive=True)
    if not hits:
        raise FileNotFoundError(f"no {pattern} under {d}")
    return hits[0]


def counter_means(d: str) -> dict:
    """{kernel: {counter: mean per dispatch}} from a --pmc output directory."""
    rows = list(csv.DictReader(open(_find(d, "*counter_collection.csv"))))
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in rows:
        acc[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in acc.items()}


def traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir) -> dict:
    f, w = counter_means(fetch_dir), counter_means(write_dir)
    cf_raw, cw_raw = counter_means(copy_fetch_dir), counter_means(copy_write_dir)
    copy_k = max(cf_raw, key=lambda k: cf_raw[k].get("FETCH_SIZE", 0))
    cf = COPY_BYTES / (cf_raw[copy_k]["FETCH_SIZE"] * 1024)
    cw = COPY_BYTES / (cw_raw[copy_k]["WRITE_SIZE"] * 1024)
    kernels = {}
    for k in f:
        if k in w and "FETCH_SIZE" in f[k] and "WRITE_SIZE" in w[k]:
            kernels[k] = {"fetch_kib": f[k]["FETCH_SIZE"], "write_kib": w[k]["WRITE_SIZE"],
                          "bytes": (f[k]["FETCH_SIZE"] * cf + w[k]["WRITE_SIZE"] * cw) * 1024}
    return {"digest": source_digest(), "fetch_scale": cf, "write_scale": cw,
            "copy_kernel": copy_k, "kernels": kernels}


def stats_markdown(stats_csv: str, title: str, command: str, note: str = "") -> str:
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# {title}", "", "Command (from the repository root on one MI355X):", "",
             f"    {command}", ""]
    if note:
        lines += [note, ""]
    lines += ["| Kernel | Calls | Average (us) | Min (us) | Max (us) | Share |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| {r['Name']} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.1f}% |")
    return "\n".join(lines) + "\n"


def counters_markdown(dirs: list, title: str, commands: list, kernels: list) -> str:
    """Mean per dispatch of every counter found in the given --pmc output
    directories, one row per kernel whose name contains one of `kernels`."""
    merged = collections.defaultdict(dict)
    for d in dirs:
        for k, cs in counter_means(d).items():
            merged[k].update(cs)
    names = sorted({c for cs in merged.values() for c in cs})
    lines = [f"# {title}", "", "Counters (mean per dispatch), one rocprofv3 run per group:", ""]
    lines += [f"    {c}" for c in commands]
    lines += ["", "| Kernel | " + " | ".join(names) + " |", "|---" * (len(names) + 1) + "|"]
    for k in sorted(merged):
        short = k.split("(")[0].split("::")[-1]
        if kernels and not any(x in short for x in kernels):
            continue
        lines.append(f"| {short} | " + " | ".join(
            f"{merged[k][c]:.4g}" if c in merged[k] else "-" for c in names) + " |")
    return "\n".join(lines) + "\n"


def traffic_markdown(rec: dict, title: str, commands: list, algorithmic: dict) -> str:
    """Markdown table of a traffic record: counter KiB, scaled HBM bytes and,
    where given, the kernel's algorithmic bytes per launch (by short name)."""
    lines = [f"# {title}", "", "Counters (KiB per dispatch), each in a rocprofv3 run of its own:", ""]
    lines += [f"    {c}" for c in commands]
    lines += ["", f"Calibration on a 1 GiB device copy: FETCH_SIZE x {rec['fetch_scale']:.4f}, "
              f"WRITE_SIZE x {rec['write_scale']:.4f} give the bytes the copy moves.", "",
              "| Kernel | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | HBM bytes (scaled) | Algorithmic bytes | Ratio |",
              "|---|---|---|---|---|---|"]
    for name, v in sorted(rec["kernels"].items(), key=lambda kv: -kv[1]["bytes"]):
        short = name.split("(")[0].split("::")[-1]
        base = short.split("<")[0]
        a = algorithmic.get(base)
        lines.append(f"| {short} | {v['fetch_kib']:.0f} | {v['write_kib']:.0f} | {v['bytes'] / 1e6:.1f} MB | "
                     + (f"{a / 1e6:.1f} MB | {v['bytes'] / a:.2f} |" if a else "- | - |"))
    lines += ["", f"Kernel source digest: `{rec['digest']}` (bench.py reports `traffic` only while the "
              "kernel sources still have this digest)."]
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("--dir", required=True)
    a.add_argument("--title", required=True)
    a.add_argument("--command", required=True)
    a.add_argument("--note", default="")
    a.add_argument("--out", required=True)
    b = sub.add_parser("traffic")
    for name in ("fetch", "write", "copy-fetch", "copy-write"):
        b.add_argument(f"--{name}", required=True)
    b.add_argument("--command", default="")
    b.add_argument("--out", required=True)
    m = sub.add_parser("counters-md")
    m.add_argument("--dir", action="append", required=True)
    m.add_argument("--title", required=True)
    m.add_argument("--command", action="append", default=[])
    m.add_argument("--kernels", default="k_bin,k_merge,k_unstage,k_transpose")
    m.add_argument("--out", required=True)
    c = sub.add_parser("traffic-md")
    c.add_argument("--json", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--command", action="append", default=[])
    c.add_argument("--algorithmic", default="{}", help="JSON {kernel: bytes per launch}")
    c.add_argument("--out", required=True)
    args = ap.parse_args()
    if args.cmd == "stats":
        md = stats_markdown(_find(args.dir, "*kernel_stats.csv"), args.title, args.command, args.note)
        with open(args.out, "w") as f:
            f.write(md)
    elif args.cmd == "counters-md":
        md = counters_markdown(args.dir, args.title, args.command, [k for k in args.kernels.split(",") if k])
        with open(args.out, "w") as f:
            f.write(md)
    elif args.cmd == "traffic-md":
        with open(args.json) as f:
            rec = json.load(f)
        md = traffic_markdown(rec, args.title, args.command, json.loads(args.algorithmic))
        with open(args.out, "w") as f:
            f.write(md)
    else:
        rec = traffic(args.fetch, args.write, args.copy_fetch, args.copy_write)
        rec["command"] = args.command
        with open(args.out, "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
