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
  and writes exactly its size; with FETCH_SIZE taken on random row gathers
  of known size as well, also scaled as random line fills need (the copy's
  scale counts a streamed 128-byte request at half its size, a random line
  fill at its size).  The record carries a digest of the kernel sources; a
  consumer treats it as stale once the sources change.

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


GATHER_ROWS = 1 << 24       # rows per gather launch of bench.py --gather-calib
GATHER_ROW_BYTES = (32, 64, 128)


def gather_fetch_scale(gather_fetch_dir: str, copy_fetch_scale: float) -> dict:
    """FETCH_SIZE scale for random line fills, from bench.py --gather-calib:
    the 128-byte-row gather reads exactly 2^24 random 128-byte lines (no
    partial-line ambiguity) plus its 8-byte indices as a stream (counted at
    the copy's scale).  Also the bytes counted per row for every width."""
    rows = list(csv.DictReader(open(_find(gather_fetch_dir, "*counter_collection.csv"))))
    g = sorted((int(r["Dispatch_Id"]), float(r["Counter_Value"])) for r in rows
               if "gather" in r["Kernel_Name"] and r["Counter_Name"] == "FETCH_SIZE")
    if len(g) != len(GATHER_ROW_BYTES):
        raise ValueError(f"expected {len(GATHER_ROW_BYTES)} gather dispatches, found {len(g)}")
    index_kib = GATHER_ROWS * 8 / 1024 / copy_fetch_scale
    per_row = {w: (kib - index_kib) * 1024 / GATHER_ROWS for w, (_, kib) in zip(GATHER_ROW_BYTES, g)}
    scale = GATHER_ROW_BYTES[-1] / per_row[GATHER_ROW_BYTES[-1]]
    return {"random_fetch_scale": scale, "fetch_bytes_counted_per_random_row": per_row}


def traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, gather_fetch_dir=None) -> dict:
    """HBM bytes per launch of every kernel.  `bytes` scales FETCH_SIZE as the
    streaming copy needs (right for streamed reads); with a gather
    calibration, `bytes_random` scales it as random line fills need (right
    for scattered reads); a kernel's real traffic lies between the two."""
    f, w = counter_means(fetch_dir), counter_means(write_dir)
    cf_raw, cw_raw = counter_means(copy_fetch_dir), counter_means(copy_write_dir)
    copy_k = max(cf_raw, key=lambda k: cf_raw[k].get("FETCH_SIZE", 0))
    cf = COPY_BYTES / (cf_raw[copy_k]["FETCH_SIZE"] * 1024)
    cw = COPY_BYTES / (cw_raw[copy_k]["WRITE_SIZE"] * 1024)
    gcal = gather_fetch_scale(gather_fetch_dir, cf) if gather_fetch_dir else None
    kernels = {}
    for k in f:
        if k in w and "FETCH_SIZE" in f[k] and "WRITE_SIZE" in w[k]:
            rec = {"fetch_kib": f[k]["FETCH_SIZE"], "write_kib": w[k]["WRITE_SIZE"],
                   "bytes": (f[k]["FETCH_SIZE"] * cf + w[k]["WRITE_SIZE"] * cw) * 1024}
            if gcal:
                rec["bytes_random"] = (f[k]["FETCH_SIZE"] * gcal["random_fetch_scale"] + w[k]["WRITE_SIZE"] * cw) * 1024
            kernels[k] = rec
    out = {"digest": source_digest(), "fetch_scale": cf, "write_scale": cw,
           "copy_kernel": copy_k, "kernels": kernels}
    if gcal:
        out.update(gcal)
    return out


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
              f"WRITE_SIZE x {rec['write_scale']:.4f} give the bytes the copy moves (streamed)."]
    rnd = "random_fetch_scale" in rec
    if rnd:
        per = ", ".join(f"{w} B rows: {b:.0f} B" for w, b in rec["fetch_bytes_counted_per_random_row"].items())
        lines += [f"Calibration on random row gathers (2^24 rows from a 4 GiB table): FETCH_SIZE counts per "
                  f"row {per}; the 128-byte rows (whole lines) give FETCH_SIZE x {rec['random_fetch_scale']:.4f} "
                  "for random line fills.  A kernel's real traffic lies between the random-scaled and the "
                  "copy-scaled bytes, by its share of streamed reads."]
    lines += ["", "| Kernel | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | HBM bytes, copy scale | "
              + ("HBM bytes, random scale | " if rnd else "") + "Algorithmic bytes | Ratio |",
              "|---|---|---|---|" + ("---|" if rnd else "") + "---|---|"]
    for name, v in sorted(rec["kernels"].items(), key=lambda kv: -kv[1]["bytes"]):
        short = name.split("(")[0].split("::")[-1]
        base = short.split("<")[0]
        a = algorithmic.get(base)
        ratio = (f"{v['bytes_random'] / a:.2f} - {v['bytes'] / a:.2f}" if rnd else f"{v['bytes'] / a:.2f}") if a else "-"
        lines.append(f"| {short} | {v['fetch_kib']:.0f} | {v['write_kib']:.0f} | {v['bytes'] / 1e6:.1f} MB | "
                     + (f"{v['bytes_random'] / 1e6:.1f} MB | " if rnd else "")
                     + (f"{a / 1e6:.1f} MB | {ratio} |" if a else "- | - |"))
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
    b.add_argument("--gather-fetch", default=None)
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
        rec = traffic(args.fetch, args.write, args.copy_fetch, args.copy_write, args.gather_fetch)
        rec["command"] = args.command
        with open(args.out, "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
