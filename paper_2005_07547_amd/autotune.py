"""Autotuner for the launch parameters of the hash path.

Sweeps the tunables of the partitioned insert -- records per thread of the
binning pass (``bin_per``: tile size and LDS staging width), slots per
partition (``part_log2``: the LDS hash width of the merge pass) -- and the
insert strategy (partitioned vs. wave-merged direct atomics) on caller-given
device-resident iterations, timing whole ``psf_iterate`` calls with HIP
events.  The result is a ranked list and the best configuration; ``tune``
optionally records it in a JSON table keyed by workload name, which
``best_params`` reads back.
"""
from __future__ import annotations

import itertools
import json
import os
import time

from . import psf

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")

DEFAULT_SPACE = {
    "insert_mode": [psf.PSF_INSERT_PARTITIONED],
    "bin_per": [8, 12, 16],
    "part_log2": [10, 11, 12],
}


def candidates(space=None):
    space = dict(DEFAULT_SPACE if space is None else space)
    keys = sorted(space)
    for vals in itertools.product(*(space[k] for k in keys)):
        c = dict(zip(keys, vals))
        if c.get("insert_mode") == psf.PSF_INSERT_DIRECT:
            c.pop("bin_per", None)
            c.pop("part_log2", None)
        yield c


def time_config(table_cfg: dict, params: dict, bufs: list, warmup: int = 2, iters: int = 8):
    """Median ms per psf_iterate over iters iterations (fresh table)."""
    import torch
    cfg = dict(table_cfg)
    cfg.update(params)
    n = int(bufs[0]["px"].numel())
    cfg.setdefault("max_batch", n)
    t = psf.Table(**cfg)
    out = torch.empty((3, n), dtype=torch.float32, device="cuda")
    found = torch.empty(n, dtype=torch.uint8, device="cuda")
    for i in range(warmup):
        t.iterate(bufs[i % len(bufs)], out=out, found=found)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(iters)]
    torch.cuda.synchronize()
    for k in range(iters):
        ev[k][0].record()
        t.iterate(bufs[(warmup + k) % len(bufs)], out=out, found=found)
        ev[k][1].record()
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    st = t.stats()
    t.close()
    return {"ms": ms[len(ms) // 2], "min_ms": ms[0], "dropped": st["dropped"]}


def tune(table_cfg: dict, bufs: list, space=None, name: str | None = None, record: bool = False,
         warmup: int = 2, iters: int = 8, log=None):
    """Time every candidate; return (best params, ranked results)."""
    results = []
    for c in candidates(space):
        try:
            r = time_config(table_cfg, c, bufs, warmup, iters)
        except psf.PsfError as e:  # e.g. a configuration this table size cannot use
            r = {"ms": float("inf"), "error": str(e)}
        r["params"] = c
        results.append(r)
        if log:
            log(f"{c} -> {r.get('ms'):.4f} ms")
    results.sort(key=lambda r: (r.get("dropped", 0) > 0, r["ms"]))
    best = results[0]["params"]
    if record and name:
        table = {}
        if os.path.exists(TABLE_PATH):
            with open(TABLE_PATH) as f:
                table = json.load(f)
        table[name] = {"params": best, "ms": results[0]["ms"], "n": int(bufs[0]["px"].numel()),
                       "log2_slots": table_cfg.get("log2_slots"), "when": time.strftime("%Y-%m-%d")}
        with open(TABLE_PATH, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return best, results


def best_params(name: str, default=None) -> dict:
    """Tuned parameters recorded for a workload name (or default / {})."""
    if os.path.exists(TABLE_PATH):
        with open(TABLE_PATH) as f:
            table = json.load(f)
        if name in table:
            return dict(table[name]["params"])
    return dict(default or {})
