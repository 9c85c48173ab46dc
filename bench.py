#!/usr/bin/env python3
"""Throughput benchmark of the PSTF hash path on one MI355X.

One step is one whole iteration of the hot path on the plain workload
(1280x720, 1 spp, 4 vertices per path = 3,686,400 vertex records; 2^22-slot
table; Eq. 11 with T_max = 5): insert every record, apply the temporal blend,
then query the approximant at every record (psf_iterate).  Inputs are
synthetic (procedural scene generator, seeded) and resident in HBM before the
timed region.  `value` comes from a pass without per-kernel instrumentation;
a second pass of the same length brackets every kernel launch with HIP events
on the library's stream and gives the per-kernel times and the roofline of
the dominant kernel.  The JSON line also carries the CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
REC_BYTES = 52         # position, normal, direction, rgb, roughness (f32)
QRY_BYTES = 40 + 12    # query fields in, rgb out
CELL_INSERT, CELL_UPDATE, CELL_QUERY = 40, 64, 24


def _workload(name):
    from synth import workloads as W
    return {"plain": W.plain, "tiny": W.tiny, "precision": W.precision}[name]()


def algorithmic_bytes(n, c, state_bytes=4):
    """Bytes the method must move per iteration for n records (queries = n)
    touching c distinct cells, split by kernel kind.  With 16-bit state
    (state_bytes 2) a cell's update reads and writes 6 bytes of approximant
    instead of 12 and a lookup reads 6 instead of 12."""
    upd = CELL_UPDATE - 2 * 3 * (4 - state_bytes)
    qry = CELL_QUERY - 3 * (4 - state_bytes)
    return {
        "bin": n * REC_BYTES,
        "merge_blend": c * (CELL_INSERT + upd),
        "query": n * QRY_BYTES + c * qry,
        "iteration": n * (REC_BYTES + QRY_BYTES) + c * (CELL_INSERT + upd + qry),
    }


KERNEL_SYMBOL = {"bin": "k_bin", "merge_blend": "k_merge", "query": "k_unstage",
                 "merge": "k_merge", "update": "k_update", "insert_direct": "k_insert_direct"}


def measured_traffic(workload: str, kernel: str, key: str = "bytes"):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary (profiles/traffic_<workload>.json; key "bytes": FETCH_SIZE at the
    streaming copy's scale, "bytes_random": at the random-gather scale), or
    None when there is none or the kernel sources changed since it was
    taken."""
    from paper_2005_07547_amd import profiling
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("digest") != profiling.source_digest():
        return None
    sym = KERNEL_SYMBOL.get(kernel, kernel)
    # rocprofv3 records demangled names ("void psf::k_merge<true>(...)")
    pat = re.compile(r"(^|[\s:])" + re.escape(sym) + r"[<(]")
    hits = [v for name, v in rec["kernels"].items() if pat.search(name)]
    return int(hits[0][key]) if len(hits) == 1 and key in hits[0] else None


def device_rates(torch, dev, reps=5):
    """Rates of the memory operations the hash path is made of, measured with
    HIP events over torch's own kernels: a streaming 1 GiB copy (bytes moved
    per second), gathers of 2^24 random 16-byte rows (torch.take of each
    row's four words; rows per second) and
    2^24 random binary32 and u32 atomic adds (index_add_, adds per second),
    each from a 4 GiB table (beyond the L2 and the Infinity Cache) and a
    2 MiB one (L2-resident).  Seeded indices; the best of `reps` launches."""
    def best(fn):
        ts = []
        for _ in range(reps + 1):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b) / 1e3)
        return min(ts[1:])
    out = {}
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    t = best(lambda: dst.copy_(src))
    out["copy_GBps"] = round(2 * nbytes / t / 1e9, 1)
    del src, dst
    g = torch.Generator(device="cpu").manual_seed(7)
    rows = 1 << 24
    for label, table_bytes in (("beyond_l2", 1 << 32), ("l2_resident", 1 << 21)):
        table = torch.ones(table_bytes // 4, dtype=torch.float32, device=dev)
        # a 16-byte row is read as its four words (torch.take; the row
        # kernels of index_select run far below the memory system here)
        idx = torch.randint(0, table.numel() // 4, (rows,), generator=g).to(dev)
        words = (idx * 4).unsqueeze(1) + torch.arange(4, device=dev)
        t = best(lambda: torch.take(table, words))
        out[f"gather16_{label}_rows_per_s"] = float(f"{rows / t:.3g}")
        del words
        flat_idx = torch.randint(0, table.numel(), (rows,), generator=g).to(dev)
        vals = torch.ones(rows, dtype=torch.float32, device=dev)
        t = best(lambda: table.index_add_(0, flat_idx, vals))
        out[f"atomic_f32_{label}_per_s"] = float(f"{rows / t:.3g}")
        itable = table.view(torch.int32)
        ivals = torch.ones(rows, dtype=torch.int32, device=dev)
        t = best(lambda: itable.index_add_(0, flat_idx, ivals))
        out[f"atomic_u32_{label}_per_s"] = float(f"{rows / t:.3g}")
        del table, idx, flat_idx, vals, ivals, itable
        torch.cuda.empty_cache()
    return out


def _oracle_rate(orc, rec, budget_s):
    """Whole iterations (insert, update, query) of rec on orc until the time
    budget is used (at least one); returns (records/s, iterations, seconds)."""
    n = len(rec["px"])
    t0 = time.perf_counter()
    done = 0
    while True:
        orc.insert(rec)
        orc.update()
        orc.query(rec)
        done += 1
        el = time.perf_counter() - t0
        if el >= budget_s or el / done * (done + 1) > budget_s * 1.5:
            break
    return n * done / el, done, el


def cpu_baseline(wl, rec, budget_s):
    """The oracle as it stands on the host cores: the key-sharded variant on
    every host thread (the headline value) and the single-threaded oracle,
    each on whole iterations of the same records within its time budget."""
    import oracle
    n = len(rec["px"])
    threads = max(1, min(16, os.cpu_count() or 1))
    many, done_m, el_m = _oracle_rate(oracle.ShardedOracle(threads, **wl["table"]), rec, budget_s)
    one, done_1, el_1 = _oracle_rate(oracle.Oracle(**wl["table"]), rec, budget_s / 2)
    return {"value": round(many, 1), "unit": "vertex records/s", "cores": threads, "kind": "oracle",
            "sample": f"{done_m} whole iteration(s) (insert+update+query) of {n} records of the "
                      f"{wl['name']} workload, key-sharded oracle on {threads} host threads, {el_m:.1f} s",
            "single_thread": {"value": round(one, 1), "cores": 1,
                              "sample": f"{done_1} whole iteration(s) of the same records, {el_1:.1f} s"},
            "host_cpu": host_cpu(), "host_threads": os.cpu_count()}


def host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def device_info(torch) -> dict:
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": getattr(p, "gcnArchName", ""), "compute_units": p.multi_processor_count,
            "memory_gib": round(p.total_memory / 2 ** 30, 1)}


def _dev(rec, torch):
    return {k: (None if v is None else torch.from_numpy(v).cuda()) for k, v in rec.items()}


TUNED = {"use": True}


def tuned(name: str) -> dict:
    """Launch parameters the autotuner recorded for a workload (the
    committed paper_2005_07547_amd/tuning.json), or {} with --untuned."""
    if not TUNED["use"]:
        return {}
    from paper_2005_07547_amd import autotune
    return autotune.best_params(name)


def with_params(cfg: dict, params: dict, flags: int = 0) -> dict:
    c = dict(cfg)
    c.update(params)
    c["flags"] = int(params.get("flags", 0)) | flags
    return c


PRECISION_STATES = (("f32", 0), ("f16", 1), ("bf16", 2), ("f16_ef", 3), ("bf16_ef", 4))


def form_precision(torch, psf, W, iters=64, pool=16):
    """Precision workload (1920x1080, 5 vertices, HDR lognormal(0, 2), 2^24
    slots): the config's 64 iterations on a fresh table per state format
    (FP32; FP16 and BF16 re-rounded every blend; both with the FP32
    rounding residual carried), frames cycled from a pool of 16 distinct
    iterations resident in HBM.  A second pass of the same length brackets
    every kernel with HIP events for the per-kernel times and the roofline."""
    import numpy as np
    wl = W.precision()
    sc = W.make_scene(wl)
    n = W.records_per_iteration(wl)
    frames = [_dev(sc.generate(wl["gen"], i), torch) for i in range(pool)]
    params = tuned(wl["name"])
    o = torch.empty((3, n), dtype=torch.float32, device="cuda")
    f = torch.empty(n, dtype=torch.uint8, device="cuda")
    out = {}
    for name, code in PRECISION_STATES:
        res = {}
        for flags in (0, psf.PSF_FLAG_TIMING):
            t = psf.Table(**dict(with_params(wl["table"], params, flags), max_batch=n, state_dtype=code))
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(iters)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(iters):
                ev[k][0].record()
                t.iterate(frames[k % pool], out=o, found=f)
                ev[k][1].record()
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            st = t.stats()
            if flags:
                kt = {k: {"launches": v[0], "avg_ms": round(v[1] / max(1, v[0]), 5)}
                      for k, v in t.kernel_times().items()}
                touched = st["touched_total"] / max(1, st["updates"])
                ab = algorithmic_bytes(n, touched, state_bytes=4 if code == 0 else 2)
                dom = max(kt, key=lambda k: kt[k]["avg_ms"] * kt[k]["launches"])
                ach = ab.get(dom, 0) / (kt[dom]["avg_ms"] * 1e-3) / 1e9
                res.update({"kernels": kt, "cells_touched_per_iteration": int(touched),
                            "algorithmic_bytes_per_iteration": int(ab["iteration"]),
                            "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1),
                                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                                         "algorithmic_bytes_per_launch": int(ab.get(dom, 0)),
                                         "avg_launch_ms": kt[dom]["avg_ms"]}})
            else:
                ms = np.array([a.elapsed_time(b) for a, b in ev])
                res.update({"records_per_s": round(n * iters / el, 1), "ms_per_iter": round(el / iters * 1e3, 4),
                            "p50_iter_ms": round(float(np.percentile(ms, 50)), 4),
                            "p99_iter_ms": round(float(np.percentile(ms, 99)), 4),
                            "saturated": st["saturated"], "dropped": st["dropped"]})
            t.close()
        touched = res["cells_touched_per_iteration"]
        res["iteration_hbm_frac"] = round(algorithmic_bytes(n, touched, state_bytes=4 if code == 0 else 2)
                                          ["iteration"] / (res["ms_per_iter"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        out[name] = res
    del frames
    return {"workload": wl["name"], "records_per_iteration": n, "iterations": iters,
            "frames": f"{pool} distinct iterations resident in HBM, cycled", "params": params,
            "by_state": out,
            "note": "error vs the binary64 oracle over all 64 iterations is asserted in tests/test_gpu_precision.py"}


def form_batched(torch, psf, W, iters=8, sessions=16):
    """16 uneven sessions: one batched iteration per step versus the same
    sessions iterated one after another (plain per-session path)."""
    import numpy as np
    wls = W.batched_sessions(sessions)
    frames, ns = [], []
    for wl in wls:
        sc = W.make_scene(wl)
        frames.append([_dev(sc.generate(wl["gen"], i), torch) for i in range(2)])
        ns.append(W.records_per_iteration(wl))
    total = sum(ns)
    res = {}
    for mode in ("plain_per_session", "batched"):
        tabs = [psf.Table(**dict(with_params(wl["table"], tuned("batched-16")), max_batch=n))
                for wl, n in zip(wls, ns)]
        outs = [torch.empty((3, n), dtype=torch.float32, device="cuda") for n in ns]
        fnds = [torch.empty(n, dtype=torch.uint8, device="cuda") for n in ns]
        batch = psf.Batch(len(wls))

        def step(k):
            fr = [f[k % 2] for f in frames]
            if mode == "batched":
                batch.iterate(tabs, fr, outs=outs, founds=fnds)
            else:
                for t, r, o, f in zip(tabs, fr, outs, fnds):
                    t.iterate(r, out=o, found=f)

        for k in range(2):
            step(k)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(iters)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(iters):
            ev[k][0].record()
            step(k)
            ev[k][1].record()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ms = np.array([a.elapsed_time(b) for a, b in ev])
        res[mode] = {"records_per_s": round(total * iters / el, 1),
                     "ms_per_iter": round(el / iters * 1e3, 4),
                     "p50_iter_ms": round(float(np.percentile(ms, 50)), 4),
                     "p99_iter_ms": round(float(np.percentile(ms, 99)), 4),
                     "dropped": int(sum(t.stats()["dropped"] for t in tabs))}
        if mode == "batched":
            # the same batched iteration captured once per frame in a HIP
            # graph (one context per graph) and replayed
            ctxs = [psf.Batch(len(wls)) for _ in range(2)]
            graphs = []
            gs = torch.cuda.Stream()
            gs.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(gs):
                for k in range(2):
                    g = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g, stream=gs):
                        ctxs[k].iterate(tabs, [f[k] for f in frames], outs=outs, founds=fnds)
                    graphs.append(g)
            torch.cuda.current_stream().wait_stream(gs)
            for k in range(2):
                graphs[k].replay()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(iters):
                graphs[k % 2].replay()
            torch.cuda.synchronize()
            gel = time.perf_counter() - t0
            res["batched_graph_replay"] = {"records_per_s": round(total * iters / gel, 1),
                                           "ms_per_iter": round(gel / iters * 1e3, 4)}
            del graphs
            for c in ctxs:
                c.close()
        for t in tabs:
            t.close()
        batch.close()
        del tabs, outs, fnds
    res["speedup_batched_over_plain"] = round(res["batched"]["records_per_s"] /
                                              res["plain_per_session"]["records_per_s"], 3)
    return {"sessions": len(wls), "records_per_iteration": total, "params": tuned("batched-16"), **res}


EST_IN_BYTES = 17 * 4      # position, normal, two directions, roughness, g, w/p
EST_OUT_BYTES = 12 + 1     # estimate rgb, applied flag
EST_CELL_BYTES = 2 * 24    # two cell lookups (key + state)


def form_estimate(torch, psf, W, iters=32, warm_frames=4):
    """Two fields per cell and the fused estimator epilogue on the plain
    workload: both fields are learned over a few frames, then every vertex of
    a frame gets the control-variate estimate (beta 0.75) in one call."""
    import numpy as np
    wl = W.plain()
    sc = W.make_scene(wl)
    n = W.records_per_iteration(wl)
    params = tuned(wl["name"])
    oe = psf.Table(**dict(with_params(wl["table"], params, psf.PSF_FLAG_TIMING), max_batch=n))
    fl = psf.Table(**dict(with_params(W.fl_table(wl["table"]), params), max_batch=n))
    a = None
    for i in range(warm_frames):
        rec = sc.generate(wl["gen"], i)
        args, flr = W.estimator_inputs(rec, wl["gen"])
        oe.iterate(_dev(rec, torch))
        fl.iterate(_dev(flr, torch))
        a = _dev(args, torch)
    out = torch.empty((3, n), dtype=torch.float32, device="cuda")
    app = torch.empty(n, dtype=torch.uint8, device="cuda")
    for _ in range(2):
        psf.estimate(oe, fl, a, psf.PSF_EST_CV, 0.75, out=out, applied=app)
    torch.cuda.synchronize()
    oe.kernel_times(reset=True)
    t0 = time.perf_counter()
    for _ in range(iters):
        psf.estimate(oe, fl, a, psf.PSF_EST_CV, 0.75, out=out, applied=app)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt = oe.kernel_times()
    launches, total = kt.get("estimate", (0, 0.0))
    avg_ms = total / max(1, launches)
    per_launch = n * (EST_IN_BYTES + EST_OUT_BYTES + EST_CELL_BYTES)
    ach = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None
    res = {"workload": wl["name"], "vertices": n, "mode": "control variate, beta 0.75",
           "vertices_per_s": round(n * iters / el, 1), "ms_per_call": round(el / iters * 1e3, 4),
           "applied_fraction": round(float(app.float().mean()), 4),
           "roofline": {"bound": "hbm", "kernel": "estimate", "achieved": None if ach is None else round(ach, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": None if ach is None else round(ach / HBM_PEAK_GBS, 4),
                        "algorithmic_bytes_per_launch": per_launch, "avg_launch_ms": round(avg_ms, 5)}}
    oe.close()
    fl.close()
    return res


def form_progressive(torch, psf, W, iters=16, width=1280, height=720, verts=4):
    """The progressive solver with its path sampler on the GPU (Sec. 2.2;
    Algorithm 2 with next-event estimation): every frame psf_sample_paths
    traces one path per pixel through the tiny workload's box (emitter under
    the ceiling; camera inside the box so every pixel sees it) and
    psf_progressive_step looks up the previous approximant at each path's
    next vertex, forms the samples, inserts and blends them -- nothing
    leaves the device.  Also: the closed furnace run to convergence the same
    way, against rho L_e / (1 - rho)."""
    import numpy as np
    prims, _ = W.box_scene()
    scene = psf.Scene(prims)
    cam = psf.camera((0.5, 0.5, 0.02), (0.0, 0.0, 1.0), (0.0, 1.0, 0.0), 60.0, width, height, 1)
    n = width * height * verts
    cfg = dict(W.tiny()["table"], log2_slots=23, flags=psf.PSF_FLAG_TIMING, cam=(0.5, 0.5, 0.02),
               kappa=W.kappa_for(60.0, height, 4.0, -10), e_min=-10)
    t = psf.Table(**dict(cfg, max_batch=n))
    samples = torch.empty((3, n), dtype=torch.float32, device="cuda")
    buf = None

    def frame(k):
        nonlocal buf
        x, nx, tp, le = psf.sample_paths(scene, cam, verts, psf.PSF_PATHS_LOE, psf.PSF_ORIGIN_CAMERA, seed=17,
                                         frame=k, out=buf)
        if buf is None:
            buf = dict(x, qx=nx["px"], qy=nx["py"], qz=nx["pz"], qnx=nx["nx"], qny=nx["ny"], qnz=nx["nz"],
                       qox=nx["ox"], qoy=nx["oy"], qoz=nx["oz"], qrough=nx["rough"], t_r=tp[0], t_g=tp[1],
                       t_b=tp[2], le_r=le[0], le_g=le[1], le_b=le[2])
        return x, nx, tp, le

    for k in range(4):
        x, nx, tp, le = frame(k)
        t.progressive_step(x, nx, tp, le, out=samples)
    torch.cuda.synchronize()
    t.kernel_times(reset=True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(iters)]
    t0 = time.perf_counter()
    for k in range(iters):
        ev[k][0].record()
        x, nx, tp, le = frame(4 + k)
        ev[k][1].record()
        t.progressive_step(x, nx, tp, le, out=samples)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt = {k: round(v[1] / max(1, v[0]), 5) for k, v in t.kernel_times().items()}
    kt["sample_paths"] = round(float(np.mean([a.elapsed_time(b) for a, b in ev])), 5)
    st = t.stats()
    res = {"scene": "box of the tiny workload with a 0.5 x 0.5 emitter, camera inside, Algorithm 2 with NEE",
           "paths": width * height, "vertices_per_path": verts, "records_per_frame": n,
           "records_per_s": round(n * iters / el, 1), "ms_per_frame": round(el / iters * 1e3, 4),
           "kernels_avg_ms": kt, "skipped_per_frame": st["skipped"] // (iters + 4), "dropped": st["dropped"],
           "frames_run": iters + 4}
    t.close()
    # the closed furnace, every frame sampled and filtered on the device
    le_f, rho = np.array([1.0, 0.5, 0.25]), np.array([0.5, 0.6, 0.7])
    fs = psf.Scene(W.furnace_scene(tuple(le_f), tuple(rho)))
    fcam = psf.camera((0, 0, 0), (0, 0, 1), (0, 1, 0), 60.0, 65536, 1)
    ft = psf.Table(**W.furnace_table())
    for k in range(200):
        x, nx, tp, le = psf.sample_paths(fs, fcam, 2, psf.PSF_PATHS_LOE, psf.PSF_ORIGIN_POINT, seed=23, frame=k)
        ft.progressive_step(x, nx, tp, le)
    L = ft.export()["L"].astype(np.float64)
    want = (rho * le_f / (1.0 - rho))[:, None]
    rel = np.abs(L / want - 1.0)
    res["furnace"] = {"frames": 200, "paths_per_frame": 65536, "vertices_per_path": 2,
                      "field": "L_o minus emission (Algorithm 2, NEE + balance heuristic)",
                      "mean_rel_error_to_closed_form": round(float(rel.mean()), 7),
                      "p90_rel_error": round(float(np.percentile(rel, 90)), 7)}
    ft.close()
    return res


def form_weighted(torch, psf, W, iters=16):
    """MIS-weighted counters (Eq. 5-6 with w != 1): the plain workload's fused
    iteration on a weighted table whose records carry balance-heuristic
    weights (10% of them 0: a technique the field leaves out), beside the
    same frames on an unweighted table; per-kernel averages from HIP events."""
    wl = W.plain()
    sc = W.make_scene(wl)
    n = W.records_per_iteration(wl)
    frames = []
    for i in range(2):
        rec = dict(sc.generate(wl["gen"], i))
        rec["weight"] = W.mis_weights(n, seed=40 + i, excluded=0.1)
        frames.append(_dev(rec, torch))
    plain = [{k: v for k, v in f.items() if k != "weight"} for f in frames]
    # the weighted table takes its own default partition width (its merge
    # holds a binary64 weight sum per slot in LDS as well)
    pw = dict(tuned(wl["name"]), part_log2=0)
    res = {"workload": wl["name"], "records_per_iteration": n, "params": tuned(wl["name"]),
           "params_weighted": pw, "weights": "balance heuristic of two lognormal(0, 1) densities, 10% zero"}
    for name, weighted, fr in (("weighted", 1, frames), ("unweighted", 0, plain)):
        p = pw if weighted else tuned(wl["name"])
        t = psf.Table(**dict(with_params(wl["table"], p, psf.PSF_FLAG_TIMING), max_batch=n, weighted=weighted))
        o = torch.empty((3, n), dtype=torch.float32, device="cuda")
        f = torch.empty(n, dtype=torch.uint8, device="cuda")
        for i in range(4):
            t.iterate(fr[i % 2], out=o, found=f)
        torch.cuda.synchronize()
        t.kernel_times(reset=True)
        t0 = time.perf_counter()
        for k in range(iters):
            t.iterate(fr[k % 2], out=o, found=f)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        kt = {k: round(v[1] / max(1, v[0]), 5) for k, v in t.kernel_times().items()}
        st = t.stats()
        res[name] = {"records_per_s": round(n * iters / el, 1), "ms_per_iter": round(el / iters * 1e3, 4),
                     "kernels_avg_ms": kt, "skipped_per_iter": st["skipped"] // (iters + 4),
                     "dropped": st["dropped"]}
        t.close()
    res["note"] = ("per-kernel events add a little to ms_per_iter; error vs the binary64 oracle is "
                   "asserted in tests/test_gpu_weights.py")
    return res


def form_serving(torch, psf, W, n_sessions=48, rate=20.0, budget_gb=200.0, frames_per_session=3):
    """Poisson arrivals at 20/s, resolutions lognormal around 720p, 32-128
    iterations each, 1 spp, 4 vertices; continuous batching under an HBM
    budget.  Every session renders a scene of its own (seeded by the
    session, diffuse-only or half glossy) and cycles through frames of its
    own distinct iterations, resident in HBM before the run."""
    from paper_2005_07547_amd import serving
    from synth import Scene
    draws = serving.draw_requests(n_sessions, rate=rate, seed=5)
    reqs = []
    wl = W.plain()
    for sid, arrival, cls, iters, seed in draws:
        w, h = serving.RES_CLASSES[cls]
        gen = dict(wl["gen"], width=w, height=h, seed=seed)
        sc = Scene(Scene.RANDOM, seed=seed, glossy_frac=-1.0 if sid % 2 else 0.5)
        frames = [_dev(sc.generate(gen, f), torch) for f in range(frames_per_session)]
        log2 = int(min(25, max(16, math.ceil(math.log2(w * h * 4)) + 1)))
        # sessions take the launch parameters tuned for the batched form
        # (many uneven sessions sharing launches)
        cfg = with_params(dict(wl["table"], log2_slots=log2,
                               kappa=W.kappa_for(60.0, h, 8.0 * math.sqrt(2.0), -5)),
                          tuned("batched-16"))
        reqs.append(serving.SessionRequest(sid=sid, arrival=arrival, iterations=iters, table_cfg=cfg,
                                           frames=frames, records=w * h * 4))
    srv = serving.Server(budget_bytes=int(budget_gb * (1 << 30)), max_active=64)
    summ = srv.run(reqs, time_limit=240)
    summ = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in summ.items()}
    summ.update({"arrival_rate_per_s": rate, "budget_gb": budget_gb})

    # At 20 arrivals/s the device idles between sessions, so the rate above
    # is the arrival rate's.  The server's capacity: the same sessions all
    # arriving at once, beside the plain path running them one after another.
    def fresh():
        return [serving.SessionRequest(sid=r.sid, arrival=0.0, iterations=r.iterations, table_cfg=r.table_cfg,
                                       frames=r.frames, records=r.records) for r in reqs]

    # (run twice: the first pays the device allocations of 48 resident
    # tables, which the plain path below, freeing each table before the
    # next, reuses from torch's cache; the second run is timed)
    sat_cold = None
    for _ in range(2):
        srv = serving.Server(budget_bytes=int(budget_gb * (1 << 30)), max_active=64)
        sat = srv.run(fresh(), time_limit=240)
        sat_cold = sat_cold or sat
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    for r in fresh():
        tab = psf.Table(**dict(r.table_cfg, max_batch=max(1, r.records)))
        o = torch.empty((3, r.records), dtype=torch.float32, device="cuda")
        f = torch.empty(r.records, dtype=torch.uint8, device="cuda")
        for i in range(r.iterations):
            tab.iterate(r.frames[i % len(r.frames)], out=o, found=f)
        torch.cuda.synchronize()
        done += r.records * r.iterations
        tab.close()
    plain_el = time.perf_counter() - t0
    summ["all_at_once"] = {"records_per_s": round(sat["records_per_s"], 1), "wall_s": round(sat["wall_s"], 4),
                           "p50_iter_ms": round(sat["p50_iter_ms"], 4), "p99_iter_ms": round(sat["p99_iter_ms"], 4),
                           "peak_active": sat["peak_active"], "dropped": sat["dropped"],
                           "first_run_records_per_s": round(sat_cold["records_per_s"], 1)}
    summ["plain_one_session_after_another"] = {"records_per_s": round(done / plain_el, 1),
                                               "wall_s": round(plain_el, 4)}
    summ["speedup_served_over_plain"] = round(sat["records_per_s"] / (done / plain_el), 3)
    summ["frames"] = (f"a scene per session, {frames_per_session} distinct iterations per session cycled, "
                      "resident in HBM")
    return summ


def graph_replay(torch, psf, wl, bufs, out, found, steps, n, params=None):
    """The same iterations replayed from HIP graphs (one graph per input
    buffer, captured from psf_iterate on a fresh table after an eager warm-up):
    launch overhead removed."""
    t = psf.Table(**dict(with_params(wl["table"], params or {}), max_batch=max(n, 1)))
    for b in bufs[:2]:
        t.iterate(b, out=out, found=found)
    torch.cuda.synchronize()
    graphs = []
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for b in bufs:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                t.iterate(b, out=out, found=found)
            graphs.append(g)
    torch.cuda.current_stream().wait_stream(s)
    for k in range(2):
        graphs[k % len(graphs)].replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        graphs[k % len(graphs)].replay()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    t.close()
    return {"value": round(n * steps / el, 1), "ms_per_step": round(el / steps * 1e3, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=32)
    ap.add_argument("--repeats", type=int, default=10,
                    help="fresh-table repeats of `steps` iterations for p50/p99")
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--workload", default="plain", choices=["plain", "tiny", "precision"])
    ap.add_argument("--pool", type=int, default=8, help="distinct iteration buffers, cycled")
    ap.add_argument("--insert-mode", type=int, default=0)
    ap.add_argument("--split", action="store_true", help="separate insert/update/query calls")
    ap.add_argument("--state", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="no per-kernel events")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay measurement")
    ap.add_argument("--forms", default="precision,batched,serving,estimate,progressive,weighted",
                    help="comma list of extra forms to measure (precision,batched,serving,estimate,"
                         "progressive,weighted) or ''")
    ap.add_argument("--untuned", action="store_true",
                    help="library default launch parameters instead of the recorded tuned ones")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run only a plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--gather-calib", action="store_true",
                    help="run only random row gathers of known bytes (32, 64 and 128-byte rows from a "
                         "4 GiB table; calibrates HBM byte counters for random requests)")
    ap.add_argument("--rates", action="store_true",
                    help="run only the device-rate probes: streaming copy, random 16-byte row gathers "
                         "and random binary32/u32 atomics, beyond and within the L2 (torch kernels)")
    args = ap.parse_args()
    TUNED["use"] = not args.untuned

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the hash path is "
                                   "measured on a single MI355X (--gpus 1)"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2005_07547_amd import psf
    from synth import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calib:
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_read": nbytes, "copy_calib_bytes_written": nbytes,
                          "launches": 3}), flush=True)
        return
    if args.rates:
        print(json.dumps({"rates": device_rates(torch, dev)}), flush=True)
        return
    if args.gather_calib:
        # 2^24 rows gathered per launch at seeded random row indices from a
        # table far larger than the L2 and the Infinity Cache; each launch
        # reads rows * row_bytes of the table plus 8-byte indices and writes
        # rows * row_bytes.  One launch per row width, in order 32, 64, 128.
        rows = 1 << 24
        table = torch.ones(1 << 30, dtype=torch.float32, device=dev)  # 4 GiB
        g = torch.Generator(device="cpu").manual_seed(12345)
        out = {}
        for row_bytes in (32, 64, 128):
            width = row_bytes // 4
            view = table.view(-1, width)
            idx = torch.randint(0, view.shape[0], (rows,), generator=g).to(dev)
            torch.cuda.synchronize()
            got = torch.index_select(view, 0, idx)
            torch.cuda.synchronize()
            out[row_bytes] = {"rows": rows, "table_bytes_read": rows * row_bytes, "index_bytes_read": rows * 8,
                              "bytes_written": rows * row_bytes, "checksum": float(got.sum())}
            del got, idx
        print(json.dumps({"gather_calib": out}), flush=True)
        return
    wl = _workload(args.workload)
    sc = W.make_scene(wl)
    n = W.records_per_iteration(wl)
    pool = max(1, min(args.pool, args.warmup + args.steps))
    host = []
    bufs = []
    for i in range(pool):
        rec = sc.generate(wl["gen"], i)
        if wl["diffuse_only"]:
            rec = dict(rec)
            rec["rough"] = None
        host.append(rec)
        bufs.append({k: (None if v is None else torch.from_numpy(v).to(dev)) for k, v in rec.items()})
    out = torch.empty((3, n), dtype=torch.float32, device=dev)
    found = torch.empty(n, dtype=torch.uint8, device=dev)
    dtype_code = {"f32": psf.PSF_STATE_F32, "f16": psf.PSF_STATE_F16, "bf16": psf.PSF_STATE_BF16}[args.state]
    params = tuned(wl["name"]) if args.insert_mode == psf.PSF_INSERT_AUTO else {}
    steps = args.steps

    def timed_pass(flags, steps=steps, warmup=args.warmup):
        """Warm up, then time exactly `steps` iterations of a fresh table
        (wall clock around the loop, HIP events around every step)."""
        table = psf.Table(**dict(with_params(wl["table"], params, flags), state_dtype=dtype_code,
                                 max_batch=max(n, 1), **({} if params else {"insert_mode": args.insert_mode})))

        def step(i):
            b = bufs[i % pool]
            if args.split:
                table.insert(b)
                table.update()
                table.query(b, out=out, found=found)
            else:
                table.iterate(b, out=out, found=found)

        for i in range(warmup):
            step(i)
        torch.cuda.synchronize()
        if flags & psf.PSF_FLAG_TIMING:
            table.kernel_times(reset=True)
        st0 = table.stats()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            ev[k][0].record()
            step(warmup + k)
            ev[k][1].record()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        iter_ms = np.array([x.elapsed_time(y) for x, y in ev])
        st1 = table.stats()
        kt = table.kernel_times() if flags & psf.PSF_FLAG_TIMING else {}
        table.close()
        return el, iter_ms, st0, st1, kt

    # the measured pass runs the library as a caller would (no per-kernel
    # events); a second pass of the same length brackets every kernel launch
    # with HIP events on the library's stream for the per-kernel times and
    # the roofline
    elapsed, iter_ms, st0, st1, _ = timed_pass(0)
    # per-iteration latency: every iteration of `repeats` runs, each on a
    # fresh table (its first frames included)
    lat = [iter_ms] + [timed_pass(0, warmup=0)[1] for _ in range(max(0, args.repeats - 1))]
    lat = np.concatenate(lat)
    kt, inst_ms, probes = {}, None, None
    if not args.no_timing:
        el2, _, _, _, kt = timed_pass(psf.PSF_FLAG_TIMING)
        inst_ms = round(el2 / steps * 1e3, 4)
        # probes each inserted sample needed in its partition (last bin: 16+),
        # from a short pass of its own (the histogram costs LDS atomics)
        _, _, p0, p1, _ = timed_pass(psf.PSF_FLAG_PROBE_STATS, min(steps, 4))
        probes = [int(b - a) for a, b in zip(p0["probe_hist"], p1["probe_hist"])]
        while len(probes) > 1 and probes[-1] == 0:
            probes.pop()
    touched = (st1["touched_total"] - st0["touched_total"]) / max(1, st1["updates"] - st0["updates"])
    ab = algorithmic_bytes(n, touched)
    kernels = {k: {"launches": v[0], "avg_ms": v[1] / max(1, v[0])} for k, v in kt.items()}
    roofline = None
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
        per_launch = ab.get(dom)
        if per_launch is None:  # split mode kernels: attribute the insert bytes
            per_launch = {"merge": touched * CELL_INSERT, "update": touched * CELL_UPDATE,
                          "insert_direct": n * REC_BYTES + touched * CELL_INSERT}.get(dom, 0)
        ach = per_launch / (kernels[dom]["avg_ms"] * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(wl["name"], dom),
                    "traffic_random_scale": measured_traffic(wl["name"], dom, "bytes_random"),
                    "algorithmic_bytes_per_launch": int(per_launch),
                    "avg_launch_ms": round(kernels[dom]["avg_ms"], 5)}
    iter_gbs = ab["iteration"] / (elapsed / steps) / 1e9
    result = {
        "metric": "vertex records/s (insert+temporal update+query)",
        "value": round(n * steps / elapsed, 1),
        "unit": "vertex records/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.state == "f32" else f"f32 accumulate, {args.state} state",
        "data": "synthetic (seeded procedural scene, records resident in HBM)",
        "config": {"workload": wl["name"], "records_per_iteration": n,
                   "log2_slots": wl["table"]["log2_slots"], "iterations_timed": steps,
                   "mode": "split" if args.split else "psf_iterate",
                   "insert_mode": args.insert_mode, "pool_buffers": pool, "params": params},
        "p50_iter_ms": round(float(np.percentile(lat, 50)), 4),
        "p99_iter_ms": round(float(np.percentile(lat, 99)), 4),
        "latency_sample": f"{lat.size} iterations: {max(1, args.repeats)} fresh-table runs of {steps} "
                          "(the first run after warm-up iterations)",
        "iteration_hbm_frac": round(iter_gbs / HBM_PEAK_GBS, 4),
        "cells_touched_per_iteration": int(touched),
        "occupancy": round(st1["occupied"] / (1 << wl["table"]["log2_slots"]), 4),
        "dropped": st1["dropped"],
        "kernels": kernels,
        "instrumented_ms_per_step": inst_ms,
        "probe_hist": probes,
        "roofline": roofline,
        "device": device_info(torch),
    }
    if not args.no_graph and not args.split:
        result["graph_replay"] = graph_replay(torch, psf, wl, bufs, out, found, args.steps, n, params)
    del bufs, out, found
    torch.cuda.empty_cache()
    forms = {}
    for name in [f for f in args.forms.split(",") if f]:
        fn = {"precision": form_precision, "batched": form_batched, "serving": form_serving,
              "estimate": form_estimate, "progressive": form_progressive, "weighted": form_weighted}[name]
        print(f"# measuring form {name}", file=sys.stderr, flush=True)
        forms[name] = fn(torch, psf, W)
        torch.cuda.empty_cache()
    if forms:
        result["forms"] = forms
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(wl, host[0], args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
