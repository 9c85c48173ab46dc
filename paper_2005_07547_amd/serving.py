"""Continuous-batching server for render sessions.

Each session is a stream of frames (iterations) of one renderer: its hash
table stays resident in HBM for the session's lifetime.  Requests arrive
over time; at every tick the server

1. admits waiting sessions while the resident bytes (tables plus input
   buffers) stay within the HBM budget and the active count within its cap;
2. runs one iteration (insert, temporal update, query) of every active
   session in a single batched call (``psf_iterate_batch``), so sessions that
   joined at different times share the device;
3. retires sessions that have run all their iterations.  Reading a retired
   table's statistics and destroying it synchronise the stream, which would
   leave the device idle while the host forms the next tick, so retired
   sessions are flushed (statistics read, table closed, memory returned to
   the budget) only when no tick is in flight, when a waiting session needs
   their memory, or at the end of the run.  Until then their tables still
   count against the budget.

The host keeps two ticks in flight (the next tick is launched before the
previous one is waited for), so host bookkeeping overlaps device work.  Per
session-iteration latency is measured from the moment the iteration became
runnable (its tick was formed) to the completion of its tick on the device.

Inputs: frames come from per-resolution-class pools resident in HBM (the
caller provides them; generation stays off the critical path).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

from . import psf


@dataclass
class SessionRequest:
    sid: int
    arrival: float          # seconds from the start of the run
    iterations: int
    table_cfg: dict
    frames: list            # device record dicts, cycled per iteration
    records: int = 0        # records per iteration
    # filled in by the server
    admitted_at: float = math.nan
    finished_at: float = math.nan
    done: int = 0
    inflight: int = 0
    footprint: int = 0
    table: object = None
    out: object = None
    found: object = None
    latencies_ms: list = field(default_factory=list)


def session_table_cfg(cfg: dict, records: int, lean: bool = True) -> dict:
    """The table configuration a session is served with: staging sized to
    its records, and, where the configuration allows it, no frame
    accumulators (a served session only ever takes fused iterations)."""
    import ctypes
    lib = psf.load()
    out = dict(cfg, max_batch=max(1, records))
    if lean:
        trial = dict(out, flags=int(out.get("flags", 0)) | psf.PSF_FLAG_NO_ACCUMULATORS)
        if lib.psf_table_bytes(ctypes.byref(psf.make_config(**trial))):
            out = trial
    return out


def table_footprint(cfg: dict, records: int, lean: bool = True) -> int:
    """Device bytes a session holds while resident: its table plus its output
    buffers (inputs are shared pools)."""
    import ctypes
    lib = psf.load()
    c = psf.make_config(**session_table_cfg(cfg, records, lean))
    return int(lib.psf_table_bytes(ctypes.byref(c))) + records * 13


class Server:
    def __init__(self, budget_bytes: int, max_active: int = 64, keep_tables: bool = False, lean: bool = True):
        import torch
        self.lean = bool(lean)
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.batch = psf.Batch(max_active)
        self.keep_tables = keep_tables
        self.resident = 0
        self.peak_resident = 0
        self.peak_active = 0
        self.ticks = 0
        self.records = 0
        self.dropped = 0
        self.flushes = 0
        self._retired = []  # finished sessions whose tables are not yet released
        self._torch = torch

    def _admit(self, s: SessionRequest, now: float):
        torch = self._torch
        s.table = psf.Table(**session_table_cfg(s.table_cfg, s.records, self.lean))
        s.out = torch.empty((3, s.records), dtype=torch.float32, device="cuda")
        s.found = torch.empty(s.records, dtype=torch.uint8, device="cuda")
        s.admitted_at = now
        self.resident += s.footprint

    def _retire(self, s: SessionRequest, now: float):
        s.finished_at = now
        if not self.keep_tables:
            s.out = s.found = None
        self._retired.append(s)

    def _flush(self):
        """Release the retired sessions' tables (synchronises the stream)."""
        if not self._retired:
            return
        for s in self._retired:
            self.dropped += s.table.stats()["dropped"]
            self.resident -= s.footprint
            if not self.keep_tables:
                s.table.close()
                s.table = None
        self._retired = []
        self.flushes += 1

    def run(self, requests: list, time_limit: float = 600.0, on_tick=None):
        """Serve every request; returns a summary dict.  requests are sorted
        by arrival time (seconds from the start)."""
        torch = self._torch
        pending = sorted(requests, key=lambda r: r.arrival)
        for r in pending:
            r.footprint = table_footprint(r.table_cfg, r.records, self.lean)
            if r.footprint > self.budget:
                raise ValueError(f"session {r.sid} needs {r.footprint} bytes, above the budget")
        waiting: list = []
        active: list = []
        inflight = []  # (event, start time, sessions of the tick)
        t0 = time.perf_counter()
        finished = []
        while pending or waiting or active or inflight:
            now = time.perf_counter() - t0
            if now > time_limit:
                raise TimeoutError("serving run exceeded its time limit")
            while pending and pending[0].arrival <= now:
                waiting.append(pending.pop(0))
            # retired tables are released when the device is idle anyway, or
            # when the next waiting session needs their memory
            if self._retired and (not inflight or (
                    waiting and self.resident + waiting[0].footprint > self.budget)):
                self._flush()
            # admission in arrival order while memory and slots allow
            while waiting and len(active) < self.max_active and \
                    self.resident + waiting[0].footprint <= self.budget:
                s = waiting.pop(0)
                self._admit(s, now)
                active.append(s)
            self.peak_resident = max(self.peak_resident, self.resident)
            self.peak_active = max(self.peak_active, len(active))
            # every active session with iterations left joins the tick; the
            # stream orders a session's consecutive iterations
            runnable = [s for s in active if s.done + s.inflight < s.iterations]
            if runnable:
                tables = [s.table for s in runnable]
                frames = [s.frames[(s.done + s.inflight) % len(s.frames)] for s in runnable]
                for s in runnable:
                    s.inflight += 1
                self.batch.iterate(tables, frames, outs=[s.out for s in runnable],
                                   founds=[s.found for s in runnable])
                ev = torch.cuda.Event()
                ev.record()
                inflight.append((ev, time.perf_counter(), runnable))
                self.ticks += 1
            # complete the oldest tick when two are in flight, or when idle
            if inflight and (len(inflight) >= 2 or not runnable):
                ev, started, group = inflight.pop(0)
                ev.synchronize()
                end = time.perf_counter()
                for s in group:
                    s.latencies_ms.append((end - started) * 1e3)
                    s.inflight -= 1
                    s.done += 1
                    self.records += s.records
                    if s.done >= s.iterations:
                        active.remove(s)
                        self._retire(s, end - t0)
                        finished.append(s)
                if on_tick:
                    on_tick(self)
            elif not runnable and not inflight and not waiting and pending:
                time.sleep(min(0.001, max(0.0, pending[0].arrival - now)))
        self._flush()
        wall = time.perf_counter() - t0
        lat = sorted(x for s in finished for x in s.latencies_ms)

        def pct(q):
            if not lat:
                return math.nan
            return lat[min(len(lat) - 1, int(round(q / 100.0 * (len(lat) - 1))))]

        return {
            "sessions": len(finished), "ticks": self.ticks, "records": self.records,
            "wall_s": wall, "records_per_s": self.records / wall if wall > 0 else math.nan,
            "p50_iter_ms": pct(50), "p99_iter_ms": pct(99),
            "peak_active": self.peak_active, "peak_resident_bytes": self.peak_resident,
            "dropped": self.dropped, "flushes": self.flushes,
            "mean_queue_s": sum(s.admitted_at - s.arrival for s in finished) / max(1, len(finished)),
        }


# ---------------------------------------------------------------- workload
RES_CLASSES = ((128, 128), (320, 180), (640, 360), (960, 540), (1280, 720), (1920, 1080),
               (2560, 1440), (3840, 2160))


def draw_requests(n_sessions: int, rate: float = 20.0, seed: int = 5, iter_range=(32, 128)):
    """Poisson arrivals at `rate` per second; pixel counts lognormal around
    720p (921,600 * exp(0.5 Z)) clipped to [128^2, 3840x2160], mapped to the
    nearest resolution class; iterations uniform in iter_range.  Returns a
    list of (sid, arrival, class index, iterations, scene seed)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_sessions):
        t += rng.exponential(1.0 / rate)
        pix = 921600.0 * math.exp(0.5 * rng.standard_normal())
        pix = min(max(pix, 128 * 128), 3840 * 2160)
        cls = int(np.argmin([abs(math.log(w * h / pix)) for w, h in RES_CLASSES]))
        iters = int(rng.integers(iter_range[0], iter_range[1] + 1))
        out.append((i, t, cls, iters, 500 + i))
    return out
