"""Shared test helpers: fixture parsing and record construction (no method arithmetic)."""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FIELDS = ("px", "py", "pz", "nx", "ny", "nz", "ox", "oy", "oz", "r", "g", "b", "rough", "footprint",
          "weight")


def golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([c.strip() for c in line.split("|")])
    return rows


def records(n, **cols):
    """Record dict of n entries; unspecified fields default to a +z normal,
    +z direction, unit radiance and no roughness or footprint array."""
    base = {"px": 0.0, "py": 0.0, "pz": 0.0, "nx": 0.0, "ny": 0.0, "nz": 1.0,
            "ox": 0.0, "oy": 0.0, "oz": 1.0, "r": 1.0, "g": 1.0, "b": 1.0}
    out = {}
    for k in FIELDS:
        v = cols.get(k, base.get(k))
        if v is None:
            out[k] = None
            continue
        a = np.asarray(v, dtype=np.float32)
        out[k] = np.broadcast_to(a, (n,)).copy() if a.ndim == 0 else a.astype(np.float32)
    return out


def concat(recs):
    out = {}
    for k in FIELDS:
        parts = [r.get(k) for r in recs]
        out[k] = None if any(p is None for p in parts) else np.concatenate(parts)
    return out


def take(rec, idx):
    return {k: (None if v is None else np.ascontiguousarray(v[idx])) for k, v in rec.items()}


# ----------------------------------------------------------------- GPU side
def to_device(rec):
    import torch
    return {k: (None if v is None else torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).cuda())
            for k, v in rec.items()}


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


# Relative error bounds of the stored approximant against the binary64
# oracle, per state format (psf_config.state_dtype), in the format's normal
# range.  Blend arithmetic is binary32 (FP32 state: 1e-5, the target's
# tolerance).  A 16-bit format re-rounded by every blend carries, per Sec.
# 2.4's recursion E_k = (1 - a_k) E_(k-1) + d_k with |d_k| <= u |L_k| and
# a_k >= 1/T_max, at most u T_max (T_max = 5 in every workload here); with
# the residual carried (error feedback) a lookup sees one rounding: u.
U_F16, U_BF16, T_MAX_WORKLOADS = 2.0 ** -11, 2.0 ** -8, 5.0
STATE_BOUND = {0: 1e-5, 1: U_F16 * T_MAX_WORKLOADS, 2: U_BF16 * T_MAX_WORKLOADS,
               3: U_F16 + 1e-5, 4: U_BF16 + 1e-5}


def rel_err(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    den = np.maximum(np.abs(want), 1e-30)
    return np.abs(got - want) / den


def compare_cells(gpu_ex, orc_ex, rtol, label=""):
    """Keys and counts bit-exact, approximant within rtol (relative)."""
    assert np.array_equal(gpu_ex["keys"], orc_ex["keys"]), f"{label}: key sets differ"
    assert np.array_equal(gpu_ex["c_old"].astype(np.uint64), orc_ex["c_old"]), f"{label}: c_old differs"
    assert np.array_equal(gpu_ex["n_new"].astype(np.uint64), orc_ex["n_new"]), f"{label}: n_new differs"
    e = rel_err(gpu_ex["L"], orc_ex["L"])
    worst = float(e.max()) if e.size else 0.0
    assert worst <= rtol, f"{label}: worst relative error {worst:.3e} > {rtol:.1e}"
    return worst
