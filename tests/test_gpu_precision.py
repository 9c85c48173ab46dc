"""Precision form: FP16 / BF16 approximant storage with an FP32 blend,
checked against the binary64 oracle."""
import numpy as np
import pytest

from tests.helpers import compare_cells, records, rel_err, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_07547_amd import psf
    psf.load()
    return torch, psf


def _one_cell_state(psf, dtype, values):
    t = psf.Table(log2_slots=8, state_dtype=dtype)
    v = np.asarray(values, dtype=np.float32)
    rec = records(len(v), px=0.5, py=0.5, pz=0.5, r=v, g=v, b=v)
    t.iterate(to_device(rec))
    ex = t.export()
    return ex["L"][:, 0], t.stats()


def test_f16_round_to_nearest_even_and_saturation(env):
    torch, psf = env
    # 1 + 2^-11 lies halfway between 1 and 1 + 2^-10: ties to even -> 1
    L, _ = _one_cell_state(psf, psf.PSF_STATE_F16, [1.0 + 2.0 ** -11])
    assert L[0] == 1.0
    # 1 + 3 * 2^-11 lies halfway between 1 + 2^-10 and 1 + 2^-9: ties to even -> 1 + 2^-9
    L, _ = _one_cell_state(psf, psf.PSF_STATE_F16, [1.0 + 3 * 2.0 ** -11])
    assert L[0] == 1.0 + 2.0 ** -9
    # just above the tie rounds up
    L, _ = _one_cell_state(psf, psf.PSF_STATE_F16, [1.0 + 2.0 ** -11 + 2.0 ** -20])
    assert L[0] == 1.0 + 2.0 ** -10
    L, st = _one_cell_state(psf, psf.PSF_STATE_F16, [1.0e6])
    assert L[0] == 65504.0 and st["saturated"] == 1
    L, st = _one_cell_state(psf, psf.PSF_STATE_F16, [-7.0e4, -7.0e4])
    assert L[0] == -65504.0 and st["saturated"] == 1
    L, st = _one_cell_state(psf, psf.PSF_STATE_F16, [65504.0])
    assert L[0] == 65504.0 and st["saturated"] == 0


def test_bf16_round_to_nearest_even(env):
    torch, psf = env
    # bf16 keeps 8 significant bits: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    L, _ = _one_cell_state(psf, psf.PSF_STATE_BF16, [1.0 + 2.0 ** -8])
    assert L[0] == 1.0
    L, _ = _one_cell_state(psf, psf.PSF_STATE_BF16, [1.0 + 3 * 2.0 ** -8])
    assert L[0] == 1.0 + 2.0 ** -6
    L, st = _one_cell_state(psf, psf.PSF_STATE_BF16, [3.0e38])
    assert np.isfinite(L[0]) and st["saturated"] == 0


@pytest.mark.parametrize("dtype_name", ["F16", "BF16"])
def test_tiny_workload_reduced_precision_keys_and_counts_exact(env, dtype_name):
    import oracle
    from synth import workloads as W
    torch, psf = env
    wl = W.tiny(alpha_mode=W.ALPHA_PAPER)
    sc = W.make_scene(wl)
    orc = oracle.Oracle(**wl["table"])
    t = psf.Table(**dict(wl["table"], state_dtype=getattr(psf, f"PSF_STATE_{dtype_name}")))
    for it in range(wl["iterations"]):
        rec = dict(sc.generate(wl["gen"], it))
        rec["rough"] = None
        t.iterate(to_device(rec))
        orc.insert(rec)
        orc.update()
    tol = {"F16": 2.5e-3, "BF16": 2.0e-2}[dtype_name]
    worst = compare_cells(t.export(), orc.export(), tol, dtype_name)
    print(f"tiny {dtype_name}: worst relative error {worst:.3e}")


# Error model of the stored approximant (Sec. 2.4 blend, FP32 arithmetic,
# round-to-nearest-even store of a 16-bit format with unit roundoff u):
# E_k = (1 - a_k) E_{k-1} + d_k with |d_k| <= u |L_k|, so with a_k >= 1/T_max
# the steady-state error is at most u * T_max * max|L| over the window.
U_F16, U_BF16, T_MAX = 2.0 ** -11, 2.0 ** -8, 5.0


def test_precision_workload_sampled_cells(env):
    """1920x1080, 5 vertices/path (10,368,000 records/iteration), 2^24
    slots, lognormal(0, 2) radiance: FP32, FP16 and BF16 tables fed the same
    frames; a sample of cells tracked by the binary64 oracle."""
    import oracle
    from synth import workloads as W
    torch, psf = env
    wl = W.precision()
    iters = 16
    sc = W.make_scene(wl)
    n = W.records_per_iteration(wl)
    tabs = {name: psf.Table(**dict(wl["table"], state_dtype=getattr(psf, f"PSF_STATE_{name}"),
                                   max_batch=n))
            for name in ("F32", "F16", "BF16")}
    orc = oracle.Oracle(**wl["table"])
    first = sc.generate(wl["gen"], 0)
    k0, _ = orc.keys(first)
    rng = np.random.default_rng(3)
    sample = np.unique(rng.choice(k0[k0 != np.uint64(2 ** 64 - 1)], size=4000))
    orc.set_filter(sample)
    for it in range(iters):
        rec = first if it == 0 else sc.generate(wl["gen"], it)
        d = to_device(rec)
        for t in tabs.values():
            t.iterate(d)
        orc.insert(rec)
        orc.update()
        del d
    torch.cuda.synchronize()
    o = orc.export()
    report = {}
    for name, t in tabs.items():
        g = t.export()
        idx = np.searchsorted(g["keys"], o["keys"])
        assert np.all(g["keys"][idx] == o["keys"])
        sub = {k: (v[:, idx] if v.ndim == 2 else v[idx]) for k, v in g.items()}
        assert np.array_equal(sub["c_old"].astype(np.uint64), o["c_old"])
        ref = o["L"]
        ok = (np.abs(ref) <= 65504.0) & (np.abs(ref) >= 2.0 ** -14) if name == "F16" else np.ones_like(ref, bool)
        e = rel_err(sub["L"], ref)[ok]
        report[name] = (float(e.max()), float(np.percentile(e, 99)), int((~ok).sum()))
        assert t.stats()["dropped"] == 0
    print("precision workload relative error (max, p99, excluded):", report)
    assert report["F32"][0] <= 1e-5
    assert report["F16"][1] <= 2e-3
    assert report["F16"][0] <= U_F16 * T_MAX * 2
    assert report["BF16"][1] <= U_BF16 * T_MAX
    assert report["BF16"][0] <= U_BF16 * T_MAX * 2
