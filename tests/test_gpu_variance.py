"""GPU parity of the per-cell luminance variance (PSF_FLAG_TRACK_VARIANCE)
against the binary64 oracle.

The variance is formed from sums of Y and Y^2, so its rounding error scales
with the second moment V + Y^2 (Y the luminance of the approximant), not
with V: the bar is the FP32 state's 1e-5 relative, applied to V + Y^2 (for
the 16-bit state formats, whose blend continues from the stored value,
that format's state bound).  Keys bit-exact with the oracle.  Covers the
direct insert, the partitioned insert with a separate update, the fused
iteration, the batched iteration, 16-bit states, the full-size plain
workload on sampled cells, and the argument checks.
"""
import numpy as np
import pytest

from tests.helpers import STATE_BOUND, compare_cells, to_device

pytestmark = pytest.mark.gpu
RTOL = 1e-5


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_07547_amd import psf
    psf.load()
    return torch, psf


def _luma(L):
    L = np.asarray(L, dtype=np.float64)
    return (L[0] + 2.0 * L[1] + L[2]) / 4.0


def _compare_variance(t, orc, rtol, label):
    kg, vg = t.export_variance()
    ko, vo = orc.export_variance()
    assert np.array_equal(kg, ko), f"{label}: key sets differ"
    L = orc.export()["L"]
    second = vo + _luma(L) ** 2
    err = np.abs(vg.astype(np.float64) - vo) / np.maximum(second, 1e-30)
    worst = float(err.max()) if err.size else 0.0
    assert worst <= rtol, f"{label}: worst variance error {worst:.3e} of V + Y^2 > {rtol:.1e}"
    assert np.all(vg >= 0.0)
    return worst


def _tiny_frames(iterations, alpha_mode):
    from synth import workloads as W
    wl = W.tiny(alpha_mode=alpha_mode)
    sc = W.make_scene(wl)
    out = []
    for it in range(iterations):
        rec = dict(sc.generate(wl["gen"], it))
        rec["rough"] = None
        out.append(rec)
    return wl, out


@pytest.mark.parametrize("how", ["direct", "partitioned", "fused"])
@pytest.mark.parametrize("alpha_mode", [0, 1, 2])
def test_tiny_variance_every_strategy(env, how, alpha_mode):
    import oracle
    torch, psf = env
    wl, frames = _tiny_frames(6, alpha_mode)
    mode = psf.PSF_INSERT_DIRECT if how == "direct" else psf.PSF_INSERT_PARTITIONED
    t = psf.Table(**dict(wl["table"], insert_mode=mode, flags=psf.PSF_FLAG_TRACK_VARIANCE))
    orc = oracle.Oracle(**wl["table"])
    for rec in frames:
        d = to_device(rec)
        if how == "fused":
            t.iterate(d)
        else:
            t.insert(d)
            t.update()
        orc.insert(rec)
        orc.update()
    torch.cuda.synchronize()
    compare_cells(t.export(), orc.export(), RTOL, f"{how} mode {alpha_mode}")
    worst = _compare_variance(t, orc, RTOL, f"{how} mode {alpha_mode}")
    print(f"{how} alpha mode {alpha_mode}: worst variance error {worst:.2e} of V + Y^2")


@pytest.mark.parametrize("name", ["F16", "BF16", "F16_EF", "BF16_EF"])
def test_tiny_variance_reduced_precision_state(env, name):
    import oracle
    torch, psf = env
    wl, frames = _tiny_frames(6, 0)
    code = getattr(psf, f"PSF_STATE_{name}")
    t = psf.Table(**dict(wl["table"], state_dtype=code, flags=psf.PSF_FLAG_TRACK_VARIANCE))
    orc = oracle.Oracle(**wl["table"])
    for rec in frames:
        t.iterate(to_device(rec))
        orc.insert(rec)
        orc.update()
    torch.cuda.synchronize()
    _compare_variance(t, orc, STATE_BOUND[code], name)


def test_variance_table_keeps_the_same_cells_as_a_plain_one(env):
    """Tracking the variance changes neither the keys, the counts nor the
    approximant (the partitioned insert stages every record on its own in
    such a table, so its sums may round differently: within 1e-5)."""
    torch, psf = env
    wl, frames = _tiny_frames(4, 0)
    a = psf.Table(**wl["table"])
    b = psf.Table(**dict(wl["table"], flags=psf.PSF_FLAG_TRACK_VARIANCE))
    for rec in frames:
        d = to_device(rec)
        oa, fa = a.iterate(d)
        ob, fb = b.iterate(d)
        assert torch.equal(fa, fb)
        assert torch.allclose(oa, ob, rtol=1e-5, atol=0.0)
    ea, eb = a.export(), b.export()
    assert np.array_equal(ea["keys"], eb["keys"]) and np.array_equal(ea["c_old"], eb["c_old"])


def test_batched_sessions_variance(env):
    import oracle
    from synth import workloads as W
    torch, psf = env
    ss = []
    for wl in W.batched_sessions(4):
        g = dict(wl["gen"], width=max(16, wl["gen"]["width"] // 8), height=max(16, wl["gen"]["height"] // 8))
        wl = dict(wl, gen=g, table=dict(wl["table"], log2_slots=max(14, wl["table"]["log2_slots"] - 4)))
        ss.append((wl, W.make_scene(wl)))
    # sessions 0 and 2 keep the variance, 1 and 3 do not
    fl = [psf.PSF_FLAG_TRACK_VARIANCE if i % 2 == 0 else 0 for i in range(len(ss))]
    tables = [psf.Table(**wl["table"], flags=f) for (wl, _), f in zip(ss, fl)]
    orcs = [oracle.Oracle(**wl["table"]) for wl, _ in ss]
    batch = psf.Batch(8)
    for it in range(3):
        recs = [sc.generate(wl["gen"], it) for wl, sc in ss]
        batch.iterate(tables, [to_device(r) for r in recs])
        for o, r in zip(orcs, recs):
            o.insert(r)
            o.update()
    torch.cuda.synchronize()
    for i, (wl, _) in enumerate(ss):
        compare_cells(tables[i].export(), orcs[i].export(), RTOL, wl["name"])
        if fl[i]:
            _compare_variance(tables[i], orcs[i], RTOL, wl["name"])


@pytest.mark.timeout(300)
def test_plain_workload_variance_sampled(env):
    """1280x720, 4 vertices/path (3,686,400 records per iteration), 2^22
    slots, 4 fused iterations; 8000 sampled cells tracked by the oracle."""
    import os
    import oracle
    from synth import workloads as W
    torch, psf = env
    wl = W.plain()
    sc = W.make_scene(wl)
    t = psf.Table(**dict(wl["table"], flags=psf.PSF_FLAG_TRACK_VARIANCE))
    orc = oracle.ShardedOracle(min(16, os.cpu_count() or 1), **wl["table"])
    rng = np.random.default_rng(7)
    for it in range(4):
        rec = sc.generate(wl["gen"], it)
        if it == 0:
            k0, _ = orc.keys(rec)
            orc.set_filter(np.unique(rng.choice(k0[k0 != np.uint64(2 ** 64 - 1)], size=8000)))
        t.iterate(to_device(rec))
        orc.insert(rec)
        orc.update()
    torch.cuda.synchronize()
    kg, vg = t.export_variance()
    ko, vo = orc.export_variance()
    idx = np.searchsorted(kg, ko)
    assert np.all(kg[idx] == ko)
    g = t.export()
    assert np.array_equal(g["c_old"][idx].astype(np.uint64), orc.export()["c_old"])
    second = vo + _luma(orc.export()["L"]) ** 2
    err = np.abs(vg[idx].astype(np.float64) - vo) / np.maximum(second, 1e-30)
    print(f"{len(ko)} sampled cells: worst variance error {err.max():.2e} of V + Y^2; "
          f"cells with V > 0: {(vo > 0).mean():.2f}")
    assert err.max() <= RTOL
    assert t.stats()["dropped"] == 0


@pytest.mark.parametrize("mode", [1, 2])
def test_variance_ignores_rejected_records(env, mode):
    """Records with a non-finite value or position are skipped: they add
    nothing to a cell's squared-luminance sum (the partitioned path stages
    them for lookup only)."""
    import oracle
    torch, psf = env
    wl, frames = _tiny_frames(3, 0)
    t = psf.Table(**dict(wl["table"], insert_mode=mode, flags=psf.PSF_FLAG_TRACK_VARIANCE))
    orc = oracle.Oracle(**wl["table"])
    for i, rec in enumerate(frames):
        rec = {k: (None if v is None else v.copy()) for k, v in rec.items()}
        n = len(rec["px"])
        rec["g"][i::97] = np.nan
        rec["r"][i + 5::131] = np.inf
        rec["px"][i + 11::173] = np.nan
        t.iterate(to_device(rec))
        orc.insert(rec)
        orc.update()
    torch.cuda.synchronize()
    assert t.stats()["skipped"] == orc.counters()["skipped"]
    compare_cells(t.export(), orc.export(), RTOL, f"mode {mode}")
    _compare_variance(t, orc, RTOL, f"mode {mode}")


@pytest.mark.parametrize("how", ["counters", "clear", "region"])
def test_variance_after_resets(env, how):
    """A counter reset (global or by region) restarts the variance at the
    next blend; clearing the table forgets it."""
    import oracle
    torch, psf = env
    wl, frames = _tiny_frames(6, 0)
    t = psf.Table(**dict(wl["table"], flags=psf.PSF_FLAG_TRACK_VARIANCE))
    orc = oracle.Oracle(**wl["table"])
    for i, rec in enumerate(frames):
        if i == 3:
            if how == "region":
                t.reset_region((0.0, 0.0, 0.0), (0.5, 1.0, 1.0))
                orc.reset_region((0.0, 0.0, 0.0), (0.5, 1.0, 1.0))
            else:
                what = psf.PSF_RESET_COUNTERS if how == "counters" else psf.PSF_RESET_CLEAR
                t.reset(what)
                orc.reset(what)
        t.iterate(to_device(rec))
        orc.insert(rec)
        orc.update()
    torch.cuda.synchronize()
    compare_cells(t.export(), orc.export(), RTOL, how)
    _compare_variance(t, orc, RTOL, how)


def test_variance_insert_split_over_staging_capacity(env):
    """A frame larger than the partitioned insert's staging (max_batch 4096,
    8192 records) is inserted in chunks whose squared-luminance sums meet in
    the pending accumulator before the blend."""
    import oracle
    torch, psf = env
    wl, frames = _tiny_frames(3, 0)
    t = psf.Table(**dict(wl["table"], insert_mode=psf.PSF_INSERT_PARTITIONED, max_batch=4096,
                         flags=psf.PSF_FLAG_TRACK_VARIANCE))
    orc = oracle.Oracle(**wl["table"])
    for rec in frames:
        assert len(rec["px"]) > 4096
        t.iterate(to_device(rec))
        orc.insert(rec)
        orc.update()
    torch.cuda.synchronize()
    compare_cells(t.export(), orc.export(), RTOL, "split")
    _compare_variance(t, orc, RTOL, "split")


@pytest.mark.parametrize("mode", [1, 2])
def test_variance_edge_inputs(env, mode):
    """An empty launch changes nothing; one record gives variance 0; two
    records of one cell give the population variance of their luminances;
    a 256-slot table (one partition)."""
    import oracle
    from tests.helpers import records
    torch, psf = env
    cfg = dict(log2_slots=8, alpha_mode=psf.PSF_ALPHA_CONST, alpha=0.5)
    t = psf.Table(**dict(cfg, insert_mode=mode, flags=psf.PSF_FLAG_TRACK_VARIANCE))
    orc = oracle.Oracle(**cfg)
    empty = records(0)
    t.iterate(to_device(empty))
    k, v = t.export_variance()
    assert k.size == 0
    one = records(1, px=0.5, py=0.5, pz=0.5, r=2.0, g=1.0, b=0.5)
    t.iterate(to_device(one))
    orc.insert(one)
    orc.update()
    k, v = t.export_variance()
    assert k.size == 1 and v[0] == 0.0
    two = records(2, px=0.5, py=0.5, pz=0.5, r=[0.0, 0.0], g=[0.0, 2.0], b=[0.0, 0.0])
    t.iterate(to_device(two))
    orc.insert(two)
    orc.update()
    torch.cuda.synchronize()
    _compare_variance(t, orc, RTOL, f"edge mode {mode}")


def test_variance_argument_checks(env):
    torch, psf = env
    with pytest.raises(psf.PsfError) as e:
        psf.Table(log2_slots=12, flags=psf.PSF_FLAG_TRACK_VARIANCE, weighted=1)
    assert e.value.status == psf.PSF_NOT_SUPPORTED
    with pytest.raises(psf.PsfError) as e:
        psf.Table(log2_slots=12, flags=psf.PSF_FLAG_TRACK_VARIANCE, payload=psf.PSF_PAYLOAD_SH2_YCOCG,
                  insert_mode=psf.PSF_INSERT_DIRECT)
    assert e.value.status == psf.PSF_NOT_SUPPORTED
    with pytest.raises(psf.PsfError) as e:
        psf.Table(log2_slots=14, flags=psf.PSF_FLAG_TRACK_VARIANCE, part_log2=12)
    assert e.value.status == psf.PSF_INVALID_ARGUMENT
    with pytest.raises(psf.PsfError) as e:
        psf.Table(log2_slots=14, weighted=1, part_log2=12)
    assert e.value.status == psf.PSF_INVALID_ARGUMENT
    t = psf.Table(log2_slots=12)
    with pytest.raises(psf.PsfError) as e:
        t.export_variance()
    assert e.value.status == psf.PSF_NOT_SUPPORTED
    # an empty table exports nothing; a cleared one likewise
    v = psf.Table(log2_slots=12, flags=psf.PSF_FLAG_TRACK_VARIANCE)
    k, var = v.export_variance()
    assert k.size == 0 and var.size == 0
