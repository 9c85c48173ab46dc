"""MIS-weighted counters on the GPU (Eq. 5-6 with weights w != 1, Sec. 2.5's
down-weighted fields; Eq. 10-11 on the weighted counters) against the
oracle: every insert strategy, the fused iteration, split inserts, the
batched form, and the tables' argument checks.

Counters are binary32 weight sums on the GPU (binary64 in the oracle), so
they are compared to a relative tolerance instead of bit for bit; keys and
found flags stay bit-exact.  The partitioned insert rounds each frame's
binary64 weight sum once, which is checked exactly, with run-to-run
reproducibility."""
import numpy as np
import pytest

from tests.helpers import rel_err, to_device

pytestmark = pytest.mark.gpu
RTOL_F32 = 1e-5


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_07547_amd import psf
    psf.load()
    return torch, psf


def _weights(n, it, bad=True):
    from synth import workloads as W
    w = W.mis_weights(n, seed=100 + it, excluded=0.1)
    if bad:
        idx = np.arange(3 + it, n, 397)
        w[idx[0::3]] = np.nan
        w[idx[1::3]] = -1.0
        w[idx[2::3]] = np.inf
    return w


def _tiny(it, alpha_mode=0):
    from synth import workloads as W
    wl = W.tiny(alpha_mode=alpha_mode)
    rec = dict(W.make_scene(wl).generate(wl["gen"], it))
    rec["rough"] = None
    return wl, rec


def _compare(t, orc, label):
    g, o = t.export(), orc.export()
    assert np.array_equal(g["keys"], o["keys"]), f"{label}: key sets differ"
    assert g["c_old"].dtype == np.float32
    assert rel_err(g["c_old"], o["c_old"]).max() <= RTOL_F32, label
    assert np.array_equal(g["n_new"] == 0, o["n_new"] == 0), label
    assert rel_err(g["L"], o["L"]).max() <= RTOL_F32, label


MODES = [("direct", 1, False), ("partitioned", 2, False), ("fused", 2, True), ("fused-auto", 0, True)]


@pytest.mark.parametrize("alpha_mode", [0, 2])
@pytest.mark.parametrize("name,insert_mode,fused", MODES)
def test_weighted_whole_iterations(env, name, insert_mode, fused, alpha_mode):
    import oracle
    torch, psf = env
    wl, _ = _tiny(0, alpha_mode)
    cfg = dict(wl["table"], weighted=1)
    orc = oracle.Oracle(**cfg)
    t = psf.Table(**cfg, insert_mode=insert_mode)
    skipped = 0
    for it in range(6):
        _, rec = _tiny(it, alpha_mode)
        rec["weight"] = _weights(len(rec["px"]), it)
        skipped += int((~(np.isfinite(rec["weight"]) & (rec["weight"] > 0))).sum())
        d = to_device(rec)
        orc.insert(rec)
        orc.update()
        if fused:
            out, found = t.iterate(d)
        else:
            t.insert(d)
            t.update()
            out, found = t.query(d)
        torch.cuda.synchronize()
        w_out, w_found = orc.query(rec)
        assert np.array_equal(found.cpu().numpy(), w_found), (name, it)
        assert rel_err(out.cpu().numpy(), w_out).max() <= RTOL_F32, (name, it)
    _compare(t, orc, name)
    st = t.stats()
    assert st["skipped"] == skipped == orc.counters()["skipped"]
    assert st["dropped"] == 0 and st["updates"] == 6


@pytest.mark.parametrize("fused", [False, True])
def test_weighted_plain_workload_first_iterations(env, fused):
    """Full-size frames (1280x720, 4 vertices, 3,686,400 records) with the
    tuned binning width: many tiles, every partition."""
    import oracle
    from synth import workloads as W
    torch, psf = env
    wl = W.plain()
    sc = W.make_scene(wl)
    cfg = dict(wl["table"], weighted=1)
    orc = oracle.Oracle(**cfg)
    t = psf.Table(**cfg, insert_mode=2, bin_per=12, part_log2=11)
    for it in range(2):
        rec = dict(sc.generate(wl["gen"], it))
        rec["weight"] = _weights(len(rec["px"]), it, bad=False)
        d = to_device(rec)
        orc.insert(rec)
        orc.update()
        if fused:
            out, found = t.iterate(d)
        else:
            t.insert(d)
            t.update()
            out, found = t.query(d)
        torch.cuda.synchronize()
        w_out, w_found = orc.query(rec)
        assert np.array_equal(found.cpu().numpy(), w_found), it
        assert rel_err(out.cpu().numpy(), w_out).max() <= RTOL_F32, it
        del d, out, found
    _compare(t, orc, "plain")


def test_partitioned_weight_sums_round_once_and_reproduce(env):
    """The partitioned insert sums a frame's weights in binary64 and rounds
    once: a first frame's counters are the oracle's binary64 sums rounded
    to binary32, and two runs of the full-size workload agree bit for bit
    (counters and approximant), whatever the order of the LDS atomics."""
    import oracle
    from synth import workloads as W
    torch, psf = env
    wl, rec = _tiny(0)
    rec["weight"] = _weights(len(rec["px"]), 0, bad=False)
    cfg = dict(wl["table"], weighted=1)
    orc = oracle.Oracle(**cfg)
    orc.insert(rec)
    t = psf.Table(**cfg, insert_mode=2)
    t.insert(to_device(rec))
    torch.cuda.synchronize()
    g, o = t.export(), orc.export()
    assert np.array_equal(g["keys"], o["keys"])
    assert np.array_equal(g["n_new"], o["n_new"].astype(np.float32))

    wl = W.plain()
    sc = W.make_scene(wl)
    cfg = dict(wl["table"], weighted=1)
    runs = [psf.Table(**cfg, insert_mode=2), psf.Table(**cfg, insert_mode=2)]
    for it in range(3):
        rec = dict(sc.generate(wl["gen"], it))
        rec["weight"] = _weights(len(rec["px"]), it, bad=False)
        d = to_device(rec)
        for t in runs:
            t.iterate(d)
        del d
    torch.cuda.synchronize()
    a, b = runs[0].export(), runs[1].export()
    assert np.array_equal(a["keys"], b["keys"])
    assert np.array_equal(a["c_old"].view(np.uint32), b["c_old"].view(np.uint32))
    assert np.array_equal(a["L"].view(np.uint32), b["L"].view(np.uint32))


@pytest.mark.parametrize("insert_mode", [1, 2])
def test_weighted_table_without_weights_equals_plain_table(env, insert_mode):
    torch, psf = env
    wl, _ = _tiny(0)
    a = psf.Table(**wl["table"], weighted=1, insert_mode=insert_mode)
    b = psf.Table(**wl["table"], insert_mode=insert_mode)
    for it in range(4):
        _, rec = _tiny(it)
        d = to_device(rec)
        a.iterate(d)
        b.iterate(d)
    torch.cuda.synchronize()
    ea, eb = a.export(), b.export()
    assert np.array_equal(ea["keys"], eb["keys"])
    assert np.array_equal(ea["c_old"], eb["c_old"].astype(np.float32))
    if insert_mode == 2:
        # binary64 sums: the order of the atomics is immaterial
        assert np.array_equal(ea["L"], eb["L"])
    else:
        # binary32 global atomics: their order differs from run to run
        assert rel_err(ea["L"], eb["L"]).max() <= RTOL_F32


def test_weighted_insert_split_over_capacity(env):
    """An insert larger than the binning capacity runs in chunks; every
    per-record array, weights and footprints included, advances with them."""
    import oracle
    from synth import workloads as W
    torch, psf = env
    wl, rec = _tiny(0)
    n = len(rec["px"])
    rec["weight"] = _weights(n, 0)
    rec["footprint"] = W.footprints(rec, wl, spread=1.5)
    cfg = dict(wl["table"], weighted=1)
    t = psf.Table(**cfg, insert_mode=2, max_batch=4096)
    assert n > 4096
    orc = oracle.Oracle(**cfg)
    for it in range(2):
        t.insert(to_device(rec))
        t.update()
        orc.insert(rec)
        orc.update()
    torch.cuda.synchronize()
    _compare(t, orc, "split")


def test_weighted_sessions_in_a_batch(env):
    """A weighted session with weights, one without, and an unweighted one
    share one batched launch; each matches its oracle."""
    import oracle
    torch, psf = env
    wl, _ = _tiny(0)
    cfgs = [dict(wl["table"], weighted=1), dict(wl["table"], weighted=1), dict(wl["table"])]
    tables = [psf.Table(**c, insert_mode=2) for c in cfgs]
    orcs = [oracle.Oracle(**c) for c in cfgs]
    batch = psf.Batch(4)
    for it in range(3):
        recs = []
        for j in range(3):
            _, rec = _tiny(it + 10 * j)
            if j == 0:
                rec["weight"] = _weights(len(rec["px"]), it)
            recs.append(rec)
        res = batch.iterate(tables, [to_device(r) for r in recs])
        torch.cuda.synchronize()
        for o, r, (out, found) in zip(orcs, recs, res):
            o.insert(r)
            o.update()
            w_out, w_found = o.query(r)
            assert np.array_equal(found.cpu().numpy(), w_found), it
            assert rel_err(out.cpu().numpy(), w_out).max() <= RTOL_F32, it
    for j in range(2):
        _compare(tables[j], orcs[j], f"session {j}")
    e, o = tables[2].export(), orcs[2].export()
    assert np.array_equal(e["keys"], o["keys"])
    assert np.array_equal(e["c_old"].astype(np.uint64), o["c_old"])


def test_weights_need_a_weighted_table(env):
    torch, psf = env
    wl, rec = _tiny(0)
    rec["weight"] = np.ones(len(rec["px"]), np.float32)
    t = psf.Table(**wl["table"])
    with pytest.raises(psf.PsfError):
        t.insert(to_device(rec))
    with pytest.raises(psf.PsfError):
        t.iterate(to_device(rec))
    with pytest.raises(psf.PsfError):
        psf.Table(**wl["table"], weighted=2)


@pytest.mark.parametrize("dtype_name,tol", [("F16", 2.5e-3), ("BF16", 2.0e-2)])
def test_weighted_reduced_precision_state(env, dtype_name, tol):
    """Weighted counters with a 16-bit approximant: keys exact, counters as
    for FP32 state, the approximant within the storage format's error."""
    import oracle
    torch, psf = env
    wl, _ = _tiny(0)
    cfg = dict(wl["table"], weighted=1)
    orc = oracle.Oracle(**cfg)
    t = psf.Table(**cfg, insert_mode=2, state_dtype=getattr(psf, f"PSF_STATE_{dtype_name}"))
    for it in range(wl["iterations"]):
        _, rec = _tiny(it)
        rec["weight"] = _weights(len(rec["px"]), it)
        t.iterate(to_device(rec))
        orc.insert(rec)
        orc.update()
    torch.cuda.synchronize()
    g, o = t.export(), orc.export()
    assert np.array_equal(g["keys"], o["keys"])
    assert rel_err(g["c_old"], o["c_old"]).max() <= RTOL_F32
    assert rel_err(g["L"], o["L"]).max() <= tol


@pytest.mark.parametrize("insert_mode", [1, 2])
def test_weighted_progressive_step(env, insert_mode):
    """The progressive solver step on a weighted table: each vertex's
    sample carries its MIS weight into the counters (closed furnace)."""
    import oracle
    from synth import workloads as W
    torch, psf = env
    cfg = dict(W.furnace_table(), weighted=1)
    t = psf.Table(**dict(cfg, insert_mode=insert_mode))
    o = oracle.Oracle(**cfg)

    def dev3(arrs):
        return tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs)

    for it in range(12):
        x, nx, tp, em = W.furnace_paths(2048, 2, it)
        x = dict(x, weight=_weights(len(x["px"]), it, bad=False))
        want = oracle.progressive_step(o, x, nx, tp, em)
        got = t.progressive_step(to_device(x), to_device(nx), dev3(tp), dev3(em))
        torch.cuda.synchronize()
        assert rel_err(got.cpu().numpy(), want).max() <= RTOL_F32, it
    _compare(t, o, "progressive")
