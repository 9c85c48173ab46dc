"""GPU parity of the two-field estimators (psf_estimate) against the oracle:
the worked examples exactly, the tiny and a reduced plain workload within
the binary32 tolerance, the applied flags bit for bit."""
import numpy as np
import pytest

from tests.helpers import golden_rows, records, to_device

pytestmark = pytest.mark.gpu
RTOL = 2e-5  # state within 1e-5 of binary64, plus a few binary32 roundings


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2005_07547_amd import psf
    psf.load()
    return torch, psf


def _dev(d):
    return to_device({k: v for k, v in d.items()})


def _check(psf, oracle, oe_t, fl_t, oe_o, fl_o, a, mode, param):
    import torch
    out, applied = psf.estimate(oe_t, fl_t, _dev(a), mode, param)
    torch.cuda.synchronize()
    want, w_app = oracle.estimate(oe_o, fl_o, a, mode, param)
    assert np.array_equal(applied.cpu().numpy(), w_app)
    # scale of the terms the estimate adds up, from the oracle's lookups
    base = {k: a.get(k) for k in ("px", "py", "pz", "nx", "ny", "nz", "rough", "footprint")}
    L, _ = oe_o.query(dict(base, ox=a["oox"], oy=a["ooy"], oz=a["ooz"]))
    h, _ = fl_o.query(dict(base, ox=a["oix"], oy=a["oiy"], oz=a["oiz"]))
    g = np.stack([a["gr"], a["gg"], a["gb"]]).astype(np.float64)
    w = a["wp"].astype(np.float64)
    p = abs(float(np.float32(param)))
    scale = np.abs(w * g) + w * p * np.abs(h) + p * np.abs(L) + np.abs(w * h) + np.abs(L)
    err = np.abs(out.cpu().numpy().astype(np.float64) - want)
    assert np.all(err <= RTOL * scale + 1e-30), float((err / np.maximum(scale, 1e-30)).max())
    return out, applied


def test_worked_examples_exactly(env):
    import oracle
    torch, psf = env
    cfg = dict(kappa=0.0, e_min=-2, max_level=0, log2_slots=12)
    for mode, param, L, h, g, wp, want in golden_rows("estimators.txt"):
        L, h, g, wp = float(L), float(h), float(g), float(wp)
        a = {k: np.array([v], dtype=np.float32) for k, v in dict(
            px=0.3, py=0.2, pz=0.1, nx=0.0, ny=0.0, nz=1.0, oox=0.0, ooy=0.6, ooz=0.8, oix=0.6, oiy=0.0,
            oiz=0.8, rough=1.0, gr=g, gg=g, gb=g, wp=wp).items()}
        oe = psf.Table(**cfg)
        fl = psf.Table(**dict(cfg, rough_thr=float("inf")))
        oe.iterate(to_device(records(1, px=0.3, py=0.2, pz=0.1, ox=0.0, oy=0.6, oz=0.8, rough=1.0,
                                     r=L, g=L, b=L)))
        fl.iterate(to_device(records(1, px=0.3, py=0.2, pz=0.1, ox=0.6, oy=0.0, oz=0.8, rough=1.0,
                                     r=h, g=h, b=h)))
        m = psf.PSF_EST_CV if mode == "cv" else psf.PSF_EST_BIASED
        out, applied = psf.estimate(oe, fl, _dev(a), m, float(param))
        torch.cuda.synchronize()
        assert applied.cpu().numpy()[0] == 1
        assert np.all(out.cpu().numpy()[:, 0] == np.float32(want)), (mode, param, out.cpu().numpy()[:, 0])


@pytest.mark.parametrize("mode,param", [(0, 0.75), (0, 1.0), (1, 0.0), (1, 0.5), (1, 1.0)])
def test_tiny_workload_estimators(env, mode, param):
    import oracle
    from synth import workloads as W
    torch, psf = env
    wl = W.tiny()
    sc = W.make_scene(wl)
    oe_t, fl_t = psf.Table(**wl["table"]), psf.Table(**W.fl_table(wl["table"]))
    oe_o, fl_o = oracle.Oracle(**wl["table"]), oracle.Oracle(**W.fl_table(wl["table"]))
    for it in range(3):
        rec = dict(sc.generate(wl["gen"], it))
        rec["rough"] = None
        a, fl = W.estimator_inputs(rec, wl["gen"])
        oe_t.iterate(to_device(rec))
        fl_t.iterate(to_device(fl))
        oe_o.insert(rec)
        oe_o.update()
        fl_o.insert(fl)
        fl_o.update()
    # the last frame's vertices, and the same vertices with shifted samples
    _, applied = _check(psf, oracle, oe_t, fl_t, oe_o, fl_o, a, mode, param)
    assert applied.sum() > 0.5 * applied.numel()
    a2 = dict(a, gr=a["gr"] * np.float32(0.5), oix=a["oiy"], oiy=a["oiz"], oiz=a["oix"])
    _check(psf, oracle, oe_t, fl_t, oe_o, fl_o, a2, mode, param)


def test_reduced_plain_workload_with_glossy_vertices(env):
    import oracle
    from synth import workloads as W
    torch, psf = env
    wl = W.plain()
    g = dict(wl["gen"], width=320, height=180)
    sc = W.make_scene(wl)
    cfg = dict(wl["table"], log2_slots=20)
    oe_t, fl_t = psf.Table(**cfg), psf.Table(**W.fl_table(cfg))
    oe_o, fl_o = oracle.Oracle(**cfg), oracle.Oracle(**W.fl_table(cfg))
    for it in range(2):
        rec = sc.generate(g, it)
        a, fl = W.estimator_inputs(rec, g)
        oe_t.iterate(to_device(rec))
        fl_t.iterate(to_device(fl))
        oe_o.insert(rec)
        oe_o.update()
        fl_o.insert(fl)
        fl_o.update()
    for mode, param in ((0, 0.5), (1, 0.25)):
        _check(psf, oracle, oe_t, fl_t, oe_o, fl_o, a, mode, param)


def test_invalid_estimate_arguments(env):
    torch, psf = env
    t = psf.Table(log2_slots=10)
    a = {k: torch.zeros(4, dtype=torch.float32, device="cuda") for k in psf.EST_FIELDS}
    for mode, param in ((2, 1.0), (0, float("inf")), (1, float("nan"))):
        with pytest.raises(psf.PsfError):
            psf.estimate(t, t, a, mode, param)
    with pytest.raises(psf.PsfError):
        psf.estimate(t, t, dict(a, wp=None), 0, 1.0)
    out, applied = psf.estimate(t, t, a, 0, 1.0)  # empty tables: plain estimate, nothing applied
    torch.cuda.synchronize()
    assert int(applied.sum()) == 0 and float(out.abs().sum()) == 0.0


def test_estimators_with_footprint_levels(env):
    import oracle
    from synth import workloads as W
    torch, psf = env
    wl = W.tiny()
    sc = W.make_scene(wl)
    oe_t, fl_t = psf.Table(**wl["table"]), psf.Table(**W.fl_table(wl["table"]))
    oe_o, fl_o = oracle.Oracle(**wl["table"]), oracle.Oracle(**W.fl_table(wl["table"]))
    for it in range(2):
        rec = dict(sc.generate(wl["gen"], it))
        rec["rough"] = None
        rec["footprint"] = W.footprints(rec, wl, spread=1.5)
        a, fl = W.estimator_inputs(rec, wl["gen"])
        a["footprint"] = rec["footprint"]
        fl = dict(fl, footprint=rec["footprint"])
        oe_t.iterate(to_device(rec))
        fl_t.iterate(to_device(fl))
        oe_o.insert(rec)
        oe_o.update()
        fl_o.insert(fl)
        fl_o.update()
    _, applied = _check(psf, oracle, oe_t, fl_t, oe_o, fl_o, a, 0, 0.75)
    assert applied.sum() > 0.5 * applied.numel()
