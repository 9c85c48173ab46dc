"""GPU parity of the two-band SH YCoCg cell payload (Sec. 2.6) against the
binary64 oracle: keys and counters bit-exact; the six state numbers and the
lookups within 1e-5 of the magnitude of the terms they are made of (the
state is binary32; the per-frame fit is binary64 on both sides)."""
import numpy as np
import pytest

from tests.helpers import records, to_device
from tests.test_oracle_sh import basis, ycocg_to_rgb

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_07547_amd import psf
    psf.load()
    return torch, psf


def _cfg(wl, **kw):
    return dict(wl["table"], normal_bins_log2=0, payload=1, insert_mode=1, **kw)


def _compare(psf, t, orc, rec):
    g = psf.export_sh(t)
    o = orc.export()
    assert np.array_equal(g["keys"], o["keys"])
    if orc._cfg.get("weighted"):
        # binary32 counter words against binary64 weight sums
        assert np.allclose(g["c_old"].astype(np.float64), o["c_old"], rtol=1e-6)
    else:
        assert np.array_equal(g["c_old"].astype(np.float64), o["c_old"])
    scale = np.max(np.abs(o["coeff"]), axis=0) + 1e-30
    err = np.max(np.abs(g["coeff"].astype(np.float64) - o["coeff"]), axis=0) / scale
    assert float(err.max()) <= TOL, float(err.max())
    out, found = t.query(to_device(rec))
    w_out, w_found = orc.query(rec)
    assert np.array_equal(found.cpu().numpy(), w_found)
    # error bound of a binary32 evaluation: relative to the terms' magnitude
    nrm = np.stack([rec["nx"], rec["ny"], rec["nz"]]).astype(np.float64)
    kq, _ = orc_keys(orc, rec)
    mag = _term_magnitude(o, kq, nrm)
    d = np.abs(out.cpu().numpy().astype(np.float64) - w_out).max(axis=0)
    hit = w_found.astype(bool)
    assert np.all(d[hit] <= TOL * mag[hit] + 1e-30), float((d[hit] / mag[hit]).max())
    return float(err.max())


def orc_keys(orc, rec):
    import oracle
    plain = oracle.Oracle(**{k: v for k, v in orc._cfg.items()})
    return plain.keys(rec)


def _term_magnitude(o, keys, nrm):
    idx = np.searchsorted(o["keys"], keys)
    idx = np.clip(idx, 0, max(0, len(o["keys"]) - 1))
    c = o["coeff"][:, idx]
    b = basis(nrm)
    return np.sum(np.abs(c[:4] * b), axis=0) + np.abs(c[4]) + np.abs(c[5])


def _oracle(cfg):
    import oracle
    o = oracle.ShOracle(**cfg)
    o._cfg = cfg
    return o


@pytest.mark.parametrize("weighted", [0, 1])
def test_tiny_workload_sh_payload_matches_the_oracle(env, weighted):
    from synth import workloads as W
    torch, psf = env
    wl = W.tiny(alpha_mode=W.ALPHA_PAPER)
    sc = W.make_scene(wl)
    cfg = _cfg(wl, weighted=weighted)
    t = psf.Table(**cfg)
    orc = _oracle(cfg)
    rng = np.random.default_rng(8)
    for it in range(5):
        rec = dict(sc.generate(wl["gen"], it))
        rec["rough"] = None
        if weighted:
            rec["weight"] = rng.uniform(0.1, 2.0, rec["px"].shape[0]).astype(np.float32)
        t.iterate(to_device(rec))
        orc.insert(rec)
        orc.update()
    torch.cuda.synchronize()
    worst = _compare(psf, t, orc, rec)
    print(f"tiny SH payload (weighted={weighted}): worst coefficient error {worst:.2e}")
    st = t.stats()
    assert st["dropped"] == 0 and st["updates"] == 5


def test_linear_luminance_is_recovered_on_the_device(env):
    torch, psf = env
    rng = np.random.default_rng(9)
    a = np.array([1.3, 0.4, -0.25, 0.6])
    m = 4000
    nrm = rng.normal(size=(3, m))
    nrm /= np.linalg.norm(nrm, axis=0)
    nrm = nrm.astype(np.float32)
    rgb = ycocg_to_rgb(a @ basis(nrm.astype(np.float64)), 0.1, -0.05).astype(np.float32)
    rec = records(m, px=0.25, py=0.25, pz=0.25, nx=nrm[0], ny=nrm[1], nz=nrm[2], r=rgb[0], g=rgb[1], b=rgb[2])
    t = psf.Table(log2_slots=10, e_min=0, kappa=0.0, normal_bins_log2=0, payload=1, insert_mode=1)
    t.iterate(to_device(rec))
    ex = psf.export_sh(t)
    assert len(ex["keys"]) == 1
    assert np.allclose(ex["coeff"][:4, 0], a, atol=3e-6)
    assert np.allclose(ex["coeff"][4:, 0], [0.1, -0.05], atol=1e-6)


def test_sh_table_arguments(env):
    torch, psf = env
    with pytest.raises(psf.PsfError):
        psf.Table(log2_slots=10, payload=1, insert_mode=2)
    with pytest.raises(psf.PsfError):
        psf.Table(log2_slots=10, payload=1, state_dtype=1)
    with pytest.raises(psf.PsfError):
        psf.Table(log2_slots=10, payload=2)
    t = psf.Table(log2_slots=10, payload=1)
    with pytest.raises(psf.PsfError):
        t.export()
    plain = psf.Table(log2_slots=10)
    with pytest.raises(psf.PsfError):
        psf.export_sh(plain)
