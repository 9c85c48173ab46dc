"""Pins of the oracle's two-band SH YCoCg cell payload (Sec. 2.6): what the
reading must reproduce in closed form.  Cells are keyed by position only
(one normal bin), so a cell's samples carry different normals."""
import numpy as np

import oracle
from tests.helpers import records

K0, K1 = 0.28209479177387814, 0.4886025119029199


def basis(n):
    return np.stack([np.full(n.shape[1], K0), K1 * n[1], K1 * n[2], K1 * n[0]])


def ycocg_to_rgb(y, co, cg):
    return np.stack([y + co - cg, y + cg, y - co - cg])


def _normals(m, rng, hemisphere=False):
    v = rng.normal(size=(3, m))
    v /= np.linalg.norm(v, axis=0)
    if hemisphere:
        v[2] = np.abs(v[2])
    return v.astype(np.float32)


def _cell_records(nrm, rgb):
    m = nrm.shape[1]
    # one cell: every record at the same point, fixed level, one normal bin
    return records(m, px=0.25, py=0.25, pz=0.25, nx=nrm[0], ny=nrm[1], nz=nrm[2], r=rgb[0], g=rgb[1], b=rgb[2])


def _orc(**kw):
    return oracle.ShOracle(normal_bins_log2=0, e_min=0, kappa=0.0, **kw)


def test_rgb_ycocg_round_trip():
    rng = np.random.default_rng(0)
    rgb = rng.uniform(-1, 2, size=(3, 100))
    y = 0.25 * rgb[0] + 0.5 * rgb[1] + 0.25 * rgb[2]
    co = 0.5 * rgb[0] - 0.5 * rgb[2]
    cg = -0.25 * rgb[0] + 0.5 * rgb[1] - 0.25 * rgb[2]
    assert np.allclose(ycocg_to_rgb(y, co, cg), rgb, atol=1e-15)


def test_constant_field_is_reproduced_at_every_normal():
    rng = np.random.default_rng(1)
    nrm = _normals(500, rng)
    rgb = np.tile(np.array([[0.7], [0.4], [0.2]], dtype=np.float32), (1, 500))
    o = _orc()
    o.insert(_cell_records(nrm, rgb))
    o.update()
    q = _normals(50, rng)
    got, found = o.query(_cell_records(q, np.zeros((3, 50), np.float32)))
    assert found.all()
    assert np.allclose(got, rgb[:, :1].astype(np.float64), rtol=1e-12, atol=1e-12)
    ex = o.export()
    # band 1 is zero, band 0 carries Y / k0
    assert np.allclose(ex["coeff"][1:4, 0], 0.0, atol=1e-12)
    r, g, b = (float(np.float32(v)) for v in (0.7, 0.4, 0.2))
    assert abs(ex["coeff"][0, 0] * K0 - (0.25 * r + 0.5 * g + 0.25 * b)) < 1e-12


def test_luminance_linear_in_the_normal_is_recovered():
    rng = np.random.default_rng(2)
    a = np.array([1.3, 0.4, -0.25, 0.6])
    nrm = _normals(2000, rng)
    y = a @ basis(nrm.astype(np.float64))
    co, cg = 0.1, -0.05
    rgb = ycocg_to_rgb(y, co, cg).astype(np.float32)
    o = _orc()
    o.insert(_cell_records(nrm, rgb))
    o.update()
    ex = o.export()
    # float32 records: the fitted coefficients agree to the inputs' rounding
    # and the ridge's 1e-7 shrinkage
    assert np.allclose(ex["coeff"][:4, 0], a, rtol=0, atol=2e-6)
    q = _normals(100, rng)
    got, _ = o.query(_cell_records(q, np.zeros((3, 100), np.float32)))
    want = ycocg_to_rgb(a @ basis(q.astype(np.float64)), co, cg)
    assert np.allclose(got, want, atol=5e-6)


def test_chroma_is_the_plain_mean():
    rng = np.random.default_rng(3)
    nrm = _normals(300, rng)
    rgb = rng.uniform(0, 2, size=(3, 300)).astype(np.float32)
    o = _orc()
    o.insert(_cell_records(nrm, rgb))
    o.update()
    r64 = rgb.astype(np.float64)
    ex = o.export()
    assert abs(ex["coeff"][4, 0] - np.mean(0.5 * r64[0] - 0.5 * r64[2])) < 1e-12
    assert abs(ex["coeff"][5, 0] - np.mean(-0.25 * r64[0] + 0.5 * r64[1] - 0.25 * r64[2])) < 1e-12


def test_flat_cell_reproduces_its_mean_at_its_normal():
    """All normals equal: only the combination of coefficients seen at that
    normal is determined; the fit returns the samples' mean there."""
    rng = np.random.default_rng(4)
    m = 64
    nrm = np.tile(np.array([[0.0], [0.6], [0.8]], dtype=np.float32), (1, m))
    rgb = rng.uniform(0, 1, size=(3, m)).astype(np.float32)
    o = _orc()
    o.insert(_cell_records(nrm, rgb))
    o.update()
    got, _ = o.query(_cell_records(nrm[:, :1], np.zeros((3, 1), np.float32)))
    assert np.allclose(got[:, 0], rgb.astype(np.float64).mean(axis=1), rtol=1e-6)


def test_coefficients_blend_with_constant_alpha():
    """Two frames of two linear fields: the state is the Eq. 10 blend of the
    two fits (first touch alpha = 1, then the constant alpha)."""
    rng = np.random.default_rng(5)
    a1, a2 = np.array([1.0, 0.2, 0.0, -0.1]), np.array([0.5, -0.3, 0.4, 0.2])
    o = _orc(alpha_mode=oracle.ALPHA_CONST, alpha=0.25)
    for a in (a1, a2):
        nrm = _normals(1500, rng)
        rgb = ycocg_to_rgb(a @ basis(nrm.astype(np.float64)), 0.0, 0.0).astype(np.float32)
        o.insert(_cell_records(nrm, rgb))
        o.update()
    c = o.export()["coeff"][:4, 0]
    assert np.allclose(c, 0.75 * a1 + 0.25 * a2, atol=3e-6)


def test_cells_are_independent_and_weights_act_as_repeats():
    """Weight 2 on a record equals the record twice (Eq. 5-6 with w)."""
    rng = np.random.default_rng(6)
    nrm = _normals(40, rng)
    rgb = rng.uniform(0, 1, size=(3, 40)).astype(np.float32)
    rec = _cell_records(nrm, rgb)
    twice = {k: (None if v is None else np.concatenate([v, v])) for k, v in rec.items()}
    w = dict(rec, weight=np.full(40, 2.0, np.float32))
    a, b = _orc(), _orc()
    a.insert(twice)
    b.insert(w)
    a.update()
    b.update()
    ea, eb = a.export(), b.export()
    assert np.array_equal(ea["c_old"], eb["c_old"])
    assert np.allclose(ea["coeff"], eb["coeff"], rtol=1e-12, atol=1e-14)
