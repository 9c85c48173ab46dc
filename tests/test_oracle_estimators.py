"""Pins of the oracle's two-field estimators (Sec. 2.5 fields, Sec. 4.2
control variate, Sec. 5 biased estimator): hand-derived worked examples, the
limits the paper names, and unbiasedness when the control variate's integral
is exact."""
import math

import numpy as np

import oracle
from tests.helpers import golden_rows, records

CFG = dict(kappa=0.0, e_min=-2, max_level=0)       # one fixed grid level
FL_CFG = dict(CFG, rough_thr=float("inf"))          # f L_i field: directional keys


def _vertex(n=1, **kw):
    base = dict(px=0.3, py=0.2, pz=0.1, nx=0.0, ny=0.0, nz=1.0, oox=0.0, ooy=0.6, ooz=0.8,
                oix=0.6, oiy=0.0, oiz=0.8, rough=1.0, gr=1.0, gg=1.0, gb=1.0, wp=1.0)
    base.update(kw)
    return {k: np.broadcast_to(np.asarray(v, dtype=np.float32), (n,)).copy() if np.ndim(v) == 0
            else np.asarray(v, dtype=np.float32) for k, v in base.items()}


def _fields(a, L, h):
    """Oracles holding one blended cell each: L at (x, w_o), h at (x, w_i)."""
    oe, fl = oracle.Oracle(**CFG), oracle.Oracle(**FL_CFG)
    oe.insert(records(1, px=a["px"][:1], py=a["py"][:1], pz=a["pz"][:1], ox=a["oox"][:1],
                      oy=a["ooy"][:1], oz=a["ooz"][:1], rough=a["rough"][:1], r=L, g=L, b=L))
    fl.insert(records(1, px=a["px"][:1], py=a["py"][:1], pz=a["pz"][:1], ox=a["oix"][:1],
                      oy=a["oiy"][:1], oz=a["oiz"][:1], rough=a["rough"][:1], r=h, g=h, b=h))
    oe.update()
    fl.update()
    return oe, fl


def test_estimators_worked_examples():
    for mode, param, L, h, g, wp, want in golden_rows("estimators.txt"):
        a = _vertex(gr=float(g), gg=float(g), gb=float(g), wp=float(wp))
        oe, fl = _fields(a, float(L), float(h))
        m = oracle.EST_CV if mode == "cv" else oracle.EST_BIASED
        e, applied = oracle.estimate(oe, fl, a, m, float(param))
        assert applied[0] == 1
        assert np.all(e[:, 0] == float(want)), (mode, param, e[:, 0], want)


def test_limits_named_by_the_paper():
    """beta = 0 is the plain estimate; gamma = 0 is the predictor alone
    (path space filtering); gamma = 1 is the control variate with beta = 1."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        L, h, g, wp = rng.uniform(0.1, 5.0, 4).astype(np.float32)
        a = _vertex(gr=g, gg=g, gb=g, wp=wp)
        oe, fl = _fields(a, L, h)
        e0, _ = oracle.estimate(oe, fl, a, oracle.EST_CV, 0.0)
        assert np.allclose(e0, float(wp) * float(g), rtol=0, atol=0)
        p0, _ = oracle.estimate(oe, fl, a, oracle.EST_BIASED, 0.0)
        assert np.all(p0 == float(L))
        c1, _ = oracle.estimate(oe, fl, a, oracle.EST_CV, 1.0)
        b1, _ = oracle.estimate(oe, fl, a, oracle.EST_BIASED, 1.0)
        assert np.allclose(c1, b1, rtol=1e-15)


def test_missing_cell_keeps_plain_estimate():
    a = _vertex(n=2, gr=[2.0, 2.0], gg=[2.0, 2.0], gb=[2.0, 2.0], wp=[3.0, 3.0])
    oe, fl = _fields(a, 5.0, 1.0)
    # second vertex: a sampled direction in another octahedral bin, whose
    # f L_i cell was never filled
    a["oix"][1], a["oiy"][1], a["oiz"][1] = -0.6, 0.0, 0.8
    e, applied = oracle.estimate(oe, fl, a, oracle.EST_CV, 0.5)
    assert list(applied) == [1, 0]
    assert np.all(e[:, 1] == 6.0)
    assert np.all(e[:, 0] == 3.0 * (2.0 - 0.5) + 2.5)


def test_exact_control_variate_leaves_the_expectation_unchanged():
    """If h = c in every direction and its integral over projected solid
    angle, pi c, is the cell value L, then with uniform projected-solid-angle
    sampling (w = 1, wp = pi) the estimate is pi g for every beta: the
    control variate changes no expectation (the estimator stays unbiased).
    Adding beta L inside the wp factor instead would give pi (g - beta c +
    beta pi c) and fail here."""
    c = 0.75
    rng = np.random.default_rng(7)
    k = 256
    # directions spread over the upper hemisphere (normal +z)
    u, v = rng.uniform(0, 1, k), rng.uniform(0, 1, k)
    r, phi = np.sqrt(u), 2 * np.pi * v
    dx, dy = r * np.cos(phi), r * np.sin(phi)
    dz = np.sqrt(np.maximum(0.0, 1 - dx * dx - dy * dy))
    g = rng.uniform(0.0, 4.0, k)
    a = _vertex(n=k, oix=dx, oiy=dy, oiz=dz, gr=g, gg=g, gb=g, wp=np.float32(math.pi))
    oe, fl = oracle.Oracle(**CFG), oracle.Oracle(**FL_CFG)
    oe.insert(records(1, px=0.3, py=0.2, pz=0.1, ox=0.0, oy=0.6, oz=0.8, rough=1.0,
                      r=math.pi * c, g=math.pi * c, b=math.pi * c))
    fl.insert(records(k, px=a["px"], py=a["py"], pz=a["pz"], ox=a["oix"], oy=a["oiy"], oz=a["oiz"],
                      rough=a["rough"], r=c, g=c, b=c))
    oe.update()
    fl.update()
    pi32 = float(np.float32(math.pi))
    for beta in (0.3, 1.0, 2.0):
        e, applied = oracle.estimate(oe, fl, a, oracle.EST_CV, beta)
        assert applied.all()
        # pi g, up to the binary32 rounding of the stored pi c and of pi
        assert np.allclose(e, pi32 * a["gr"].astype(np.float64), rtol=0, atol=1e-6 * (1 + beta))
