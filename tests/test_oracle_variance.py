"""Pins of the oracle's per-cell luminance variance.

The paper keeps no per-cell variance; this project's reading (the spread of
a cell's samples around its approximant under the blend's own weights) is
pinned here against facts the oracle does not compute itself: numpy's
population variance for one frame and for linear accumulation (the blend's
linear limit, Sec. 2.4), numpy's weighted variance under the closed-form
weights of constant-alpha averaging, and the same identity under Eq. 11
with alpha read back from the blended state; hand-derived values fix the
luminance weights of Y = (r + 2 g + b) / 4.
"""
import numpy as np

import oracle
from oracle import ALPHA_CONST, ALPHA_LINEAR, ALPHA_PAPER, RESET_COUNTERS
from tests.helpers import concat, records


def _cfg(**kw):
    c = dict(cam=(0.0, 0.0, 0.0), kappa=0.0, e_min=0, max_level=15, normal_bins_log2=2,
             dir_bins_log2=3, rough_thr=0.3, alpha_mode=ALPHA_PAPER, alpha=0.2, t_max=5.0)
    c.update(kw)
    return c


def _cell(values, cell=(0, 0, 0), seed=0, weight=None):
    """Records of one unit cell (positions strictly inside it) with the
    given (3, n) values."""
    v = np.asarray(values, dtype=np.float32)
    n = v.shape[1]
    rng = np.random.default_rng(seed)
    p = (np.asarray(cell, dtype=np.float64)[:, None] + rng.uniform(0.05, 0.95, size=(3, n))).astype(np.float32)
    return records(n, px=p[0], py=p[1], pz=p[2], r=v[0], g=v[1], b=v[2], weight=weight)


def _y(v):
    v = np.asarray(v, dtype=np.float64)
    return (v[0] + 2.0 * v[1] + v[2]) / 4.0


def _var(orc):
    keys, var = orc.export_variance()
    return var


def test_luminance_weights_hand_derived():
    # two samples whose luminances are 0 and 1: population variance 1/4,
    # whichever channel carries the difference ((0, 2, 0) and (4, 0, 0) and
    # (0, 0, 4) all have Y = 1)
    for other in ((0.0, 2.0, 0.0), (4.0, 0.0, 0.0), (0.0, 0.0, 4.0)):
        orc = oracle.Oracle(**_cfg())
        orc.insert(_cell(np.array([[0.0, other[0]], [0.0, other[1]], [0.0, other[2]]])))
        orc.update()
        assert _var(orc)[0] == 0.25
    # chroma alone (Y constant) gives no luminance variance: (2, 0, 2) and (0, 2, 0)
    orc = oracle.Oracle(**_cfg())
    orc.insert(_cell(np.array([[2.0, 0.0], [0.0, 2.0], [2.0, 0.0]])))
    orc.update()
    assert _var(orc)[0] == 0.0


def test_single_frame_is_population_variance():
    rng = np.random.default_rng(5)
    v = rng.exponential(1.0, size=(3, 17)).astype(np.float32)
    orc = oracle.Oracle(**_cfg())
    orc.insert(_cell(v))
    orc.update()
    np.testing.assert_allclose(_var(orc)[0], np.var(_y(v)), rtol=1e-12)


def test_linear_mode_is_variance_of_every_sample():
    # linear accumulation weights every sample so far equally: the variance
    # is the plain population variance of all of them
    rng = np.random.default_rng(11)
    orc = oracle.Oracle(**_cfg(alpha_mode=ALPHA_LINEAR))
    seen = []
    for f in range(9):
        n = int(rng.integers(1, 7))
        v = (rng.exponential(1.0, size=(3, n)) * (1 + f % 3)).astype(np.float32)
        orc.insert(_cell(v, seed=f))
        orc.update()
        seen.append(_y(v))
        np.testing.assert_allclose(_var(orc)[0], np.var(np.concatenate(seen)), rtol=1e-11)


def _mixture(ys, betas):
    """Weighted population variance: sample i of frame j weighs beta_j / n_j."""
    y = np.concatenate(ys)
    w = np.concatenate([np.full(len(f), b / len(f)) for f, b in zip(ys, betas)])
    mean = np.average(y, weights=w)
    return np.average((y - mean) ** 2, weights=w), mean


def test_constant_mode_is_mixture_variance():
    # constant alpha: frame j of k weighs a (1 - a)^(k - j), the first frame
    # (alpha 1) (1 - a)^(k - 1)
    a = 0.3
    a32 = float(np.float32(a))
    rng = np.random.default_rng(13)
    orc = oracle.Oracle(**_cfg(alpha_mode=ALPHA_CONST, alpha=a))
    ys = []
    for f in range(12):
        n = int(rng.integers(1, 6))
        v = rng.uniform(0.0, 4.0, size=(3, n)).astype(np.float32)
        orc.insert(_cell(v, seed=f))
        orc.update()
        ys.append(_y(v))
        k = len(ys)
        betas = [(1 - a32) ** (k - 1)] + [a32 * (1 - a32) ** (k - 1 - j) for j in range(1, k)]
        want, mean = _mixture(ys, betas)
        np.testing.assert_allclose(_var(orc)[0], want, rtol=1e-11)
        # the mixture mean is the approximant's luminance
        np.testing.assert_allclose(_y(orc.export()["L"][:, 0]), mean, rtol=1e-12)


def test_eq11_is_mixture_variance_with_alpha_from_state():
    # Eq. 11: each frame's alpha is read back from the blended state (the
    # blend is L_new = (1 - alpha) L_old + alpha m); the variance must be
    # the mixture variance under the weights those alphas give
    rng = np.random.default_rng(17)
    orc = oracle.Oracle(**_cfg(alpha_mode=ALPHA_PAPER, t_max=4.0))
    ys, alphas = [], []
    L_old = None
    for f in range(24):
        n = int(rng.integers(1, 9))
        v = rng.uniform(0.0, 10.0, size=(3, n)).astype(np.float32)
        orc.insert(_cell(v, seed=f))
        orc.update()
        L = orc.export()["L"][0, 0]
        m = v[0].astype(np.float64).mean()
        alphas.append(1.0 if L_old is None else (L - L_old) / (m - L_old))
        L_old = L
        ys.append(_y(v))
        k = len(ys)
        betas = [alphas[j] * np.prod([1.0 - x for x in alphas[j + 1:]]) for j in range(k)]
        want, _ = _mixture(ys, betas)
        np.testing.assert_allclose(_var(orc)[0], want, rtol=1e-8)


def test_constant_field_has_no_variance():
    orc = oracle.Oracle(**_cfg())
    c = np.float32(0.7)
    for f in range(10):
        n = 1 + f % 4
        orc.insert(_cell(np.full((3, n), c, dtype=np.float32), seed=f))
        orc.update()
        assert 0.0 <= _var(orc)[0] <= 1e-15


def test_counter_reset_restarts_the_variance():
    rng = np.random.default_rng(19)
    orc = oracle.Oracle(**_cfg())
    for f in range(4):
        orc.insert(_cell(rng.uniform(0, 5, size=(3, 4)).astype(np.float32), seed=f))
        orc.update()
    orc.reset(RESET_COUNTERS)
    v = rng.uniform(0, 5, size=(3, 6)).astype(np.float32)
    orc.insert(_cell(v, seed=9))
    orc.update()
    np.testing.assert_allclose(_var(orc)[0], np.var(_y(v)), rtol=1e-12)


def test_weight_equals_repeats():
    # a sample of weight k counts as k copies of itself (Eq. 5-6)
    v = np.array([[1.0, 3.0], [0.5, 2.0], [2.0, 0.0]], dtype=np.float32)
    a = oracle.Oracle(**_cfg(), weighted=1)
    a.insert(_cell(v, weight=np.array([1.0, 3.0], dtype=np.float32)))
    a.update()
    b = oracle.Oracle(**_cfg())
    b.insert(_cell(v[:, [0, 1, 1, 1]]))
    b.update()
    np.testing.assert_allclose(_var(a)[0], _var(b)[0], rtol=1e-13)


def test_sharded_variance_identical():
    rng = np.random.default_rng(23)
    single = oracle.Oracle(**_cfg())
    sharded = oracle.ShardedOracle(4, **_cfg())
    for f in range(5):
        parts = [_cell(rng.exponential(1.0, size=(3, int(rng.integers(1, 5)))).astype(np.float32),
                       cell=(i, f % 2, 0), seed=10 * f + i) for i in range(12)]
        rec = concat(parts)
        single.insert(rec)
        sharded.insert(rec)
        single.update()
        sharded.update()
    k1, v1 = single.export_variance()
    k2, v2 = sharded.export_variance()
    assert np.array_equal(k1, k2)
    assert np.array_equal(v1, v2)
