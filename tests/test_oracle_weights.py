"""Pins of the MIS-weighted counters (Eq. 5-6 with weights w != 1; Sec. 2.5's
down-weighted fields, Eq. 10-11 on weighted counters) in the oracle.

None of these retypes the oracle's formulas: each compares two oracle runs
whose results the mathematics ties together, or checks a property the
definition fixes.
  * a record of integer weight k is k records of weight 1 (the counter is a
    sum of weights, the numerator a weighted sum), over several frames of
    the PAPER blend, so alpha's counters are pinned too;
  * MIS weights that partition one: a sample split into copies of weights w
    and 1 - w is that sample inserted once;
  * scaling every weight by 2^k leaves the approximant unchanged (alpha and
    the mean are ratios of weight sums) and scales the counters;
  * the first blend of a cell is the weighted mean of its samples and lies
    between their extremes;
  * weights that are not finite and > 0 reject the sample;
  * without weights a weighted table equals an unweighted one.
"""
import numpy as np
import pytest

import oracle
from oracle import ALPHA_CONST, ALPHA_LINEAR, ALPHA_PAPER
from synth import workloads as W
from tests.helpers import concat, records, take


def _frame(it):
    wl = W.tiny(alpha_mode=ALPHA_PAPER)
    rec = dict(W.make_scene(wl).generate(wl["gen"], it))
    rec["rough"] = None
    return wl, rec


def _run(table, frames, weighted=1):
    o = oracle.Oracle(**dict(table, weighted=weighted))
    for rec in frames:
        o.insert(rec)
        o.update()
    return o


@pytest.mark.parametrize("alpha_mode", [ALPHA_PAPER, ALPHA_LINEAR, ALPHA_CONST])
def test_integer_weight_equals_repeated_records(alpha_mode):
    wl, _ = _frame(0)
    table = dict(wl["table"], alpha_mode=alpha_mode, t_max=50.0)
    weighted, repeated = [], []
    for it in range(4):
        _, rec = _frame(it)
        n = len(rec["px"])
        k = (np.arange(n) * 7 + it) % 3 + 1  # 1, 2 or 3
        weighted.append(dict(rec, weight=k.astype(np.float32)))
        idx = np.repeat(np.arange(n), k)
        repeated.append(take(rec, idx))
    a = _run(table, weighted)
    b = _run(table, repeated, weighted=0)
    ea, eb = a.export(), b.export()
    assert np.array_equal(ea["keys"], eb["keys"])
    assert np.array_equal(ea["c_old"], eb["c_old"].astype(np.float64))
    np.testing.assert_allclose(ea["L"], eb["L"], rtol=1e-12, atol=0)


def test_weights_partitioning_one_equal_a_single_sample():
    wl, _ = _frame(0)
    frames_w, frames_1 = [], []
    for it in range(3):
        _, rec = _frame(it)
        n = len(rec["px"])
        w = ((np.arange(n) * 37 + 11 * it) % 255 + 1).astype(np.float32) / np.float32(256.0)
        frames_w.append(concat([dict(rec, weight=w), dict(rec, weight=np.float32(1.0) - w)]))
        frames_1.append(rec)
    a = _run(wl["table"], frames_w)
    b = _run(wl["table"], frames_1, weighted=0)
    ea, eb = a.export(), b.export()
    assert np.array_equal(ea["keys"], eb["keys"])
    assert np.array_equal(ea["c_old"], eb["c_old"].astype(np.float64))
    np.testing.assert_allclose(ea["L"], eb["L"], rtol=1e-12, atol=1e-300)


def test_scaling_all_weights_keeps_the_approximant():
    wl, _ = _frame(0)
    table = dict(wl["table"], t_max=50.0)
    frames = []
    for it in range(3):
        _, rec = _frame(it)
        frames.append(dict(rec, weight=W.mis_weights(len(rec["px"]), seed=it, excluded=0.0)))
    a = _run(table, frames)
    b = _run(table, [dict(r, weight=r["weight"] * np.float32(8.0)) for r in frames])
    ea, eb = a.export(), b.export()
    assert np.array_equal(ea["keys"], eb["keys"])
    assert np.array_equal(eb["c_old"], 8.0 * ea["c_old"])
    assert np.array_equal(ea["L"], eb["L"])


def test_first_blend_is_a_weighted_mean_inside_the_sample_range():
    # one cell, five samples: the mean moves toward the heavy sample
    vals = np.array([1.0, 2.0, 4.0, 8.0, 16.0], dtype=np.float32)
    w = np.array([0.5, 0.25, 0.125, 0.0625, 2.0], dtype=np.float32)
    o = oracle.Oracle(weighted=1, e_min=0, kappa=0.0)
    o.insert(records(5, px=0.5, py=0.5, pz=0.5, r=vals, g=vals, b=vals, weight=w))
    o.update()
    ex = o.export()
    assert ex["c_old"].tolist() == [2.9375]
    L = ex["L"][0, 0]
    # sum w v = 0.5 + 0.5 + 0.5 + 0.5 + 32 = 34, over 2.9375
    assert L == 34.0 / 2.9375
    assert vals.min() < L < vals.max() and L > np.mean(vals.astype(np.float64))


def test_invalid_weights_reject_the_sample():
    wl, rec = _frame(0)
    n = len(rec["px"])
    w = W.mis_weights(n, seed=3, excluded=0.2)
    bad_idx = np.arange(5, n, 211)
    w[bad_idx[0::3]] = np.nan
    w[bad_idx[1::3]] = -0.5
    w[bad_idx[2::3]] = np.inf
    a = oracle.Oracle(**dict(wl["table"], weighted=1))
    a.insert(dict(rec, weight=w))
    good = np.isfinite(w) & (w > 0)
    b = oracle.Oracle(**dict(wl["table"], weighted=1))
    b.insert(take(dict(rec, weight=w), np.nonzero(good)[0]))
    assert a.counters()["skipped"] == int((~good).sum())
    a.update()
    b.update()
    ea, eb = a.export(), b.export()
    assert np.array_equal(ea["keys"], eb["keys"]) and np.array_equal(ea["c_old"], eb["c_old"])
    assert np.array_equal(ea["L"], eb["L"])


def test_weighted_table_without_weights_is_the_plain_table():
    wl, _ = _frame(0)
    frames = [_frame(it)[1] for it in range(3)]
    a = _run(wl["table"], frames)
    b = _run(wl["table"], frames, weighted=0)
    ea, eb = a.export(), b.export()
    assert ea["c_old"].dtype == np.float64 and eb["c_old"].dtype == np.uint64
    assert np.array_equal(ea["c_old"], eb["c_old"].astype(np.float64))
    assert np.array_equal(ea["L"], eb["L"])


def test_unweighted_table_refuses_weights():
    o = oracle.Oracle()
    with pytest.raises(ValueError):
        o.insert(records(2, weight=np.ones(2, np.float32)))
