"""The key-sharded oracle (one map per host thread) equals the single-threaded
oracle bit for bit: cells are independent and each sees its samples in array
order."""
import numpy as np

import oracle
from synth import workloads as W


def _same(a, b):
    for k in ("keys", "n_new", "c_old"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["L"].view(np.uint64), b["L"].view(np.uint64))
    assert np.array_equal(a["s"].view(np.uint64), b["s"].view(np.uint64))


def test_sharded_equals_single_on_the_tiny_and_plain_workloads():
    for wl, frames in ((W.tiny(alpha_mode=W.ALPHA_PAPER), 4), (W.plain(), 2)):
        sc = W.make_scene(wl)
        one = oracle.Oracle(**wl["table"])
        many = oracle.ShardedOracle(5, **wl["table"])
        for it in range(frames):
            rec = dict(sc.generate(wl["gen"], it))
            if wl["name"] != "tiny":
                rec = {k: (None if v is None else v[: 400_000]) for k, v in rec.items()}
            # a few rejected records
            rec["px"] = rec["px"].copy()
            rec["px"][::997] = np.nan
            for o in (one, many):
                o.insert(rec)
            if it + 1 < frames:
                assert one.update() == many.update()
        _same(one.export(), many.export())  # pending sums included
        assert one.counters() == many.counters()
        one.update()
        many.update()
        a, fa = one.query(rec)
        b, fb = many.query(rec)
        assert np.array_equal(fa, fb) and np.array_equal(a.view(np.uint64), b.view(np.uint64))
        assert fa.sum() > 0


def test_sharded_filter_keeps_the_same_cells():
    wl = W.tiny(alpha_mode=W.ALPHA_PAPER)
    sc = W.make_scene(wl)
    rec = dict(sc.generate(wl["gen"], 0))
    one = oracle.Oracle(**wl["table"])
    many = oracle.ShardedOracle(3, **wl["table"])
    k, _ = one.keys(rec)
    pick = np.unique(k[k != np.uint64(2 ** 64 - 1)])[::7]
    for o in (one, many):
        o.set_filter(pick)
        o.insert(rec)
        o.update()
    a, b = one.export(), many.export()
    _same(a, b)
    assert np.array_equal(a["keys"], pick)
