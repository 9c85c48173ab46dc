"""Pins of the footprint level rule (Sec. 2.3 selects levels by the path
footprint): hand-derived vectors, rejection of invalid footprints, agreement
with binary64 log2 away from powers of two, and agreement with the camera-
distance rule when the footprint is the width that rule assumes."""
import math
import struct

import numpy as np

import oracle
from tests.helpers import golden_rows, records

KEY_LEVEL = lambda k: (np.asarray(k, dtype=np.uint64) >> np.uint64(59)) & np.uint64(15)  # noqa: E731


def _f32(h):
    return struct.unpack(">f", bytes.fromhex(h))[0]


def test_footprint_levels_golden():
    for e_min, max_level, bits, want in golden_rows("footprint_levels.txt"):
        o = oracle.Oracle(e_min=int(e_min), max_level=int(max_level), kappa=0.0)
        k, _ = o.keys(records(1, px=0.1, py=0.2, pz=0.3, footprint=_f32(bits)))
        assert k[0] != np.uint64(2**64 - 1)
        assert int(KEY_LEVEL(k)[0]) == int(want), (e_min, max_level, bits)


def test_invalid_footprints_reject_the_vertex():
    o = oracle.Oracle(e_min=-5)
    fp = np.array([0.0, -1.0, np.inf, np.nan, -0.0, 1.0], dtype=np.float32)
    rec = records(6, px=0.1, footprint=fp)
    k, _ = o.keys(rec)
    assert list(k[:5] == np.uint64(2**64 - 1)) == [True] * 5 and k[5] != np.uint64(2**64 - 1)
    o.insert(rec)
    assert o.counters()["skipped"] == 5


def test_levels_match_float64_log2_away_from_powers_of_two():
    rng = np.random.default_rng(11)
    fp = np.exp2(rng.uniform(-12, 12, 4000)).astype(np.float32)
    lg = np.log2(fp.astype(np.float64))
    keep = np.abs(lg - np.round(lg)) > 1e-4
    o = oracle.Oracle(e_min=-6, max_level=15)
    k, _ = o.keys(records(len(fp), px=0.1, footprint=fp))
    want = np.clip(np.floor(lg) + 6, 0, 15)
    assert np.array_equal(KEY_LEVEL(k)[keep].astype(np.int64), want[keep].astype(np.int64))


def test_footprint_of_the_camera_rule_gives_its_level():
    """The camera-distance rule takes the footprint to be k_s theta d; passing
    that width as the footprint selects the same level (away from level
    boundaries, where the two roundings may differ)."""
    cam = (0.0, 0.0, -10.0)
    e_min, k_s, theta = -5, 8.0 * math.sqrt(2.0), 2.0 * math.tan(math.radians(30.0)) / 720.0
    kappa = float(np.float32((k_s * theta / 2.0 ** e_min) ** 2))
    rng = np.random.default_rng(5)
    p = rng.uniform(-8, 8, (3, 3000)).astype(np.float32)
    d = np.sqrt(np.sum((p.astype(np.float64) - np.array(cam)[:, None]) ** 2, axis=0))
    width = np.sqrt(kappa) * 2.0 ** e_min * d
    lg = np.log2(width) - e_min
    keep = np.abs(lg - np.round(lg)) > 1e-4
    by_cam = oracle.Oracle(cam=cam, kappa=kappa, e_min=e_min)
    by_fp = oracle.Oracle(cam=cam, kappa=kappa, e_min=e_min)
    rec = records(p.shape[1], px=p[0], py=p[1], pz=p[2])
    k_cam, _ = by_cam.keys(rec)
    k_fp, _ = by_fp.keys(dict(rec, footprint=width.astype(np.float32)))
    assert keep.mean() > 0.99
    assert np.array_equal(k_cam[keep], k_fp[keep])


def test_multi_level_lookup_worked_example():
    """Sec. 2.3's hierarchy: a cell of edge 1 (level 2 with e_min -2) holds
    5; a query of footprint 0.25 (level 0, edge 0.25) whose own cell and
    level-1 cell are empty is answered two levels up."""
    o = oracle.Oracle(e_min=-2, kappa=0.0)
    o.insert(records(1, px=0.3, py=0.3, pz=0.3, footprint=1.0, r=5.0, g=5.0, b=5.0))
    o.update()
    q = records(1, px=0.6, py=0.1, pz=0.9, footprint=0.25)
    for up, lv, val in ((0, 0, 0.0), (1, 0, 0.0), (2, 3, 5.0), (5, 3, 5.0)):
        out, level = o.query_levels(q, up)
        assert int(level[0]) == lv and np.all(out[:, 0] == val), (up, level, out)
    # a vertex in the same edge-1 cell but outside it at level 2 is not answered
    far = records(1, px=1.6, py=0.1, pz=0.9, footprint=0.25)
    assert int(o.query_levels(far, 4)[1][0]) == 0
    # the coarsest level stops the climb: a vertex already at max_level has no parents
    top = oracle.Oracle(e_min=-2, kappa=0.0, max_level=2)
    top.insert(records(1, px=0.3, py=0.3, pz=0.3, footprint=1.0, r=2.0, g=2.0, b=2.0))
    top.update()
    out, level = top.query_levels(records(1, px=0.5, py=0.5, pz=0.5, footprint=8.0), 3)
    assert int(level[0]) == 1 and np.all(out[:, 0] == 2.0)


def test_multi_level_lookup_without_climb_is_the_plain_query():
    from synth import workloads as W
    wl = W.tiny()
    sc = W.make_scene(wl)
    o = oracle.Oracle(**wl["table"])
    for it in range(2):
        rec = dict(sc.generate(wl["gen"], it))
        rec["rough"] = None
        o.insert(rec)
        o.update()
    out0, found = o.query(rec)
    out1, level = o.query_levels(rec, 0)
    assert np.array_equal(found, level) and np.array_equal(out0, out1)
