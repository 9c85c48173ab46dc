"""Host-side serving logic (no GPU): the arrival/resolution model."""
import math

import numpy as np


def test_arrivals_are_poisson_and_resolutions_clipped():
    from paper_2005_07547_amd import serving
    reqs = serving.draw_requests(4000, rate=20.0, seed=5)
    t = np.array([r[1] for r in reqs])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 1 / 20.0) < 0.005        # mean inter-arrival 1/rate
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.08  # exponential: cv = 1
    cls = np.array([r[2] for r in reqs])
    assert cls.min() >= 0 and cls.max() < len(serving.RES_CLASSES)
    # lognormal around 720p: the 1280x720 class is the mode
    assert np.bincount(cls).argmax() == serving.RES_CLASSES.index((1280, 720))
    iters = np.array([r[3] for r in reqs])
    assert iters.min() >= 32 and iters.max() <= 128
    assert len({r[0] for r in reqs}) == len(reqs)


def test_sessions_take_tables_without_accumulators_where_allowed():
    """A served session's table leaves out the frame accumulators when its
    configuration allows the partitioned strategy, else stays ordinary; the
    footprint follows (psf_table_bytes is host-side arithmetic)."""
    from paper_2005_07547_amd import psf, serving
    from synth import workloads as W
    cfg = dict(W.plain()["table"], log2_slots=20)
    recs = 1 << 18
    lean = serving.session_table_cfg(cfg, recs)
    assert lean["flags"] & psf.PSF_FLAG_NO_ACCUMULATORS and lean["max_batch"] == recs
    assert serving.session_table_cfg(cfg, recs, lean=False).get("flags", 0) & psf.PSF_FLAG_NO_ACCUMULATORS == 0
    assert (serving.table_footprint(cfg, recs, lean=False) - serving.table_footprint(cfg, recs)) == 16 << 20
    direct = dict(cfg, insert_mode=psf.PSF_INSERT_DIRECT)
    assert serving.session_table_cfg(direct, recs).get("flags", 0) & psf.PSF_FLAG_NO_ACCUMULATORS == 0
    assert serving.table_footprint(direct, recs) == serving.table_footprint(direct, recs, lean=False)
