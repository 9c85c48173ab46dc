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
