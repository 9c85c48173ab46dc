"""Serving form: continuous batching with admission against an HBM budget.
Each session's result is the same alone and in the mix."""
import numpy as np
import pytest

from tests.helpers import rel_err, to_device

pytestmark = pytest.mark.gpu
RTOL_F32 = 1e-5


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_07547_amd import psf, serving
    psf.load()
    return torch, psf, serving


def _requests(serving, n=6, scale_classes=(0, 1, 1, 2, 0, 1), iters=(4, 6, 3, 5, 7, 4),
              arrivals=(0.0, 0.0, 0.002, 0.004, 0.02, 0.03)):
    from synth import Scene, workloads as W
    reqs = []
    for i in range(n):
        w, h = serving.RES_CLASSES[scale_classes[i]]
        wl = W.plain()
        gen = dict(wl["gen"], width=w, height=h, seed=900 + i)
        sc = Scene(Scene.RANDOM, seed=900 + i, glossy_frac=-1.0 if i % 2 else 0.5)
        host = [sc.generate(gen, f) for f in range(2)]
        frames = [to_device(h) for h in host]
        # cells sized for this resolution; four slots per record keeps every
        # partition far from full over the session
        cfg = dict(wl["table"], log2_slots=max(16, int(np.ceil(np.log2(w * h * 4))) + 2),
                   kappa=W.kappa_for(60.0, h, 8.0 * np.sqrt(2.0), -5))
        req = serving.SessionRequest(sid=i, arrival=arrivals[i], iterations=iters[i],
                                     table_cfg=cfg, frames=frames, records=w * h * 4)
        req.host_frames = host  # the same frames on the host, for the oracle
        reqs.append(req)
    return reqs


def test_results_same_alone_and_in_the_mix(env):
    """Every served session against the binary64 oracle fed the same frames
    (keys and counts bit-exact, FP32 state within 1e-5, last answers), and
    against the same session run alone."""
    import oracle
    from tests.helpers import compare_cells
    torch, psf, serving = env
    reqs = _requests(serving)
    srv = serving.Server(budget_bytes=64 << 30, max_active=16, keep_tables=True)
    summary = srv.run(reqs, time_limit=120)
    torch.cuda.synchronize()
    assert summary["sessions"] == len(reqs)
    assert summary["peak_active"] >= 2  # sessions overlapped on the device
    for r in reqs:
        alone = psf.Table(**dict(r.table_cfg, max_batch=r.records))
        for it in range(r.iterations):
            out, found = alone.iterate(r.frames[it % len(r.frames)])
        ea, em = alone.export(), r.table.export()
        assert np.array_equal(ea["keys"], em["keys"]), r.sid
        assert np.array_equal(ea["c_old"], em["c_old"]), r.sid
        assert rel_err(em["L"], ea["L"]).max() <= RTOL_F32
        assert r.table.stats()["updates"] == r.iterations
        assert r.table.stats()["dropped"] == 0
        assert len(r.latencies_ms) == r.iterations
        # served without frame accumulators: 16 bytes per slot less
        assert r.table.cfg.flags & psf.PSF_FLAG_NO_ACCUMULATORS
        assert alone.nbytes - r.table.nbytes == 16 << int(r.table_cfg["log2_slots"])
        assert r.footprint == serving.table_footprint(r.table_cfg, r.records, lean=False) - alone.nbytes + \
            r.table.nbytes
        orc = oracle.Oracle(**r.table_cfg)
        for it in range(r.iterations):
            orc.insert(r.host_frames[it % len(r.host_frames)])
            orc.update()
        compare_cells(em, orc.export(), RTOL_F32, f"served session {r.sid}")
        # the served answers of the session's last iteration
        w_out, w_found = orc.query(r.host_frames[(r.iterations - 1) % len(r.host_frames)])
        assert np.array_equal(r.found.cpu().numpy(), w_found), r.sid
        assert rel_err(r.out.cpu().numpy(), w_out).max() <= RTOL_F32, r.sid


def test_budget_forces_queueing(env):
    torch, psf, serving = env
    reqs = _requests(serving)
    need = max(serving.table_footprint(r.table_cfg, r.records) for r in reqs)
    srv = serving.Server(budget_bytes=int(need * 1.5), max_active=16)
    summary = srv.run(reqs, time_limit=120)
    assert summary["sessions"] == len(reqs)
    assert summary["peak_resident_bytes"] <= int(need * 1.5)
    assert summary["peak_active"] < len(reqs)
    assert summary["mean_queue_s"] > 0


def test_session_above_budget_is_rejected(env):
    torch, psf, serving = env
    reqs = _requests(serving, n=1, scale_classes=(2,), iters=(2,), arrivals=(0.0,))
    srv = serving.Server(budget_bytes=1 << 20)
    with pytest.raises(ValueError):
        srv.run(reqs)
