"""Batched form: every session's result is the same alone and in the mix,
matches the oracle, survives fallback sessions and hipGraph replay."""
import numpy as np
import pytest

from tests.helpers import compare_cells, rel_err, to_device

pytestmark = pytest.mark.gpu
RTOL_F32 = 1e-5


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_07547_amd import psf
    psf.load()
    return torch, psf


def _sessions(n_sessions=5, scale=8):
    """Uneven sessions of the batched workload, resolution divided by scale."""
    from synth import workloads as W
    out = []
    for wl in W.batched_sessions(n_sessions):
        g = dict(wl["gen"])
        g["width"] = max(16, g["width"] // scale)
        g["height"] = max(16, g["height"] // scale)
        wl = dict(wl, gen=g, table=dict(wl["table"], log2_slots=max(14, wl["table"]["log2_slots"] - 4)))
        out.append((wl, W.make_scene(wl)))
    return out


def _frame(wl, sc, it):
    return sc.generate(wl["gen"], it)


@pytest.mark.parametrize("transpose,part_log2", [(False, 0), (True, 0), (False, 12), (True, 12)])
def test_batch_equals_alone_and_oracle(env, transpose, part_log2):
    import oracle
    torch, psf = env
    ss = _sessions()
    # transposing every session's run table covers the merge pass's other
    # way of reading it; mixing flags covers sessions that differ in it;
    # 4096-slot partitions in every session take the 1024-thread merge
    fl = [psf.PSF_FLAG_TRANSPOSE_RUNS if transpose and i % 2 == 0 else 0 for i in range(len(ss))]
    alone = [psf.Table(**wl["table"], flags=f, part_log2=part_log2) for (wl, _), f in zip(ss, fl)]
    mixed = [psf.Table(**wl["table"], flags=f, part_log2=part_log2) for (wl, _), f in zip(ss, fl)]
    orcs = [oracle.Oracle(**wl["table"]) for wl, _ in ss]
    batch = psf.Batch(16)
    for it in range(3):
        recs = [_frame(wl, sc, it) for wl, sc in ss]
        dev = [to_device(r) for r in recs]
        res_alone = [t.iterate(d) for t, d in zip(alone, dev)]
        res_mix = batch.iterate(mixed, dev)
        for o, r in zip(orcs, recs):
            o.insert(r)
            o.update()
    torch.cuda.synchronize()
    for i, (wl, _) in enumerate(ss):
        ea, em = alone[i].export(), mixed[i].export()
        assert np.array_equal(ea["keys"], em["keys"]) and np.array_equal(ea["c_old"], em["c_old"])
        assert rel_err(em["L"], ea["L"]).max() <= RTOL_F32
        compare_cells(em, orcs[i].export(), RTOL_F32, wl["name"])
        (oa, fa), (om, fm) = res_alone[i], res_mix[i]
        assert np.array_equal(fa.cpu().numpy(), fm.cpu().numpy())
        assert rel_err(om.cpu().numpy(), oa.cpu().numpy()).max() <= RTOL_F32
        st = mixed[i].stats()
        assert st["updates"] == 3 and st["dropped"] == 0


def test_batch_with_fallback_sessions_and_separate_queries(env):
    import oracle
    torch, psf = env
    ss = _sessions(4)
    tables = []
    for j, (wl, _) in enumerate(ss):
        mode = psf.PSF_INSERT_DIRECT if j == 1 else psf.PSF_INSERT_AUTO
        tables.append(psf.Table(**dict(wl["table"], insert_mode=mode)))
    orcs = [oracle.Oracle(**wl["table"]) for wl, _ in ss]
    batch = psf.Batch(8)
    for it in range(2):
        recs = [_frame(wl, sc, it) for wl, sc in ss]
        qrys = [_frame(wl, sc, 100 + it) for wl, sc in ss]  # different vertices
        res = batch.iterate(tables, [to_device(r) for r in recs], [to_device(q) for q in qrys])
        for o, r in zip(orcs, recs):
            o.insert(r)
            o.update()
    torch.cuda.synchronize()
    for i in range(len(ss)):
        compare_cells(tables[i].export(), orcs[i].export(), RTOL_F32, f"session {i}")
        w_out, w_found = orcs[i].query(qrys[i])
        out, found = res[i]
        assert np.array_equal(found.cpu().numpy(), w_found)
        assert rel_err(out.cpu().numpy(), w_out).max() <= RTOL_F32


def test_batch_graph_replay_matches_eager(env):
    """Capture one batched iteration in a graph and replay it several times,
    with eager work and synchronisation between replays; every replay must
    match the same sequence run eagerly."""
    torch, psf = env
    ss = _sessions(4)
    frames = [to_device(_frame(wl, sc, 0)) for wl, sc in ss]
    eager = [psf.Table(**wl["table"]) for wl, _ in ss]
    graphed = [psf.Table(**wl["table"]) for wl, _ in ss]
    b_eager, b_graph = psf.Batch(8), psf.Batch(8)
    outs = [torch.empty((3, int(f["px"].numel())), dtype=torch.float32, device="cuda") for f in frames]
    founds = [torch.empty(int(f["px"].numel()), dtype=torch.uint8, device="cuda") for f in frames]
    # warm up the graphed tables once eagerly (kernel attributes, lazy state)
    b_graph.iterate(graphed, frames, outs=outs, founds=founds)
    b_eager.iterate(eager, frames)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            b_graph.iterate(graphed, frames, outs=outs, founds=founds)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(4):
        g.replay()
        torch.cuda.synchronize()
        ref = b_eager.iterate(eager, frames)
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work
        torch.cuda.synchronize()
        del junk
        for i in range(len(ss)):
            ea, eg = eager[i].export(), graphed[i].export()
            assert np.array_equal(ea["keys"], eg["keys"]), (rep, i)
            assert np.array_equal(ea["c_old"], eg["c_old"]), (rep, i)
            assert rel_err(eg["L"], ea["L"]).max() <= RTOL_F32
            assert np.array_equal(ref[i][1].cpu().numpy(), founds[i].cpu().numpy())
            assert rel_err(outs[i].cpu().numpy(), ref[i][0].cpu().numpy()).max() <= RTOL_F32


def test_batch_with_footprint_sessions(env):
    """Sessions whose records carry footprints (their own level rule) mixed
    with sessions that use the camera distance: each equals the oracle."""
    import oracle
    from synth import workloads as W
    torch, psf = env
    ss = _sessions(4)
    tables = [psf.Table(**wl["table"]) for wl, _ in ss]
    orcs = [oracle.Oracle(**wl["table"]) for wl, _ in ss]
    batch = psf.Batch(8)
    for it in range(2):
        recs = []
        for j, (wl, sc) in enumerate(ss):
            r = dict(_frame(wl, sc, it))
            if j % 2 == 0:
                r["footprint"] = W.footprints(r, wl, spread=1.0)
            recs.append(r)
        res = batch.iterate(tables, [to_device(r) for r in recs])
        for o, r in zip(orcs, recs):
            o.insert(r)
            o.update()
    torch.cuda.synchronize()
    for i in range(len(ss)):
        compare_cells(tables[i].export(), orcs[i].export(), RTOL_F32, f"session {i}")
        w_out, w_found = orcs[i].query(recs[i])
        out, found = res[i]
        assert np.array_equal(found.cpu().numpy(), w_found)
        assert rel_err(out.cpu().numpy(), w_out).max() <= RTOL_F32


def test_wide_partition_session_runs_alone_with_the_same_result(env):
    """A session with 4096-slot partitions beside default ones leaves the
    shared launch (it would widen every merge block's LDS) and still gets
    the result it gets alone."""
    torch, psf = env
    ss = _sessions(3)
    cfgs = [dict(wl["table"], part_log2=12 if i == 1 else 0) for i, (wl, _) in enumerate(ss)]
    alone = [psf.Table(**c) for c in cfgs]
    mixed = [psf.Table(**c) for c in cfgs]
    batch = psf.Batch(4)
    for it in range(2):
        dev = [to_device(_frame(wl, sc, it)) for wl, sc in ss]
        res_alone = [t.iterate(d) for t, d in zip(alone, dev)]
        res_mix = batch.iterate(mixed, dev)
        torch.cuda.synchronize()
        for (oa, fa), (om, fm) in zip(res_alone, res_mix):
            assert np.array_equal(fa.cpu().numpy(), fm.cpu().numpy())
            assert rel_err(om.cpu().numpy(), oa.cpu().numpy()).max() <= RTOL_F32
    for a, m in zip(alone, mixed):
        ea, em = a.export(), m.export()
        assert np.array_equal(ea["keys"], em["keys"]) and np.array_equal(ea["c_old"], em["c_old"])


@pytest.mark.timeout(600)
def test_full_size_batched_sessions_sampled_cells(env):
    """The batched workload at its stated size: 16 uneven sessions (256x256
    to 1920x1080, 1-4 spp, 3-5 vertices, 2^18-2^23-slot tables, about 115M
    records per iteration) through one batched call per iteration, 2
    iterations.  A sample of each session's cells is tracked by the binary64
    oracle (key-sharded over the host threads): keys and counts bit-exact,
    FP32 state within 1e-5, and every record that falls in a sampled cell
    gets the oracle's lookup from the fused answer pass.  The tables take
    the launch parameters the benchmark times (the autotuner's record)."""
    import os
    import oracle
    from paper_2005_07547_amd import autotune
    from synth import workloads as W
    torch, psf = env
    wls = W.batched_sessions(16)
    scs = [W.make_scene(wl) for wl in wls]
    ns = [W.records_per_iteration(wl) for wl in wls]
    assert sum(ns) > 100_000_000
    params = autotune.best_params("batched-16")
    tables = [psf.Table(**dict(wl["table"], max_batch=n, **params)) for wl, n in zip(wls, ns)]
    threads = min(16, os.cpu_count() or 1)
    orcs = [oracle.ShardedOracle(threads, **wl["table"]) for wl in wls]
    batch = psf.Batch(16)
    rng = np.random.default_rng(31)
    samples = []
    for it in range(2):
        recs = [sc.generate(wl["gen"], it) for wl, sc in zip(wls, scs)]
        if it == 0:
            for o, r in zip(orcs, recs):
                k, _ = o.keys(r)
                s = np.unique(rng.choice(k[k != np.uint64(2 ** 64 - 1)], size=3000))
                o.set_filter(s)
                samples.append(s)
        dev = [to_device(r) for r in recs]
        res = batch.iterate(tables, dev)
        for o, r in zip(orcs, recs):
            o.insert(r)
            o.update()
        torch.cuda.synchronize()
        del dev
        print(f"iteration {it + 1}: {sum(ns)} records in 16 sessions", flush=True)
    for i in range(16):
        o = orcs[i].export()
        g = tables[i].export()
        idx = np.searchsorted(g["keys"], o["keys"])
        assert np.all(g["keys"][idx] == o["keys"]), i
        assert np.array_equal(g["c_old"][idx].astype(np.uint64), o["c_old"]), i
        assert np.array_equal(g["n_new"][idx].astype(np.uint64), o["n_new"]), i
        assert rel_err(g["L"][:, idx], o["L"]).max() <= RTOL_F32, i
        assert tables[i].stats()["dropped"] == 0, i
        # the fused answers of the last iteration at the records of sampled cells
        k, _ = orcs[i].keys(recs[i])
        pick = np.nonzero(np.isin(k, samples[i]))[0]
        assert pick.size > 0
        sub = {f: (None if v is None else v[pick]) for f, v in recs[i].items()}
        w_out, w_found = orcs[i].query(sub)
        out, found = res[i]
        assert np.array_equal(found.cpu().numpy()[pick], w_found), i
        assert rel_err(out.cpu().numpy()[:, pick], w_out).max() <= RTOL_F32, i
