"""psf_iterate replayed from HIP graphs: every replay equals the same
iteration run eagerly, and the replayed table equals the oracle (Sec. 2.4's
insert + Eq. 10-11 blend + lookup, replayed as the benchmark times it)."""
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


def _workload():
    """The plain workload at a quarter of its area (640x360, 4 vertices per
    path: 921,600 records) on a 2^20-slot table."""
    from synth import workloads as W
    wl = W.plain()
    g = dict(wl["gen"], width=640, height=360)
    wl = dict(wl, gen=g, table=dict(wl["table"], log2_slots=20))
    return wl, W.make_scene(wl)


# library defaults, and the tuned plain parameters (4096-slot partitions with
# 1024-thread merge blocks, 4096-record binning tiles)
@pytest.mark.parametrize("params", [{}, {"part_log2": 12, "bin_per": 8}], ids=["default", "tuned"])
def test_iterate_graph_replay_matches_eager_and_oracle(env, params):
    import oracle
    torch, psf = env
    wl, sc = _workload()
    host = [sc.generate(wl["gen"], it) for it in range(2)]
    frames = [to_device(r) for r in host]
    n = int(frames[0]["px"].numel())
    cfg = dict(wl["table"], max_batch=n, **params)
    graphed, eager = psf.Table(**cfg), psf.Table(**cfg)
    orc = oracle.Oracle(**wl["table"])
    outs = [torch.empty((3, n), dtype=torch.float32, device="cuda") for _ in frames]
    fnds = [torch.empty(n, dtype=torch.uint8, device="cuda") for _ in frames]

    def oracle_iter(k):
        orc.insert(host[k])
        orc.update()

    # eager warm-up of both tables (lazy state, kernel attributes)
    for k in range(2):
        graphed.iterate(frames[k], out=outs[k], found=fnds[k])
        eager.iterate(frames[k])
        oracle_iter(k)
    torch.cuda.synchronize()
    graphs = []
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for k in range(2):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                graphed.iterate(frames[k], out=outs[k], found=fnds[k])
            graphs.append(g)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()

    for rep in range(6):
        k = rep % 2
        graphs[k].replay()
        torch.cuda.synchronize()
        ref_out, ref_found = eager.iterate(frames[k])
        oracle_iter(k)
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work
        torch.cuda.synchronize()
        del junk
        eg, ea = graphed.export(), eager.export()
        assert np.array_equal(eg["keys"], ea["keys"]), rep
        assert np.array_equal(eg["c_old"], ea["c_old"]), rep
        assert rel_err(eg["L"], ea["L"]).max() <= RTOL_F32, rep
        assert np.array_equal(fnds[k].cpu().numpy(), ref_found.cpu().numpy()), rep
        assert rel_err(outs[k].cpu().numpy(), ref_out.cpu().numpy()).max() <= RTOL_F32, rep

    # after eight iterations (two eager, six replayed): the oracle's cells and
    # the last replay's answers, which read the state its blend wrote
    compare_cells(graphed.export(), orc.export(), RTOL_F32, "graph replay")
    w_out, w_found = orc.query(host[1])
    assert np.array_equal(fnds[1].cpu().numpy(), w_found)
    assert rel_err(outs[1].cpu().numpy(), w_out).max() <= RTOL_F32
    del graphs
    graphed.close()
    eager.close()
