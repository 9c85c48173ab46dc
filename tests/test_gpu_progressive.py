"""GPU parity of the progressive solver step (psf_progressive_step) against
the oracle in the closed furnace: samples, found cells and blended state in
lockstep over many frames, for both insert strategies."""
import numpy as np
import pytest

from tests.helpers import compare_cells, rel_err, to_device

pytestmark = pytest.mark.gpu
RTOL = 1e-5


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2005_07547_amd import psf
    psf.load()
    return torch, psf


def _dev_arrays(arrs):
    import torch
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs)


# direct and partitioned strategies; the partitioned one also on a table
# without frame accumulators (flags 16, PSF_FLAG_NO_ACCUMULATORS)
@pytest.mark.parametrize("insert_mode,flags", [(1, 0), (2, 0), (2, 16)], ids=["direct", "partitioned", "lean"])
def test_furnace_frames_match_the_oracle(env, insert_mode, flags):
    import oracle
    from synth import workloads as W
    torch, psf = env
    cfg = W.furnace_table()
    t = psf.Table(**dict(cfg, insert_mode=insert_mode, flags=flags))
    assert flags == 0 or (flags & psf.PSF_FLAG_NO_ACCUMULATORS and not t.export()["n_new"].any())
    o = oracle.Oracle(**cfg)
    for it in range(40):
        x, nx, tp, em = W.furnace_paths(2048, 2, it)
        want = oracle.progressive_step(o, x, nx, tp, em)
        got = t.progressive_step(to_device(x), to_device(nx), _dev_arrays(tp), _dev_arrays(em))
        torch.cuda.synchronize()
        assert rel_err(got.cpu().numpy(), want).max() <= RTOL, it
        if it % 10 == 9:
            compare_cells(t.export(), o.export(), RTOL, f"frame {it}")
    L = t.export()["L"]
    assert float(L.max()) > 1.0  # transport has raised cells above their emission


def test_step_without_emission_and_invalid_arguments(env):
    import oracle
    from synth import workloads as W
    torch, psf = env
    cfg = W.furnace_table()
    t = psf.Table(**cfg)
    o = oracle.Oracle(**cfg)
    for it in range(3):
        x, nx, tp, em = W.furnace_paths(256, 3, it)
        if it == 0:
            # seed the field with emission, then transport without it
            want = oracle.progressive_step(o, x, nx, tp, em)
            got = t.progressive_step(to_device(x), to_device(nx), _dev_arrays(tp), _dev_arrays(em))
        else:
            want = oracle.progressive_step(o, x, nx, tp, None)
            got = t.progressive_step(to_device(x), to_device(nx), _dev_arrays(tp), None)
        torch.cuda.synchronize()
        assert rel_err(got.cpu().numpy(), want).max() <= RTOL, it
    compare_cells(t.export(), o.export(), RTOL)
    x, nx, tp, em = W.furnace_paths(16, 1, 0)
    with pytest.raises(psf.PsfError):
        t.progressive_step(to_device(x), {k: v for k, v in to_device(nx).items() if k != "px"}, _dev_arrays(tp))


def test_radiance_minus_emission_field_frames(env):
    """Algorithm 2's field (emission of the next vertex folded into the
    step's emission argument) in lockstep with the oracle."""
    import oracle
    from synth import workloads as W
    torch, psf = env
    cfg = W.furnace_table()
    t = psf.Table(**cfg)
    o = oracle.Oracle(**cfg)
    for it in range(20):
        x, nx, tp, em = W.furnace_paths(2048, 2, it)
        le_next = tuple(a * b for a, b in zip(tp, em))
        want = oracle.progressive_step(o, x, nx, tp, le_next)
        got = t.progressive_step(to_device(x), to_device(nx), _dev_arrays(tp), _dev_arrays(le_next))
        torch.cuda.synchronize()
        assert rel_err(got.cpu().numpy(), want).max() <= RTOL, it
    compare_cells(t.export(), o.export(), RTOL)
