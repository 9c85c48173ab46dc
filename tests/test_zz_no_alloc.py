"""psf_export_cells_noalloc (the fixed per-GPU device array instead of a
per-call allocation) against psf_export_cells on the same tables: two calls
in a row, the second on a smaller table, then a table beyond the array's
limit."""
import ctypes

import numpy as np
import pytest

from tests.helpers import records, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_07547_amd import psf
    psf.load()
    return torch, psf


def _same(a, b):
    for k in ("keys", "n_new", "c_old"):
        assert np.array_equal(a[k], b[k]), k
    # the same kernel decodes the same slots: bit for bit
    assert np.array_equal(a["L"].view(np.uint32), b["L"].view(np.uint32))


def test_noalloc_export_equals_export_twice(env):
    from synth import workloads as W
    torch, psf = env
    wl = W.plain()
    sc = W.make_scene(wl)
    big = psf.Table(**dict(wl["table"], max_batch=W.records_per_iteration(wl)))
    for it in range(2):
        big.iterate(to_device(sc.generate(wl["gen"], it)))
    # pending samples too, so n_new is exercised
    big.insert(to_device(sc.generate(wl["gen"], 2)))
    wt = W.tiny(alpha_mode=W.ALPHA_PAPER)
    st = W.make_scene(wt)
    small = psf.Table(**wt["table"])
    for it in range(3):
        rec = dict(st.generate(wt["gen"], it))
        rec["rough"] = None
        small.iterate(to_device(rec))
    torch.cuda.synchronize()
    for t in (big, small):  # the second call has fewer cells than the first
        a = t.export()
        b = t.export(noalloc=True)
        assert len(a["keys"]) > 0
        _same(a, b)
        print(f"{len(a['keys'])} cells exported without allocation")
    assert len(small.export()["keys"]) < len(big.export()["keys"])
    big.close()
    small.close()


def test_noalloc_export_rejects_more_cells_than_its_array(env):
    torch, psf = env
    n = (1 << 20) + 4096  # distinct cells of edge 1: a 128 x 128 x 65 block
    i = np.arange(n, dtype=np.int64)
    rec = records(n, px=(i % 128).astype(np.float32) + 0.5, py=((i // 128) % 128).astype(np.float32) + 0.5,
                  pz=(i // 16384).astype(np.float32) + 0.5)
    t = psf.Table(log2_slots=22, e_min=0, kappa=0.0, max_batch=n)
    t.iterate(to_device(rec))
    torch.cuda.synchronize()
    lib = psf.load()
    cap = n
    keys = np.zeros(cap, dtype=np.uint64)
    count = ctypes.c_uint64()
    st = lib.psf_export_cells_noalloc(t.handle, keys.ctypes.data, None, None, None, cap, ctypes.byref(count),
                                      psf.current_stream())
    assert st == psf.PSF_NOT_SUPPORTED
    assert count.value == n
    assert b"1048576" in lib.psf_last_error()
    # the allocating export still handles it
    assert len(t.export()["keys"]) == n
    t.close()
