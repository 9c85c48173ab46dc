"""The seeded input generator: published Philox-4x32-10 known answers,
determinism, thread-count independence and record layout."""
import numpy as np

import synth
from synth import workloads as W


def test_philox_known_answers():
    # known-answer vectors published with the Random123 library (Salmon et
    # al., SC'11) for Philox-4x32 with 10 rounds
    kat = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, want in kat:
        assert synth.philox4x32_10(ctr, key).tolist() == list(want)


def test_deterministic_and_thread_independent():
    wl = W.tiny()
    sc = W.make_scene(wl)
    a = sc.generate(wl["gen"], 3, nthreads=1)
    b = sc.generate(wl["gen"], 3, nthreads=5)
    c = sc.generate(wl["gen"], 4, nthreads=2)
    for k in synth.FIELDS:
        assert np.array_equal(a[k], b[k])
    assert not np.array_equal(a["px"], c["px"])


def test_record_layout_plain_scene():
    wl = W.plain()
    g = dict(wl["gen"], width=160, height=90)
    sc = W.make_scene(wl)
    rec = sc.generate(g, 0)
    n = 160 * 90 * 4
    assert all(rec[k].shape == (n,) for k in synth.FIELDS)
    nrm = np.stack([rec["nx"], rec["ny"], rec["nz"]])
    wo = np.stack([rec["ox"], rec["oy"], rec["oz"]])
    np.testing.assert_allclose(np.linalg.norm(nrm, axis=0), 1.0, atol=1e-5)
    np.testing.assert_allclose(np.linalg.norm(wo, axis=0), 1.0, atol=1e-5)
    # normals face the outgoing direction
    assert np.all((nrm * wo).sum(axis=0) >= -1e-6)
    assert np.all(np.isfinite(np.stack([rec[k] for k in synth.FIELDS])))
    assert np.all(rec["r"] > 0)
    # first-depth records are camera hits: outgoing direction points at the camera
    p = np.stack([rec["px"], rec["py"], rec["pz"]])[:, : 160 * 90]
    to_cam = np.asarray(wl["gen"]["cam"], dtype=np.float32)[:, None] - p
    to_cam /= np.linalg.norm(to_cam, axis=0)
    np.testing.assert_allclose((to_cam * wo[:, : 160 * 90]).sum(axis=0), 1.0, atol=1e-4)
    glossy = (rec["rough"] < 0.3).mean()
    assert 0.1 < glossy < 0.5


def test_precision_scene_glossy_share_and_hdr():
    wl = W.precision()
    g = dict(wl["gen"], width=192, height=108)
    rec = W.make_scene(wl).generate(g, 0)
    share = (rec["rough"] < 0.3).mean()
    assert 0.35 < share < 0.65
    assert rec["r"].max() > 100.0  # lognormal(0, 2) tail
