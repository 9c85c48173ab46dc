"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Keys, cell sets and counts must match bit for bit; the FP32 approximant must
be within 1e-5 relative of the binary64 oracle.  Covers both insert
strategies, the fused iteration, every temporal mode, ragged and empty
inputs, non-finite records, table overflow, resets, and the full-size plain
workload (sampled cells).
"""
import numpy as np
import pytest

from tests.helpers import (STATE_BOUND, compare_cells, concat, golden_rows, records, rel_err, take, to_device)

pytestmark = pytest.mark.gpu

RTOL_F32 = 1e-5


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def psf(torch_cuda):
    from paper_2005_07547_amd import psf as P
    P.load()
    return P


def _oracle(cfg):
    import oracle
    return oracle.Oracle(**cfg)


def _table(psf, cfg, **extra):
    c = dict(cfg)
    c.update(extra)
    return psf.Table(**c)


def _tiny(it, alpha_mode=1):
    from synth import workloads as W
    wl = W.tiny(alpha_mode=alpha_mode)
    rec = dict(W.make_scene(wl).generate(wl["gen"], it))
    rec["rough"] = None
    return wl, rec


def _gpu_export(t):
    return t.export()


# ----------------------------------------------------------------- keys
def test_keys_golden_vectors(psf, torch_cuda):
    for row in golden_rows("key_vectors.txt"):
        kappa, e_min, max_level, thr = row[0].split()
        p = [np.float32(float(x)) for x in row[1].split()]
        nrm = [np.float32(float(x)) for x in row[2].split()]
        o = [np.float32(float(x)) for x in row[3].split()]
        rough = None if row[4] == "-" else [np.float32(float(row[4]))]
        t = psf.Table(log2_slots=8, kappa=float(kappa), e_min=int(e_min), max_level=int(max_level),
                      rough_thr=float(thr))
        rec = records(1, px=[p[0]], py=[p[1]], pz=[p[2]], nx=[nrm[0]], ny=[nrm[1]], nz=[nrm[2]],
                      ox=[o[0]], oy=[o[1]], oz=[o[2]], rough=rough)
        k = int(t.keys(to_device(rec)).cpu().numpy().view(np.uint64)[0])
        want = 0xFFFFFFFFFFFFFFFF if row[5] == "SKIP" else int(row[5], 16)
        assert k == want, (row, hex(k))


def _adversarial(n, seed):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-40, 40, size=(3, n)).astype(np.float32)
    # snap a third of the coordinates onto cell boundaries of several levels
    snap = rng.random((3, n)) < 0.33
    grid = 2.0 ** rng.integers(-7, 3, size=(3, n))
    p = np.where(snap, (np.round(p / grid) * grid).astype(np.float32), p)
    p[:, ::97] = -0.0
    p[0, 5::101] = np.float32(1e-40)   # subnormal
    p[1, 7::103] = np.float32(-1e-40)
    p[2, 9::89] = np.float32(3e38)
    v = rng.normal(size=(3, n))
    v[:, ::7] = np.round(v[:, ::7])    # axis-aligned and diagonal directions
    v = (v / np.maximum(np.abs(v).sum(axis=0), 1e-30)).astype(np.float32)
    v[:, ::211] = 0.0
    w = rng.normal(size=(3, n)).astype(np.float32)
    w[:, ::13] = np.round(w[:, ::13])
    rough = rng.uniform(0.0, 0.6, size=n).astype(np.float32)
    rough[::17] = np.float32(0.3)
    bad = rng.choice(n, size=n // 50, replace=False)
    p[0, bad[: len(bad) // 3]] = np.nan
    v[1, bad[len(bad) // 3: 2 * len(bad) // 3]] = np.inf
    rough[bad[2 * len(bad) // 3:]] = np.nan
    return records(n, px=p[0], py=p[1], pz=p[2], nx=v[0], ny=v[1], nz=v[2], ox=w[0], oy=w[1],
                   oz=w[2], rough=rough)


@pytest.mark.parametrize("kappa,e_min,max_level", [(0.0, 0, 15), (0.37, -3, 9), (2.5e-3, -6, 15),
                                                    (1e30, 2, 4)])
def test_keys_bit_exact_adversarial(psf, kappa, e_min, max_level):
    cfg = dict(cam=(0.3, -1.0, 2.0), kappa=kappa, e_min=e_min, max_level=max_level,
               normal_bins_log2=2, dir_bins_log2=3, rough_thr=0.3)
    rec = _adversarial(200003, seed=int(kappa * 7) + e_min + 100)
    want, _ = _oracle(cfg).keys(rec)
    got = _table(psf, cfg, log2_slots=8).keys(to_device(rec)).cpu().numpy().view(np.uint64)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} key mismatches, first at {bad[:5]}"


def _octahedral_edges(n, seed):
    """Normals and directions whose octahedral coordinates (the L1-normalised
    x and y, or their fold 1 - |.| for z < 0) land on or within a few ulps of
    every interior bin edge of a 4 x 4 and an 8 x 8 grid, at norms from 2^-90
    to 2^90, with zero and tiny components mixed in."""
    rng = np.random.default_rng(seed)
    edges = np.array([-0.75, -0.5, -0.25, 0.0, 0.25, 0.5, 0.75])

    def vec(size):
        # target coordinates: an edge for one (or both) of the two, free
        # otherwise, inside the octahedron |u| + |w| <= 1
        u = rng.choice(edges, size) + rng.normal(0.0, 1e-3, size) * (rng.random(size) < 0.3)
        w = rng.uniform(-1.0, 1.0, size) * (1.0 - np.abs(u))
        both = rng.random(size) < 0.3
        w = np.where(both, rng.choice(edges, size) * (1.0 - np.abs(u)), w)
        fold = rng.random(size) < 0.5
        # folded half: the edge is 1 - |w| for u, so solve |w| = 1 - edge
        uf = np.where(fold, np.sign(u + 1e-30) * (1.0 - np.abs(rng.choice(edges, size))) * rng.random(size), u)
        wf = np.where(fold, np.sign(rng.normal(size=size)) * (1.0 - np.abs(u)), w)
        uf = np.where(fold, np.sign(uf) * np.minimum(np.abs(uf), 1.0 - np.abs(wf)), uf)
        zz = 1.0 - np.abs(uf) - np.abs(wf)
        z = np.where(fold, -np.maximum(zz, 0.0), np.maximum(zz, 0.0))
        scale = np.exp2(rng.integers(-90, 91, size)).astype(np.float64) * rng.uniform(0.5, 2.0, size)
        v = (np.stack([uf, wf, z]) * scale).astype(np.float32)
        # nudge one component by up to 3 ulps either way
        k = rng.integers(-3, 4, size).astype(np.int32)
        c = rng.integers(0, 3, size)
        bits = v.view(np.int32)
        cols = np.arange(size)
        bits[c, cols] = bits[c, cols] + k * np.where(v[c, cols] == 0, 0, 1)
        v = bits.view(np.float32)
        v[0, ::53] = 0.0
        v[1, 7::59] = np.float32(-1e-44)
        v[0, 11::61] = np.float32(3e-45)
        return v

    nrm, dirs = vec(n), vec(n)
    p = rng.uniform(-4, 4, size=(3, n)).astype(np.float32)
    rough = np.full(n, 0.1, dtype=np.float32)  # glossy: the direction is binned too
    return records(n, px=p[0], py=p[1], pz=p[2], nx=nrm[0], ny=nrm[1], nz=nrm[2], ox=dirs[0],
                   oy=dirs[1], oz=dirs[2], rough=rough)


@pytest.mark.parametrize("nb,db", [(2, 3), (1, 2), (2, 1)])
def test_keys_bit_exact_octahedral_bin_edges(psf, nb, db):
    cfg = dict(cam=(0.0, 0.0, 0.0), kappa=0.0, e_min=-2, max_level=15, normal_bins_log2=nb,
               dir_bins_log2=db, rough_thr=0.3)
    rec = _octahedral_edges(300007, seed=31 + nb * 7 + db)
    want, _ = _oracle(cfg).keys(rec)
    got = _table(psf, cfg, log2_slots=8).keys(to_device(rec)).cpu().numpy().view(np.uint64)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} key mismatches, first at {bad[:5]}"
    # the batch really sits on the edges: a large share of the normals'
    # unfolded coordinates lie within B 2^-18 of an integer once scaled
    v = np.stack([rec["nx"], rec["ny"], rec["nz"]]).astype(np.float64)
    l1 = np.abs(v).sum(axis=0)
    t = (v[0] / np.where(l1 > 0, l1, 1.0) * 0.5 + 0.5) * 2.0 ** nb
    assert (np.abs(t - np.rint(t)) <= 2.0 ** (nb - 18)).mean() > 0.1


def test_keys_bit_exact_workloads(psf):
    from synth import workloads as W
    for wl in (W.tiny(), W.plain()):
        rec = W.make_scene(wl).generate(wl["gen"], 5)
        if wl["diffuse_only"]:
            rec = dict(rec)
            rec["rough"] = None
        want, _ = _oracle(wl["table"]).keys(rec)
        got = _table(psf, wl["table"]).keys(to_device(rec)).cpu().numpy().view(np.uint64)
        assert np.array_equal(got, want), wl["name"]


# ----------------------------------------------------------------- whole iterations
MODES = [("direct", 1, False), ("partitioned", 2, False), ("fused", 2, True), ("fused-auto", 0, True)]


@pytest.mark.parametrize("alpha_mode", [0, 1, 2])
@pytest.mark.parametrize("name,insert_mode,fused", MODES)
def test_tiny_workload_all_iterations(psf, torch_cuda, name, insert_mode, fused, alpha_mode):
    wl, _ = _tiny(0, alpha_mode)
    orc = _oracle(wl["table"])
    t = _table(psf, wl["table"], insert_mode=insert_mode)
    for it in range(wl["iterations"]):
        _, rec = _tiny(it, alpha_mode)
        d = to_device(rec)
        orc.insert(rec)
        orc.update()
        if fused:
            out, found = t.iterate(d)
        else:
            t.insert(d)
            t.update()
            out, found = t.query(d)
        torch_cuda.cuda.synchronize()
        w_out, w_found = orc.query(rec)
        assert np.array_equal(found.cpu().numpy(), w_found), (name, it)
        assert rel_err(out.cpu().numpy(), w_out).max() <= RTOL_F32, (name, it)
    compare_cells(t.export(), orc.export(), RTOL_F32, name)
    st = t.stats()
    assert st["dropped"] == 0 and st["skipped"] == 0
    assert st["updates"] == wl["iterations"]


@pytest.mark.parametrize("name,insert_mode,fused", MODES[:3])
def test_plain_workload_full_parity_first_iterations(psf, torch_cuda, name, insert_mode, fused):
    from synth import workloads as W
    wl = W.plain()
    sc = W.make_scene(wl)
    orc = _oracle(wl["table"])
    t = _table(psf, wl["table"], insert_mode=insert_mode)
    for it in range(2):
        rec = sc.generate(wl["gen"], it)
        d = to_device(rec)
        orc.insert(rec)
        orc.update()
        if fused:
            out, found = t.iterate(d)
        else:
            t.insert(d)
            t.update()
            out, found = t.query(d)
        torch_cuda.cuda.synchronize()
    worst = compare_cells(t.export(), orc.export(), RTOL_F32, name)
    w_out, w_found = orc.query(rec)
    assert np.array_equal(found.cpu().numpy(), w_found)
    assert rel_err(out.cpu().numpy(), w_out).max() <= RTOL_F32
    print(f"{name}: worst cell relative error {worst:.2e}")


def test_plain_workload_sampled_cells_many_iterations(psf, torch_cuda):
    """Full-size plain workload in the launch configuration the benchmark
    times (fused partitioned iteration, 2^22 slots); the oracle tracks a
    sample of cells over every iteration."""
    from paper_2005_07547_amd import autotune
    from synth import workloads as W
    wl = W.plain()
    iters = 8
    sc = W.make_scene(wl)
    orc = _oracle(wl["table"])
    t = _table(psf, wl["table"], **autotune.best_params(wl["name"]))
    first = sc.generate(wl["gen"], 0)
    keys0, _ = orc.keys(first)
    rng = np.random.default_rng(1)
    sample = np.unique(rng.choice(keys0[keys0 != np.uint64(2**64 - 1)], size=3000))
    orc.set_filter(sample)
    submitted = 0
    for it in range(iters):
        rec = first if it == 0 else sc.generate(wl["gen"], it)
        orc.insert(rec)
        orc.update()
        t.iterate(to_device(rec))
        submitted += len(rec["px"])
    torch_cuda.cuda.synchronize()
    g = t.export()
    o = orc.export()
    idx = np.searchsorted(g["keys"], o["keys"])
    assert np.all(g["keys"][idx] == o["keys"])
    sub = {k: (v[:, idx] if v.ndim == 2 else v[idx]) for k, v in g.items()}
    compare_cells(sub, o, RTOL_F32, "sampled")
    st = t.stats()
    assert st["dropped"] == 0 and st["skipped"] == 0
    assert st["submitted"] == submitted
    assert st["occupied"] <= t.n_slots * 0.6


# ----------------------------------------------------------------- edge cases
@pytest.mark.parametrize("insert_mode", [1, 2])
@pytest.mark.parametrize("n", [1, 63, 65, 1023, 8191, 8193, 100003])
def test_ragged_sizes(psf, torch_cuda, insert_mode, n):
    wl, rec = _tiny(3, 0)
    rec = take(rec, np.arange(n) % len(rec["px"]))
    orc = _oracle(wl["table"])
    t = _table(psf, wl["table"], insert_mode=insert_mode)
    orc.insert(rec)
    orc.update()
    t.insert(to_device(rec))
    t.update()
    compare_cells(t.export(), orc.export(), RTOL_F32, f"n={n}")


def test_empty_inputs_are_noops(psf, torch_cuda):
    wl, rec = _tiny(0, 0)
    t = _table(psf, wl["table"])
    d = to_device(rec)
    t.insert(d, n=0)
    out, found = t.query(d, n=0)
    t.update()
    st = t.stats()
    assert st["occupied"] == 0 and st["touched_last"] == 0


@pytest.mark.parametrize("insert_mode", [1, 2])
def test_nonfinite_records_are_skipped(psf, torch_cuda, insert_mode):
    wl, rec = _tiny(1, 0)
    n = len(rec["px"])
    rec["px"][::101] = np.nan
    rec["nz"][5::103] = np.inf
    rec["g"][7::107] = -np.inf
    orc = _oracle(wl["table"])
    orc.insert(rec)
    orc.update()
    t = _table(psf, wl["table"], insert_mode=insert_mode)
    t.insert(to_device(rec))
    t.update()
    compare_cells(t.export(), orc.export(), RTOL_F32)
    assert t.stats()["skipped"] == orc.counters()["skipped"] > 0
    out, found = t.query(to_device(rec))
    w_out, w_found = orc.query(rec)
    assert np.array_equal(found.cpu().numpy(), w_found)


@pytest.mark.parametrize("insert_mode", [1, 2])
def test_overflowing_table_conserves_counts(psf, torch_cuda, insert_mode):
    # 2^4 slots and many more cells: every record is either in a cell or
    # counted as dropped, and the cells that made it match the oracle
    wl, rec = _tiny(2, 0)
    cfg = dict(wl["table"], log2_slots=4, max_probe=16)
    t = _table(psf, cfg, insert_mode=insert_mode)
    t.insert(to_device(rec))
    ex = t.export()
    st = t.stats()
    n = len(rec["px"])
    assert len(ex["keys"]) == 16
    assert st["dropped"] > 0
    assert int(ex["n_new"].sum()) + st["dropped"] + st["skipped"] == n
    orc = _oracle(wl["table"])
    orc.insert(rec)
    o = orc.export()
    idx = np.searchsorted(o["keys"], ex["keys"])
    assert np.array_equal(o["keys"][idx], ex["keys"])
    assert np.array_equal(o["n_new"][idx], ex["n_new"].astype(np.uint64))


@pytest.mark.parametrize("insert_mode", [1, 2])
def test_max_probe_one(psf, torch_cuda, insert_mode):
    wl, rec = _tiny(4, 0)
    cfg = dict(wl["table"], log2_slots=12, max_probe=1)
    t = _table(psf, cfg, insert_mode=insert_mode)
    t.insert(to_device(rec))
    st = t.stats()
    ex = t.export()
    assert int(ex["n_new"].sum()) + st["dropped"] == len(rec["px"])
    assert st["dropped"] > 0


def test_coordinate_overflow_counted(psf, torch_cuda):
    cfg = dict(kappa=0.0, e_min=-10, log2_slots=10)
    rec = records(4, px=[0.0, 40.0, -40.0, 31.9], r=[1, 2, 3, 4])
    orc = _oracle(cfg)
    orc.insert(rec)
    t = _table(psf, cfg)
    t.insert(to_device(rec))
    assert t.stats()["coord_overflow"] == orc.counters()["coord_overflow"] == 2


@pytest.mark.parametrize("insert_mode", [1, 2])
def test_reset_semantics(psf, torch_cuda, insert_mode):
    wl, rec = _tiny(5, 0)
    orc = _oracle(wl["table"])
    t = _table(psf, wl["table"], insert_mode=insert_mode)
    d = to_device(rec)
    out, found = t.query(d)
    assert int(found.sum()) == 0  # nothing blended yet
    for what in (psf.PSF_RESET_COUNTERS, psf.PSF_RESET_CLEAR):
        for _ in range(2):
            orc.insert(rec)
            orc.update()
            t.insert(d)
            t.update()
        orc.reset(what)
        t.reset(what)
        out, found = t.query(d)
        w_out, w_found = orc.query(rec)
        assert np.array_equal(found.cpu().numpy(), w_found)
        orc.insert(rec)
        orc.update()
        t.insert(d)
        t.update()
        compare_cells(t.export(), orc.export(), RTOL_F32, f"reset {what}")


def test_multiple_inserts_before_update(psf, torch_cuda):
    wl, rec = _tiny(6, 0)
    for mode in (1, 2):
        orc = _oracle(wl["table"])
        orc.insert(rec)
        orc.update()
        t = _table(psf, wl["table"], insert_mode=mode)
        parts = np.array_split(np.arange(len(rec["px"])), 3)
        for p in parts:
            t.insert(to_device(take(rec, p)))
        t.update()
        compare_cells(t.export(), orc.export(), RTOL_F32, f"mode {mode}")


def test_insert_larger_than_batch_capacity(psf, torch_cuda):
    wl, rec = _tiny(7, 0)
    big = concat([rec] * 5)
    orc = _oracle(wl["table"])
    orc.insert(big)
    orc.update()
    t = _table(psf, wl["table"], insert_mode=2, max_batch=10000)
    out, found = t.iterate(to_device(big))
    compare_cells(t.export(), orc.export(), RTOL_F32)


def test_invalid_arguments(psf, torch_cuda):
    import ctypes
    lib = psf.load()
    bad = psf.make_config(log2_slots=3)
    h = ctypes.c_void_p()
    assert lib.psf_create_table(ctypes.byref(bad), None, 0, None, ctypes.byref(h)) == psf.PSF_INVALID_ARGUMENT
    assert b"log2_slots" in lib.psf_last_error()
    good = psf.make_config(log2_slots=10)
    need = lib.psf_table_bytes(ctypes.byref(good))
    buf = torch_cuda.empty(need, dtype=torch_cuda.uint8, device="cuda")
    assert lib.psf_create_table(ctypes.byref(good), ctypes.c_void_p(buf.data_ptr()), need - 1, None,
                                ctypes.byref(h)) == psf.PSF_BUFFER_TOO_SMALL
    t = psf.Table(log2_slots=10)
    empty = psf.psf_records()
    assert lib.psf_insert_samples(t.handle, ctypes.byref(empty), 10, None) == psf.PSF_INVALID_ARGUMENT
    assert lib.psf_insert_samples(t.handle, None, 10, None) == psf.PSF_INVALID_ARGUMENT
    assert lib.psf_insert_samples(t.handle, None, 0, None) == psf.PSF_OK
    assert lib.psf_reset(t.handle, 64, None) == psf.PSF_INVALID_ARGUMENT
    for kw in (dict(alpha_mode=1, alpha=0.0), dict(t_max=0.5), dict(kappa=-1.0), dict(max_level=16),
               dict(dir_bins_log2=4), dict(state_dtype=5), dict(part_log2=5), dict(max_probe=0)):
        c = psf.make_config(log2_slots=10, **kw)
        assert lib.psf_table_bytes(ctypes.byref(c)) == 0, kw


TUNABLE = [(b, p, 0) for b in (8, 12, 16) for p in (8, 10, 12)] + [(8, 11, 4), (16, 8, 4), (12, 12, 4)]


@pytest.mark.parametrize("bin_per,part_log2,flags", TUNABLE)
def test_tunable_launch_parameters_keep_parity(psf, torch_cuda, bin_per, part_log2, flags):
    """Every launch configuration the autotuner may pick gives the oracle's
    result (two fused iterations of the plain scene at reduced resolution)."""
    from synth import workloads as W
    wl = W.plain()
    g = dict(wl["gen"], width=320, height=180)
    sc = W.make_scene(wl)
    # 2^20 slots keep every partition far from full even at 256 slots each
    cfg = dict(wl["table"], log2_slots=20)
    orc = _oracle(cfg)
    t = _table(psf, cfg, insert_mode=2, bin_per=bin_per, part_log2=part_log2, flags=flags)
    for it in range(2):
        rec = sc.generate(g, it)
        orc.insert(rec)
        orc.update()
        out, found = t.iterate(to_device(rec))
    torch_cuda.cuda.synchronize()
    assert t.stats()["dropped"] == 0
    compare_cells(t.export(), orc.export(), RTOL_F32, f"bin_per={bin_per} part_log2={part_log2} flags={flags}")
    w_out, w_found = orc.query(rec)
    assert np.array_equal(found.cpu().numpy(), w_found)
    assert rel_err(out.cpu().numpy(), w_out).max() <= RTOL_F32


@pytest.mark.parametrize("part_log2,extra", [(11, {}), (12, {}), (11, {"flags": 8}), (11, {"weighted": 1})])
def test_separate_insert_and_update_wide_merge_blocks(psf, torch_cuda, part_log2, extra):
    """The unfused merge (separate insert and update calls) at the partition
    widths whose LDS leaves one block per CU (4096 slots; 2048 with the
    variance's or the weights' further sum), where the merge runs 1024
    threads per block; against the oracle."""
    from synth import workloads as W
    wl = W.plain()
    g = dict(wl["gen"], width=320, height=180)
    sc = W.make_scene(wl)
    cfg = dict(wl["table"], log2_slots=20)
    orc = _oracle(dict(cfg, **({"weighted": 1} if extra.get("weighted") else {})))
    t = _table(psf, cfg, insert_mode=2, part_log2=part_log2, **extra)
    for it in range(2):
        rec = sc.generate(g, it)
        orc.insert(rec)
        orc.update()
        d = to_device(rec)
        t.insert(d)
        t.update()
    out, found = t.query(d)
    torch_cuda.cuda.synchronize()
    assert t.stats()["dropped"] == 0
    ge, oe = t.export(), orc.export()
    assert np.array_equal(ge["keys"], oe["keys"])
    if extra.get("weighted"):
        # binary32 weight sums against binary64 ones
        assert rel_err(ge["c_old"], oe["c_old"]).max() <= RTOL_F32
    else:
        assert np.array_equal(ge["c_old"].astype(np.uint64), oe["c_old"])
    assert rel_err(ge["L"], oe["L"]).max() <= RTOL_F32
    w_out, w_found = orc.query(rec)
    assert np.array_equal(found.cpu().numpy(), w_found)
    assert rel_err(out.cpu().numpy(), w_out).max() <= RTOL_F32


# ----------------------------------------------------------------- fused query
def _fused_cases():
    # (label, config overrides, record transform)
    def ragged(n):
        return lambda rec: take(rec, np.arange(n) % len(rec["px"]))

    def nonfinite(rec):
        rec = {k: (None if v is None else v.copy()) for k, v in rec.items()}
        rec["px"][::101] = np.nan
        rec["g"][7::107] = -np.inf
        return rec

    same = lambda rec: rec  # noqa: E731
    return [
        ("tiny", {}, same),
        ("n=1", {}, ragged(1)),
        ("n=65", {}, ragged(65)),
        ("n=8193", {}, ragged(8193)),
        ("nonfinite", {}, nonfinite),
        ("overflow", dict(log2_slots=8, max_probe=16), same),
        ("max_probe=1", dict(log2_slots=12, max_probe=1), same),
        # 16 partitions of 256 slots and 25 tiles: every wave of a merge block
        # holds many batches, so later batches find their slots again
        ("dense", dict(log2_slots=12, part_log2=8), ragged(100003)),
        ("dense-transposed", dict(log2_slots=12, part_log2=8, flags=4), ragged(100003)),
        ("transposed", dict(flags=4), same),
        ("f16", dict(state_dtype=1), same),
        ("bf16", dict(state_dtype=2), same),
        ("f16-residual", dict(state_dtype=3), same),
        ("bf16-residual", dict(state_dtype=4), same),
    ]


@pytest.mark.parametrize("case", _fused_cases(), ids=lambda c: c[0])
def test_fused_query_equals_lookup(psf, torch_cuda, case):
    """psf_iterate with the records as queries answers them in the merge
    pass; the answers must be exactly what a lookup of the same table state
    returns, and (where no key was dropped) what the oracle returns."""
    label, over, transform = case
    wl, _ = _tiny(0, 0)
    cfg = dict(wl["table"], **over)
    t = _table(psf, cfg, insert_mode=2)
    orc = _oracle(cfg)
    for it in range(3):
        _, rec = _tiny(it, 0)
        rec = transform(rec)
        d = to_device(rec)
        out, found = t.iterate(d)
        out2, found2 = t.query(d)
        torch_cuda.cuda.synchronize()
        a, b = out.cpu().numpy(), out2.cpu().numpy()
        assert np.array_equal(found.cpu().numpy(), found2.cpu().numpy()), (label, it)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (label, it)
        orc.insert(rec)
        orc.update()
    st = t.stats()
    if st["dropped"] == 0:
        w_out, w_found = orc.query(rec)
        assert np.array_equal(found.cpu().numpy(), w_found), label
        tol = STATE_BOUND[cfg.get("state_dtype", 0)]
        assert rel_err(out.cpu().numpy(), w_out).max() <= tol, label
    else:
        assert label in ("overflow", "max_probe=1", "dense", "dense-transposed"), (label, st["dropped"])


# ----------------------------------------------------------------- footprint levels
def test_footprint_keys_bit_exact(psf, torch_cuda):
    import struct
    rows = golden_rows("footprint_levels.txt")
    rng = np.random.default_rng(12)
    fp = np.concatenate([
        np.array([struct.unpack(">f", bytes.fromhex(r[2]))[0] for r in rows], dtype=np.float32),
        np.exp2(rng.uniform(-20, 20, 5000)).astype(np.float32),
        np.exp2(np.arange(-20, 21)).astype(np.float32),
        np.nextafter(np.exp2(np.arange(-20, 21)).astype(np.float32), np.float32(0)),
        np.array([0.0, -0.0, -1.0, np.inf, -np.inf, np.nan, 1e-45], dtype=np.float32)])
    n = len(fp)
    rec = records(n, px=rng.uniform(-3, 3, n), py=rng.uniform(-3, 3, n), pz=rng.uniform(-3, 3, n),
                  footprint=fp)
    for e_min, max_level in ((-5, 15), (0, 3), (-9, 7)):
        cfg = dict(kappa=0.5, cam=(0.0, 0.0, -4.0), e_min=e_min, max_level=max_level, log2_slots=12)
        want, _ = _oracle(cfg).keys(rec)
        got = _table(psf, cfg).keys(to_device(rec)).cpu().numpy().view(np.uint64)
        assert np.array_equal(got, want), (e_min, max_level)


@pytest.mark.parametrize("name,insert_mode,fused", MODES[:3])
def test_footprint_levels_whole_iterations(psf, torch_cuda, name, insert_mode, fused):
    from synth import workloads as W
    wl = W.tiny(alpha_mode=0)
    sc = W.make_scene(wl)
    orc = _oracle(wl["table"])
    t = _table(psf, wl["table"], insert_mode=insert_mode)
    for it in range(4):
        rec = dict(sc.generate(wl["gen"], it))
        rec["rough"] = None
        rec["footprint"] = W.footprints(rec, wl, spread=1.5)
        d = to_device(rec)
        orc.insert(rec)
        orc.update()
        if fused:
            out, found = t.iterate(d)
        else:
            t.insert(d)
            t.update()
            out, found = t.query(d)
        torch_cuda.cuda.synchronize()
        w_out, w_found = orc.query(rec)
        assert np.array_equal(found.cpu().numpy(), w_found), (name, it)
        assert rel_err(out.cpu().numpy(), w_out).max() <= RTOL_F32, (name, it)
    compare_cells(t.export(), orc.export(), RTOL_F32, name)
    levels = (t.export()["keys"] >> np.uint64(59)) & np.uint64(15)
    assert len(np.unique(levels)) > 1


# ----------------------------------------------------------------- local counter reset
@pytest.mark.parametrize("insert_mode", [1, 2])
def test_local_counter_reset(psf, torch_cuda, insert_mode):
    from synth import workloads as W
    wl = W.tiny(alpha_mode=0)
    sc = W.make_scene(wl)
    orc = _oracle(wl["table"])
    t = _table(psf, wl["table"], insert_mode=insert_mode)
    regions = [((0.2, -0.1, 0.3), (0.6, 0.45, 0.9)), ((-5, -5, -5), (0.5, 5, 5)), ((0.25, 0.25, 0.25), (0.25, 0.25, 0.25))]
    for it in range(5):
        rec = dict(sc.generate(wl["gen"], it))
        rec["rough"] = None
        d = to_device(rec)
        orc.insert(rec)
        orc.update()
        out, found = t.iterate(d)
        if it < len(regions):
            before = int(found.sum())
            lo, hi = regions[it]
            orc.reset_region(lo, hi)
            t.reset_region(lo, hi)
            out, found = t.query(d)
            if it < 2:  # these regions hold cells: some vertices lose their answer
                assert 0 < int(found.sum()) < before, it
        torch_cuda.cuda.synchronize()
        w_out, w_found = orc.query(rec)
        assert np.array_equal(found.cpu().numpy(), w_found), it
        assert rel_err(out.cpu().numpy(), w_out).max() <= RTOL_F32, it
        compare_cells(t.export(), orc.export(), RTOL_F32, f"after frame {it}")
    with pytest.raises(psf.PsfError):
        t.reset_region((1, 0, 0), (0, 1, 1))
    with pytest.raises(psf.PsfError):
        t.reset_region((0, 0, 0), (float("nan"), 1, 1))


def test_multi_level_lookup(psf, torch_cuda):
    """Cells learned at coarse levels (footprints x 4), queried from finer
    levels (footprints / 4) with up to 3 levels of climb: the answering level
    bit for bit, the values within the FP32 tolerance."""
    from synth import workloads as W
    wl = W.tiny(alpha_mode=0)
    sc = W.make_scene(wl)
    orc = _oracle(wl["table"])
    t = _table(psf, wl["table"])
    for it in range(3):
        rec = dict(sc.generate(wl["gen"], it))
        rec["rough"] = None
        fp = W.footprints(rec, wl, spread=1.0)
        coarse = dict(rec, footprint=fp * np.float32(4.0))
        orc.insert(coarse)
        orc.update()
        t.iterate(to_device(coarse))
    q = dict(rec, footprint=fp * np.float32(0.25))
    for up in (0, 1, 3):
        out, level = t.query_levels(to_device(q), up)
        torch_cuda.cuda.synchronize()
        w_out, w_level = orc.query_levels(q, up)
        assert np.array_equal(level.cpu().numpy(), w_level), up
        assert rel_err(out.cpu().numpy(), w_out).max() <= RTOL_F32, up
    assert int((w_level >= 2).sum()) > 0 and int((w_level == 0).sum()) < len(w_level)


@pytest.mark.parametrize("log2_slots,part_log2", [(26, 0), (25, 11)])
def test_more_than_8192_partitions_stay_partitioned(psf, torch_cuda, log2_slots, part_log2):
    """Tables of 16384 partitions (2^26 slots by default, 2^25 of 2048) stay
    on the partitioned strategy (the binning pass's histogram then takes 64
    KB of LDS); against the oracle on the plain scene at reduced resolution,
    with the fused answers."""
    from synth import workloads as W
    wl = W.plain()
    g = dict(wl["gen"], width=320, height=180)
    sc = W.make_scene(wl)
    cfg = dict(wl["table"], log2_slots=log2_slots)
    orc = _oracle(cfg)
    t = psf.Table(**cfg, part_log2=part_log2, flags=psf.PSF_FLAG_TIMING)
    for it in range(2):
        rec = sc.generate(g, it)
        out, found = t.iterate(to_device(rec))
        orc.insert(rec)
        orc.update()
    torch_cuda.cuda.synchronize()
    w_out, w_found = orc.query(rec)
    assert np.array_equal(found.cpu().numpy(), w_found)
    assert rel_err(out.cpu().numpy(), w_out).max() <= RTOL_F32
    assert {"bin", "merge_blend"} <= set(t.kernel_times())
    assert t.stats()["dropped"] == 0
    compare_cells(t.export(), orc.export(), RTOL_F32, f"2^{log2_slots} slots")
    t.close()


def test_large_table_default_partitions_stay_partitioned(psf, torch_cuda):
    """A 2^25-slot table with the default partition width takes 4096-slot
    partitions (8192 of them), so the automatic strategy stays partitioned;
    results match the oracle."""
    wl, _ = _tiny(0)
    cfg = dict(wl["table"], log2_slots=25)
    orc = _oracle(cfg)
    t = psf.Table(**cfg, flags=psf.PSF_FLAG_TIMING)
    for it in range(3):
        _, rec = _tiny(it)
        out, found = t.iterate(to_device(rec))
        orc.insert(rec)
        orc.update()
        torch_cuda.cuda.synchronize()
        w_out, w_found = orc.query(rec)
        assert np.array_equal(found.cpu().numpy(), w_found), it
        assert rel_err(out.cpu().numpy(), w_out).max() <= RTOL_F32, it
    assert {"bin", "merge_blend"} <= set(t.kernel_times())
    compare_cells(t.export(), orc.export(), RTOL_F32, "2^25 slots")
