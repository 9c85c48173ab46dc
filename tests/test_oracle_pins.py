"""Pins of the CPU oracle against facts fixed outside it.

Each test checks the oracle against something it does not compute itself:
hand-derived vectors (tests/golden), closed forms of the temporal blend's
limiting cases named in Sec. 2.4, exact identities of the per-cell means of
Eq. 5-6, brute-force grouping, and invariants (conservation, order
invariance, convexity).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import ALPHA_CONST, ALPHA_LINEAR, ALPHA_PAPER, RESET_CLEAR, RESET_COUNTERS
from synth import workloads as W
from tests.helpers import concat, golden_rows, records, take


def _cfg(**kw):
    c = dict(cam=(0.0, 0.0, 0.0), kappa=0.0, e_min=0, max_level=15, normal_bins_log2=2,
             dir_bins_log2=3, rough_thr=0.3, alpha_mode=ALPHA_PAPER, alpha=0.2, t_max=5.0)
    c.update(kw)
    return c


def _f(s):
    return np.float32(float(s))


# ----------------------------------------------------------------- key function
def test_key_vectors_golden():
    for row in golden_rows("key_vectors.txt"):
        kappa, e_min, max_level, thr = row[0].split()
        p = [_f(x) for x in row[1].split()]
        n = [_f(x) for x in row[2].split()]
        o = [_f(x) for x in row[3].split()]
        rough = None if row[4] == "-" else [_f(row[4])]
        orc = oracle.Oracle(**_cfg(kappa=float(kappa), e_min=int(e_min), max_level=int(max_level),
                                   rough_thr=float(thr)))
        rec = records(1, px=[p[0]], py=[p[1]], pz=[p[2]], nx=[n[0]], ny=[n[1]], nz=[n[2]],
                      ox=[o[0]], oy=[o[1]], oz=[o[2]], rough=rough)
        keys, _ = orc.keys(rec)
        want = 0xFFFFFFFFFFFFFFFF if row[5] == "SKIP" else int(row[5], 16)
        assert int(keys[0]) == want, (row, hex(int(keys[0])))


def test_octahedral_axes_golden():
    rows = golden_rows("octahedral_axes.txt")
    orc = oracle.Oracle(**_cfg())
    v = np.array([[float(x) for x in r[0].split()[:3]] for r in rows], dtype=np.float32)
    rec = records(len(rows), nx=v[:, 0], ny=v[:, 1], nz=v[:, 2])
    keys, _ = orc.keys(rec)
    for r, k in zip(rows, keys):
        iu, iw = (int(x) for x in r[0].split()[3:])
        assert (int(k) >> 48) & 0xF == iu * 4 + iw


def test_axis_bins_distinct():
    # the six axis directions land in six distinct bins for the normal grid
    # (B = 4) and for the direction grid (B = 8)
    axes = np.array([[0, 0, 1], [0, 0, -1], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0]],
                    dtype=np.float32)
    orc = oracle.Oracle(**_cfg(normal_bins_log2=2, dir_bins_log2=3))
    rec = records(6, nx=axes[:, 0], ny=axes[:, 1], nz=axes[:, 2], ox=axes[:, 0],
                  oy=axes[:, 1], oz=axes[:, 2], rough=np.full(6, 0.1, np.float32))
    keys, _ = orc.keys(rec)
    for shift, nbits in ((48, 4), (52, 6)):
        bins = {(int(k) >> shift) & ((1 << nbits) - 1) for k in keys}
        assert len(bins) == 6


def test_grid_coordinates_match_exact_float64_floor():
    # power-of-two scaling and floor are exact, so a float64 re-derivation of
    # floor(p * 2^-(e_min + level)) must agree everywhere (fixed level)
    rng = np.random.default_rng(7)
    n = 20000
    p = rng.uniform(-300, 300, size=(3, n)).astype(np.float32)
    for e_min in (-6, -2, 0, 3):
        orc = oracle.Oracle(**_cfg(e_min=e_min))
        rec = records(n, px=p[0], py=p[1], pz=p[2])
        keys, ovf = orc.keys(rec)
        assert not ovf.any()
        for ax, sh in ((0, 0), (1, 16), (2, 32)):
            want = np.floor(p[ax].astype(np.float64) * 2.0 ** (-e_min)).astype(np.int64) & 0xFFFF
            got = (keys >> np.uint64(sh)).astype(np.int64) & 0xFFFF
            assert np.array_equal(got, want)


def test_levels_match_float64_log_away_from_boundaries():
    # level = floor(0.5 * log2(kappa * d^2)) clamped; the float64 value of
    # 0.5*log2(.) must agree except within a hair of an integer
    rng = np.random.default_rng(8)
    n = 20000
    p = rng.uniform(-50, 50, size=(3, n)).astype(np.float32)
    cam = (1.5, -2.0, 0.25)
    kappa = 0.37
    orc = oracle.Oracle(**_cfg(cam=cam, kappa=kappa, max_level=9))
    keys, _ = orc.keys(records(n, px=p[0], py=p[1], pz=p[2]))
    lvl = (keys >> np.uint64(59)).astype(np.int64)
    d2 = sum((p[i].astype(np.float64) - cam[i]) ** 2 for i in range(3))
    h = 0.5 * np.log2(np.float64(np.float32(kappa)) * d2)
    want = np.clip(np.floor(h), 0, 9).astype(np.int64)
    ok = np.abs(h - np.round(h)) > 1e-5
    assert ok.mean() > 0.99
    assert np.array_equal(lvl[ok], want[ok])


def test_octahedral_bins_match_float64_away_from_boundaries():
    rng = np.random.default_rng(9)
    n = 20000
    v = rng.normal(size=(3, n))
    v /= np.linalg.norm(v, axis=0)
    v = v.astype(np.float32)
    orc = oracle.Oracle(**_cfg(dir_bins_log2=3))
    keys, _ = orc.keys(records(n, nx=v[0], ny=v[1], nz=v[2], ox=v[0], oy=v[1], oz=v[2],
                               rough=np.zeros(n, np.float32)))
    x, y, z = (v[i].astype(np.float64) for i in range(3))
    a = np.abs(x) + np.abs(y) + np.abs(z)
    u, w = x / a, y / a
    neg = z < 0
    su = np.where(u >= 0, 1.0, -1.0)
    sw = np.where(w >= 0, 1.0, -1.0)
    u2 = np.where(neg, (1 - np.abs(w)) * su, u)
    w2 = np.where(neg, (1 - np.abs(u)) * sw, w)
    for b, sh, nb in ((4, 48, 4), (8, 52, 6)):
        fu, fw = (u2 * 0.5 + 0.5) * b, (w2 * 0.5 + 0.5) * b
        iu = np.clip(np.floor(fu), 0, b - 1)
        iw = np.clip(np.floor(fw), 0, b - 1)
        want = (iu * b + iw).astype(np.int64)
        got = (keys >> np.uint64(sh)).astype(np.int64) & ((1 << nb) - 1)
        far = (np.abs(fu - np.round(fu)) > 1e-4) & (np.abs(fw - np.round(fw)) > 1e-4)
        assert far.mean() > 0.99
        assert np.array_equal(got[far], want[far])


def test_same_cell_same_key_neighbour_cell_differs():
    # points spread inside one cell of edge 2^e_min share a key; stepping one
    # edge along any axis changes it
    rng = np.random.default_rng(10)
    e_min = -3
    edge = 2.0 ** e_min
    base = np.array([5, -7, 11], dtype=np.float64) * edge
    n = 500
    off = rng.uniform(0, edge * 0.999, size=(3, n))
    p = (base[:, None] + off).astype(np.float32)
    orc = oracle.Oracle(**_cfg(e_min=e_min))
    keys, _ = orc.keys(records(n, px=p[0], py=p[1], pz=p[2]))
    assert len(set(keys.tolist())) == 1
    for ax in range(3):
        q = p.copy()
        q[ax] += np.float32(edge)
        k2, _ = orc.keys(records(n, px=q[0], py=q[1], pz=q[2]))
        assert set(k2.tolist()).isdisjoint(set(keys.tolist()))


# ----------------------------------------------------------------- Eq. 5-6
def _cell_records(centers, counts, values, edge_log2=0, seed=0):
    """Records placed strictly inside known unit cells (edge 2^edge_log2), so
    the grouping is known without evaluating the key function."""
    rng = np.random.default_rng(seed)
    parts = []
    for c, n, v in zip(centers, counts, values):
        edge = 2.0 ** edge_log2
        lo = np.asarray(c, dtype=np.float64) * edge
        p = (lo[:, None] + rng.uniform(0.05, 0.95, size=(3, n)) * edge).astype(np.float32)
        vv = np.asarray(v, dtype=np.float32)
        parts.append(records(n, px=p[0], py=p[1], pz=p[2], r=vv[0], g=vv[1], b=vv[2]))
    return concat(parts)


def test_grouping_by_construction():
    centers = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 5, -3), (100, -100, 7)]
    counts = [10, 1, 7, 3, 25]
    rng = np.random.default_rng(3)
    values = [rng.uniform(0.1, 5, size=(3, n)).astype(np.float32) for n in counts]
    rec = _cell_records(centers, counts, values)
    orc = oracle.Oracle(**_cfg())
    orc.insert(rec)
    ex = orc.export()
    assert len(ex["keys"]) == len(centers)
    got = {int(k): (int(n), ex["s"][:, i]) for i, (k, n) in enumerate(zip(ex["keys"], ex["n_new"]))}
    for c, n, v in zip(centers, counts, values):
        k = (0xA << 48) | ((c[2] & 0xFFFF) << 32) | ((c[1] & 0xFFFF) << 16) | (c[0] & 0xFFFF)
        assert k in got
        assert got[k][0] == n
        np.testing.assert_allclose(got[k][1], v.astype(np.float64).sum(axis=1), rtol=0, atol=1e-12)


def test_grouping_brute_force_scan():
    # O(N*C) scan over distinct keys equals the map's counts and sums
    rng = np.random.default_rng(11)
    n = 400
    p = rng.integers(-3, 3, size=(3, n)).astype(np.float32) + 0.5
    nrm = np.eye(3, dtype=np.float32)[rng.integers(0, 3, size=n)]
    rgb = rng.uniform(0, 2, size=(3, n)).astype(np.float32)
    rec = records(n, px=p[0], py=p[1], pz=p[2], nx=nrm[:, 0], ny=nrm[:, 1], nz=nrm[:, 2],
                  r=rgb[0], g=rgb[1], b=rgb[2])
    orc = oracle.Oracle(**_cfg())
    keys, _ = orc.keys(rec)
    orc.insert(rec)
    ex = orc.export()
    distinct = sorted(set(int(k) for k in keys))
    assert [int(k) for k in ex["keys"]] == distinct
    for i, k in enumerate(distinct):
        cnt = 0
        sums = [0.0, 0.0, 0.0]
        for j in range(n):
            if int(keys[j]) == k:
                cnt += 1
                for ch in range(3):
                    sums[ch] += float(rgb[ch][j])
        assert int(ex["n_new"][i]) == cnt
        for ch in range(3):
            assert abs(ex["s"][ch][i] - sums[ch]) <= 1e-12 * max(1.0, abs(sums[ch]))


def _tiny_records(it, field=0, noise=1):
    wl = W.tiny(field=field, noise=noise)
    sc = W.make_scene(wl)
    rec = dict(sc.generate(wl["gen"], it))
    rec["rough"] = None
    return wl, rec


def test_conservation_and_radiance_sum():
    wl, rec = _tiny_records(0)
    n = len(rec["px"])
    bad = np.arange(0, n, 97)
    rec["px"][bad[::2]] = np.nan
    rec["g"][bad[1::2]] = np.inf
    orc = oracle.Oracle(**wl["table"])
    orc.insert(rec)
    ex = orc.export()
    cnt = orc.counters()
    assert cnt["skipped"] == len(bad)
    assert int(ex["n_new"].sum()) == n - len(bad)
    good = np.ones(n, bool)
    good[bad] = False
    for ch, f in enumerate("rgb"):
        want = rec[f][good].astype(np.float64).sum()
        assert abs(ex["s"][ch].sum() - want) <= 1e-9 * want


def test_order_invariance():
    wl, rec = _tiny_records(1)
    perm = np.random.default_rng(5).permutation(len(rec["px"]))
    a = oracle.Oracle(**wl["table"])
    b = oracle.Oracle(**wl["table"])
    a.insert(rec)
    b.insert(take(rec, perm))
    ea, eb = a.export(), b.export()
    assert np.array_equal(ea["keys"], eb["keys"])
    assert np.array_equal(ea["n_new"], eb["n_new"])
    np.testing.assert_allclose(ea["s"], eb["s"], rtol=1e-12)
    a.update()
    b.update()
    np.testing.assert_allclose(a.export()["L"], b.export()["L"], rtol=1e-12)


def test_constant_field_gives_constant_exactly():
    # noise-free constant radiance: every cell mean equals the constant
    # exactly, and the blend keeps it (to rounding of the convex combination)
    for mode in (ALPHA_PAPER, ALPHA_CONST, ALPHA_LINEAR):
        wl = W.tiny(alpha_mode=mode, field=1, noise=0)
        sc = W.make_scene(wl)
        orc = oracle.Oracle(**wl["table"])
        amp = np.array(wl["gen"]["amp"], dtype=np.float32).astype(np.float64)
        for it in range(4):
            rec = dict(sc.generate(wl["gen"], it))
            rec["rough"] = None
            orc.insert(rec)
            ex = orc.export()
            t = ex["n_new"] > 0
            m = ex["s"][:, t] / ex["n_new"][t]
            assert np.array_equal(m, np.broadcast_to(amp[:, None], m.shape))
            orc.update()
            L = orc.export()["L"]
            np.testing.assert_allclose(L, np.broadcast_to(amp[:, None], L.shape), rtol=4e-16)


def test_linear_field_mean_is_value_at_centroid():
    lin_a = (0.3, -0.2, 0.1, 0.0, 0.5, 0.25, -0.4, 0.1, 0.6)
    lin_b = (2.0, 1.5, 3.0)
    wl = W.tiny(field=2, noise=0)
    wl["gen"]["lin_a"] = lin_a
    wl["gen"]["lin_b"] = lin_b
    sc = W.make_scene(wl)
    rec = dict(sc.generate(wl["gen"], 0))
    rec["rough"] = None
    orc = oracle.Oracle(**wl["table"])
    keys, _ = orc.keys(rec)
    orc.insert(rec)
    ex = orc.export()
    idx = np.searchsorted(ex["keys"], keys)
    cnt = np.bincount(idx, minlength=len(ex["keys"])).astype(np.float64)
    cen = np.stack([np.bincount(idx, weights=rec[f].astype(np.float64), minlength=len(cnt)) / cnt
                    for f in ("px", "py", "pz")])
    A = np.array(lin_a).reshape(3, 3)
    want = np.array(lin_b)[:, None] + A @ cen
    m = ex["s"] / ex["n_new"]
    np.testing.assert_allclose(m, want, rtol=2e-6, atol=2e-6)


# ----------------------------------------------------------------- Eq. 10-11
def _run_golden(fname, **cfg):
    orc = oracle.Oracle(**_cfg(**cfg))
    for row in golden_rows(fname):
        if row[0] != "-":
            v = [float(x) for x in row[0].split(",")]
            rec = records(len(v), px=0.5, py=0.5, pz=0.5, r=v, g=v, b=v)
            orc.insert(rec)
        orc.update()
        ex = orc.export()
        assert len(ex["keys"]) == 1
        assert int(ex["c_old"][0]) == int(row[2])
        np.testing.assert_allclose(ex["L"][:, 0], float(row[1]), rtol=1e-15, atol=1e-15)


def test_temporal_eq11_worked_example():
    _run_golden("temporal_paper_tmax2.txt", alpha_mode=ALPHA_PAPER, t_max=2.0)


def test_temporal_constant_alpha_worked_example():
    _run_golden("temporal_const_quarter.txt", alpha_mode=ALPHA_CONST, alpha=0.25)


def _frames(seed, nframes, ncells, max_per=6):
    """Random per-frame samples into a few fixed unit cells."""
    rng = np.random.default_rng(seed)
    frames = []
    for _ in range(nframes):
        counts = rng.integers(0, max_per, size=ncells)
        cells = [(i, 0, 0) for i in range(ncells)]
        vals = [rng.exponential(1.0, size=(3, c)).astype(np.float32) * (1 + i)
                for i, c in enumerate(counts)]
        frames.append((cells, counts, vals))
    return frames


def test_linear_mode_is_cumulative_mean():
    # Sec. 2.4: without the square root the blend is linear accumulation, i.e.
    # the plain sample mean over every frame so far
    orc = oracle.Oracle(**_cfg(alpha_mode=ALPHA_LINEAR))
    tot = {}
    for f, (cells, counts, vals) in enumerate(_frames(21, 12, 5)):
        keep = [i for i, c in enumerate(counts) if c > 0]
        if keep:
            orc.insert(_cell_records([cells[i] for i in keep], [counts[i] for i in keep],
                                     [vals[i] for i in keep], seed=f))
        for i in keep:
            s, n = tot.get(i, (np.zeros(3), 0))
            tot[i] = (s + vals[i].astype(np.float64).sum(axis=1), n + counts[i])
        orc.update()
        ex = orc.export()
        kx = {int(k): j for j, k in enumerate(ex["keys"])}
        for i, (s, n) in tot.items():
            j = kx[(0xA << 48) | i]
            assert int(ex["c_old"][j]) == n
            np.testing.assert_allclose(ex["L"][:, j], s / n, rtol=1e-13)


def test_constant_mode_is_exponential_weighting():
    # closed form of constant-alpha averaging: L_k = sum_j beta_j m_j with
    # beta_j = a (1-a)^(k-j) for j after the first frame and (1-a)^(k-1) for it
    a = 0.3
    orc = oracle.Oracle(**_cfg(alpha_mode=ALPHA_CONST, alpha=a))
    a32 = float(np.float32(a))
    means = []
    for f in range(10):
        v = np.random.default_rng(100 + f).uniform(0, 4, size=(3, 3)).astype(np.float32)
        orc.insert(_cell_records([(2, 2, 2)], [3], [v], seed=f))
        means.append(v.astype(np.float64).mean(axis=1))
        orc.update()
        k = len(means)
        beta = [(1 - a32) ** (k - 1)] + [a32 * (1 - a32) ** (k - 1 - j) for j in range(1, k)]
        want = sum(b * m for b, m in zip(beta, means))
        assert abs(sum(beta) - 1.0) < 1e-12
        np.testing.assert_allclose(orc.export()["L"][:, 0], want, rtol=1e-12)


def test_eq11_alpha_recovered_from_state():
    # Invert the blend: alpha = (L_new - L_old) / (m - L_old); it must satisfy
    # alpha = 1 on first touch, alpha >= 1/T_max always, alpha^2 = n/(c+n)
    # whenever that exceeds the floor.
    t_max = 4.0
    orc = oracle.Oracle(**_cfg(alpha_mode=ALPHA_PAPER, t_max=t_max))
    rng = np.random.default_rng(31)
    L_old, c_old = None, 0
    seen_floor = seen_sqrt = False
    for f in range(40):
        n = int(rng.integers(1, 9))
        v = rng.uniform(0, 10, size=n).astype(np.float32)
        orc.insert(_cell_records([(0, 0, 0)], [n], [np.stack([v, v, v])], seed=f))
        m = v.astype(np.float64).mean()
        orc.update()
        L = orc.export()["L"][0, 0]
        if L_old is None:
            assert L == m
        elif abs(m - L_old) > 1e-3:
            alpha = (L - L_old) / (m - L_old)
            ratio = n / (c_old + n)
            assert alpha >= 1 / t_max - 1e-9
            if ratio > 1 / t_max ** 2 + 1e-9:
                assert abs(alpha * alpha - ratio) < 1e-9
                seen_sqrt = True
            else:
                assert abs(alpha - 1 / t_max) < 1e-9
                seen_floor = True
        L_old, c_old = L, c_old + n
    assert seen_floor and seen_sqrt


def test_blend_stays_between_frame_means():
    # the weights of Eq. 10 are a convex combination of the frame means
    for mode in (ALPHA_PAPER, ALPHA_CONST, ALPHA_LINEAR):
        orc = oracle.Oracle(**_cfg(alpha_mode=mode))
        lo = np.full((3, 4), np.inf)
        hi = np.full((3, 4), -np.inf)
        for f, (cells, counts, vals) in enumerate(_frames(40 + mode, 15, 4)):
            keep = [i for i, c in enumerate(counts) if c > 0]
            if not keep:
                continue
            orc.insert(_cell_records([cells[i] for i in keep], [counts[i] for i in keep],
                                     [vals[i] for i in keep], seed=f))
            for i in keep:
                m = vals[i].astype(np.float64).mean(axis=1)
                lo[:, i] = np.minimum(lo[:, i], m)
                hi[:, i] = np.maximum(hi[:, i], m)
            orc.update()
            ex = orc.export()
            for j, k in enumerate(ex["keys"]):
                i = int(k) & 0xFFFF
                assert np.all(ex["L"][:, j] >= lo[:, i] * (1 - 1e-14))
                assert np.all(ex["L"][:, j] <= hi[:, i] * (1 + 1e-14))


def test_untouched_cells_unchanged():
    orc = oracle.Oracle(**_cfg())
    orc.insert(_cell_records([(0, 0, 0), (1, 1, 1)], [2, 2], [np.ones((3, 2)), 2 * np.ones((3, 2))]))
    orc.update()
    before = orc.export()
    orc.insert(_cell_records([(0, 0, 0)], [1], [5 * np.ones((3, 1))]))
    assert orc.update() == 1
    after = orc.export()
    assert after["c_old"][1] == before["c_old"][1]
    assert np.array_equal(after["L"][:, 1], before["L"][:, 1])


def test_exponential_noise_variance_of_eq11():
    # Constant field c times Exp(1) noise: the blended estimate is an unbiased
    # weighted mean whose variance is c^2 * sum_j beta_j^2 / n_j (beta_j the
    # Eq. 10 weights of each frame, n_j its sample count).  Check it by a
    # z-test over many independent cells.
    t_max = 5.0
    ncell, nframes, per = 3000, 12, 3
    rng = np.random.default_rng(77)
    orc = oracle.Oracle(**_cfg(alpha_mode=ALPHA_PAPER, t_max=t_max))
    c = 2.0
    cells = [(i % 50, i // 50, 0) for i in range(ncell)]
    betas = []
    c_old = 0
    for f in range(nframes):
        vals = [np.broadcast_to(c * rng.exponential(1.0, size=per), (3, per)).astype(np.float32)
                for _ in range(ncell)]
        orc.insert(_cell_records(cells, [per] * ncell, vals, seed=f))
        orc.update()
        alpha = 1.0 if c_old == 0 else max(math.sqrt(per / (c_old + per)), 1 / t_max)
        betas = [b * (1 - alpha) for b in betas] + [alpha]
        c_old += per
    var = c * c * sum(b * b / per for b in betas)
    L = orc.export()["L"][0]
    z_mean = (L.mean() - c) / math.sqrt(var / ncell)
    assert abs(z_mean) < 4.5
    s2 = L.var(ddof=1)
    assert abs(s2 / var - 1.0) < 0.15
    # sits between linear accumulation (variance c^2/total) and constant 1/T_max
    lin = c * c / (nframes * per)
    assert lin < var


# ----------------------------------------------------------------- lookup, reset
def test_query_semantics():
    orc = oracle.Oracle(**_cfg())
    rec = _cell_records([(0, 0, 0), (3, 0, 0)], [4, 2], [np.full((3, 4), 2.0), np.full((3, 2), 5.0)])
    orc.insert(rec)
    q = records(3, px=[0.5, 3.5, 40.5], py=[0.5, 0.5, 0.5], pz=[0.5, 0.5, 0.5])
    out, found = orc.query(q)
    assert found.tolist() == [0, 0, 0]  # nothing blended yet
    assert np.all(out == 0)
    orc.update()
    out, found = orc.query(q)
    assert found.tolist() == [1, 1, 0]
    assert out[:, 0].tolist() == [2.0, 2.0, 2.0]
    assert out[:, 1].tolist() == [5.0, 5.0, 5.0]
    assert out[:, 2].tolist() == [0.0, 0.0, 0.0]
    # a non-finite query misses
    qb = records(1, px=[np.nan])
    assert orc.query(qb)[1].tolist() == [0]
    # global counter reset: cells stay but are not reported until re-blended,
    # and the next blend starts over (alpha = 1)
    orc.reset(RESET_COUNTERS)
    assert orc.query(q)[1].tolist() == [0, 0, 0]
    orc.insert(_cell_records([(0, 0, 0)], [1], [np.full((3, 1), 7.0)]))
    orc.update()
    out, found = orc.query(q)
    assert found.tolist() == [1, 0, 0]
    assert out[:, 0].tolist() == [7.0, 7.0, 7.0]
    orc.reset(RESET_CLEAR)
    assert orc.count() == 0
    assert orc.query(q)[1].tolist() == [0, 0, 0]


def test_filter_tracks_subset_identically():
    wl, rec = _tiny_records(2)
    full = oracle.Oracle(**wl["table"])
    full.insert(rec)
    full.update()
    ef = full.export()
    pick = ef["keys"][::7]
    sub = oracle.Oracle(**wl["table"])
    sub.set_filter(pick)
    sub.insert(rec)
    sub.update()
    es = sub.export()
    assert np.array_equal(es["keys"], pick)
    j = np.searchsorted(ef["keys"], pick)
    assert np.array_equal(es["c_old"], ef["c_old"][j])
    assert np.array_equal(es["L"], ef["L"][:, j])


def test_local_counter_reset_worked_example():
    """Sec. 2.4: counters may be zeroed locally.  Level-0 cells of edge 1
    (e_min 0, fixed level); the region [0.9, 2] x [0, 1] x [0, 1] meets the
    cells [0,1) and [2,3) along x (closed upper bound) but not [-1,0).  Reset
    cells are hidden from queries until blended again, and that blend starts
    over (alpha = 1: the new mean)."""
    orc = oracle.Oracle(kappa=0.0, e_min=0, alpha_mode=oracle.ALPHA_CONST, alpha=0.25)
    xs = [0.5, 2.5, -0.5]
    rec = records(3, px=xs, py=0.5, pz=0.5, r=[1.0, 2.0, 3.0], g=[1.0, 2.0, 3.0], b=[1.0, 2.0, 3.0])
    orc.insert(rec)
    orc.update()
    orc.reset_region((0.9, 0.0, 0.0), (2.0, 1.0, 1.0))
    _, found = orc.query(rec)
    assert list(found) == [0, 0, 1]
    ex = orc.export()
    assert sorted(ex["c_old"].tolist()) == [0, 0, 1]
    rec2 = records(3, px=xs, py=0.5, pz=0.5, r=[5.0, 6.0, 7.0], g=[5.0, 6.0, 7.0], b=[5.0, 6.0, 7.0])
    orc.insert(rec2)
    orc.update()
    out, found = orc.query(rec2)
    assert list(found) == [1, 1, 1]
    # reset cells take the new mean; the kept one blends 3/4 * 3 + 1/4 * 7
    assert list(out[0]) == [5.0, 6.0, 4.0]


def test_local_counter_reset_whole_space_equals_global_reset():
    from synth import workloads as W
    wl = W.tiny()
    sc = W.make_scene(wl)
    a, b = oracle.Oracle(**wl["table"]), oracle.Oracle(**wl["table"])
    for it in range(2):
        rec = dict(sc.generate(wl["gen"], it))
        rec["rough"] = None
        for o in (a, b):
            o.insert(rec)
            o.update()
    a.reset(oracle.RESET_COUNTERS)
    b.reset_region((-1e30, -1e30, -1e30), (1e30, 1e30, 1e30))
    ea, eb = a.export(), b.export()
    assert np.array_equal(ea["keys"], eb["keys"]) and np.array_equal(ea["c_old"], eb["c_old"])
    assert int(eb["c_old"].sum()) == 0
