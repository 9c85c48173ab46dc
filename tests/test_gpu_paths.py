"""The GPU path sampler (psf_sample_paths) feeding the progressive solver
(Sec. 2.2; Algorithms 1 and 2) entirely on the device.  Pinned by what the
mathematics fixes: Philox known answers, geometric invariants of the traced
paths, the cosine-weighted direction density, the closed-form direct
illumination under a square emitter (next-event estimation and the emission
reached by scattering, balance-weighted, must average to it), and the
closed furnace's fixed points L_e / (1 - rho) (Algorithm 1) and
rho L_e / (1 - rho) (Algorithm 2's radiance minus emission)."""
import math

import numpy as np
import pytest

from tests.test_paths_closed_forms import centred_square_form_factor

pytestmark = pytest.mark.gpu

LE = np.array([1.0, 0.5, 0.25])
RHO = np.array([0.5, 0.6, 0.7])


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_07547_amd import psf
    psf.load()
    return torch, psf


def _host(d):
    return {k: v.cpu().numpy().astype(np.float64) for k, v in d.items()}


def test_philox_known_answers_on_device(env):
    torch, psf = env
    # known-answer vectors published with the Random123 library (Salmon et
    # al., SC'11) for Philox-4x32 with 10 rounds
    ctr = np.array([[0, 0, 0, 0], [0xFFFFFFFF] * 4, [0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344]],
                   dtype=np.uint32)
    key = np.array([[0, 0], [0xFFFFFFFF] * 2, [0xA4093822, 0x299F31D0]], dtype=np.uint32)
    want = np.array([[0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8],
                     [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD],
                     [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]], dtype=np.uint32)
    assert np.array_equal(psf.philox(ctr, key), want)


def _furnace(psf, mode=0):
    from synth import workloads as W
    scene = psf.Scene(W.furnace_scene(tuple(LE), tuple(RHO)))
    return scene


def test_furnace_path_geometry_and_direction_density(env):
    torch, psf = env
    scene = _furnace(psf)
    paths, verts = 1 << 16, 3
    cam = psf.camera((0, 0, 0), (0, 0, 1), (0, 1, 0), 60.0, paths, 1)
    x, nx, t, le = psf.sample_paths(scene, cam, verts, psf.PSF_PATHS_LO, psf.PSF_ORIGIN_POINT, seed=5, frame=2)
    X, N = _host(x), _host(nx)
    p = np.stack([X["px"], X["py"], X["pz"]])
    n = np.stack([X["nx"], X["ny"], X["nz"]])
    wo = np.stack([X["ox"], X["oy"], X["oz"]])
    assert np.all(np.abs(np.linalg.norm(p, axis=0) - 1.0) < 1e-5)  # on the unit sphere
    # the normal faces the outgoing direction: inward, except where a
    # grazing step leaves the sign of cos(normal, w_o) to rounding
    inward = np.all(np.abs(n + p) < 1e-5, axis=0)
    assert np.all(inward | np.all(np.abs(n - p) < 1e-5, axis=0))
    assert np.all(np.sum(n * wo, axis=0) >= -1e-6)
    assert inward.mean() > 0.9999
    assert np.all(np.abs(np.linalg.norm(wo, axis=0) - 1.0) < 1e-5)
    # a step leaves the closed sphere only where a grazing arrival left the
    # normal's orientation to rounding (then the path restarts)
    esc = ~np.isfinite(N["px"])
    assert esc.mean() < 1e-3
    for c in range(3):  # cosine-weighted scattering: f cos / p is the albedo
        tc = t[c].cpu().numpy()
        assert np.all(tc[~esc] == np.float32(RHO[c])) and np.all(tc[esc] == 0.0)
        assert np.all(le[c].cpu().numpy() == np.float32(LE[c]))
    # the next vertex of vertex i is vertex i + 1 of the same path, and the
    # outgoing direction there points back along the step
    q = np.stack([N["px"], N["py"], N["pz"]]).reshape(3, verts, paths)
    P = p.reshape(3, verts, paths)
    W = wo.reshape(3, verts, paths)
    cont = ~esc.reshape(verts, paths)[:-1]
    assert np.array_equal(q[:, :-1][:, cont], P[:, 1:][:, cont])
    step = P[:, 1:] - P[:, :-1]
    step /= np.linalg.norm(step, axis=0)
    assert np.all(np.abs(step + W[:, 1:])[:, cont] < 1e-4)
    # direction density cos / pi: E[cos] = 2/3, Var[cos] = 1/18
    cos = np.sum(step * (-P[:, :-1]), axis=0)[cont]
    z = (cos.mean() - 2.0 / 3.0) / math.sqrt(1.0 / 18.0 / cos.size)
    assert abs(z) < 4.0, z
    assert cos.min() > -1e-6


def _furnace_loop(torch, psf, mode, frames, paths=2048, verts=2):
    from synth import workloads as W
    scene = _furnace(psf)
    t = psf.Table(**W.furnace_table())
    cam = psf.camera((0, 0, 0), (0, 0, 1), (0, 1, 0), 60.0, paths, 1)
    buf = None
    over = -np.inf
    L_star = LE / (1.0 - RHO) if mode == psf.PSF_PATHS_LO else RHO * LE / (1.0 - RHO)
    for it in range(frames):
        x, nx, tp, le = psf.sample_paths(scene, cam, verts, mode, psf.PSF_ORIGIN_POINT, seed=11, frame=it, out=buf)
        buf = {**{k: v for k, v in x.items()}, "qx": nx["px"], "qy": nx["py"], "qz": nx["pz"], "qnx": nx["nx"],
               "qny": nx["ny"], "qnz": nx["nz"], "qox": nx["ox"], "qoy": nx["oy"], "qoz": nx["oz"],
               "qrough": nx["rough"], "t_r": tp[0], "t_g": tp[1], "t_b": tp[2], "le_r": le[0], "le_g": le[1],
               "le_b": le[2]}
        t.progressive_step(x, nx, tp, le)
        if it < 30 and it % 5 == 4:
            over = max(over, float(np.max(t.export()["L"] / L_star[:, None] - 1.0)))
    torch.cuda.synchronize()
    L = t.export()["L"].astype(np.float64)
    return np.abs(L / L_star[:, None] - 1.0), over


def test_furnace_algorithm_1_converges_on_the_device(env):
    """Algorithm 1 in the furnace, every frame sampled and filtered on the
    GPU: L_e / (1 - rho) within the oracle pin's bounds, approached from
    below (every sample is L_e + rho * (a value <= L*))."""
    torch, psf = env
    rel, over = _furnace_loop(torch, psf, psf.PSF_PATHS_LO, 200)
    assert over <= 1e-5
    assert float(np.mean(rel)) < 5e-4 and float(np.percentile(rel, 90)) < 1e-3, (rel.mean(), np.percentile(rel, 90))


def test_furnace_algorithm_2_with_next_event_estimation(env):
    """Algorithm 2 (L_o\\e) with next-event estimation and the balance
    heuristic: rho L_e / (1 - rho)."""
    torch, psf = env
    rel, _ = _furnace_loop(torch, psf, psf.PSF_PATHS_LOE, 200)
    assert float(np.mean(rel)) < 5e-4 and float(np.percentile(rel, 90)) < 1e-3, (rel.mean(), np.percentile(rel, 90))


def test_square_light_direct_illumination(env):
    """Floor point under a square emitter: Algorithm 2's emission argument at
    the first vertex (next-event estimate plus the balance-weighted emission
    reached by the scattering event) averages to rho L F, F the form factor;
    the share of scattering events that reach the emitter is F itself."""
    from synth import workloads as W
    torch, psf = env
    h, s = 1.0, 0.5
    light, albedo = np.array([3.0, 2.0, 1.0]), np.array([0.8, 0.5, 0.3])
    prims, c = W.square_light_scene(h, s, tuple(light), tuple(albedo))
    scene = psf.Scene(prims)
    cam = psf.camera(c["pos"], c["fwd"], c["up"], c["fov_y_deg"], 1024, 1024, 1)
    F = centred_square_form_factor(s, h)
    x, nx, tp, le = psf.sample_paths(scene, cam, 1, psf.PSF_PATHS_LOE, psf.PSF_ORIGIN_CAMERA, seed=3, frame=0)
    X = _host(x)
    assert np.all(np.abs(X["py"]) < 1e-6) and np.all(np.hypot(X["px"], X["pz"]) < 1e-3)
    for ch in range(3):
        v = le[ch].cpu().numpy().astype(np.float64)
        want = albedo[ch] * light[ch] * F
        z = (v.mean() - want) / (v.std() / math.sqrt(v.size))
        assert abs(z) < 4.0, (ch, v.mean(), want, z)
    x, nx, tp, le = psf.sample_paths(scene, cam, 1, psf.PSF_PATHS_LO, psf.PSF_ORIGIN_CAMERA, seed=4, frame=0)
    hit = np.abs(nx["py"].cpu().numpy() - h) < 1e-5
    z = (hit.mean() - F) / math.sqrt(F * (1 - F) / hit.size)
    assert abs(z) < 4.0, (hit.mean(), F, z)
    # Algorithm 1's emission argument is the vertex's own emission: 0 on the floor
    assert float(le[0].abs().max()) == 0.0


def _dist_to_prims(p, prims):
    """Distance (binary64, host) from points p (3, n) to the nearest
    primitive surface."""
    best = np.full(p.shape[1], np.inf)
    for q in prims:
        c = np.asarray(q["p"], dtype=np.float64)[:, None]
        if q["kind"] == "sphere":
            d = np.abs(np.linalg.norm(p - c, axis=0) - q["radius"])
        else:
            u, v = np.asarray(q["u"], dtype=np.float64), np.asarray(q["v"], dtype=np.float64)
            nrm = np.cross(u, v)
            nrm /= np.linalg.norm(nrm)
            r = p - c
            a = np.clip((u @ r) / (u @ u), -1, 1)
            b = np.clip((v @ r) / (v @ v), -1, 1)
            proj = c + np.outer(u, a) + np.outer(v, b)
            d = np.linalg.norm(p - proj, axis=0)
        best = np.minimum(best, d)
    return best


def test_box_scene_paths(env):
    """Camera paths in the tiny workload's open box: every vertex lies on a
    primitive, normals face the outgoing direction, a path that leaves
    through the open side restarts (no vertex is missing), and the next
    vertex of every non-final vertex is the path's following vertex or an
    escape."""
    from synth import workloads as W
    torch, psf = env
    prims, c = W.box_scene()
    scene = psf.Scene(prims)
    verts = 4
    cam = psf.camera(c["pos"], c["fwd"], c["up"], c["fov_y_deg"], 64, 64, 2)
    x, nx, tp, le = psf.sample_paths(scene, cam, verts, psf.PSF_PATHS_LOE, psf.PSF_ORIGIN_CAMERA, seed=7, frame=1)
    X, N = _host(x), _host(nx)
    p = np.stack([X["px"], X["py"], X["pz"]])
    # pixels near the image corners see past the box's open side: their
    # paths never reach the scene and leave NaN records (skipped by inserts)
    ok = np.all(np.isfinite(p), axis=0)
    assert 0.8 < ok.mean() < 1.0
    paths = 64 * 64 * 2
    assert np.all(ok.reshape(verts, paths) == ok.reshape(verts, paths)[:1])  # whole paths or none
    assert np.all(_dist_to_prims(p[:, ok], prims) < 1e-4)
    n = np.stack([X["nx"], X["ny"], X["nz"]])
    wo = np.stack([X["ox"], X["oy"], X["oz"]])
    assert np.all(np.sum(n * wo, axis=0)[ok] >= -1e-6)
    q = np.stack([N["px"], N["py"], N["pz"]])
    esc = ~np.isfinite(q[0])
    assert esc[ok].any() and (~esc[ok]).any()
    assert np.all(_dist_to_prims(q[:, ~esc], prims) < 1e-4)
    P, Q, E = p.reshape(3, verts, paths), q.reshape(3, verts, paths), esc.reshape(verts, paths)
    cont = ~E[:-1]
    assert np.array_equal(Q[:, :-1][:, cont], P[:, 1:][:, cont])
    for ch in range(3):
        tt = tp[ch].cpu().numpy().reshape(verts, paths)
        assert np.all(tt[E] == 0.0)
        assert np.all(le[ch].cpu().numpy()[ok] >= 0.0)
