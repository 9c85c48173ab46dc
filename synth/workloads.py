"""Synthetic workloads shaped like the paper's measurements.

The paper's scenes (door ajar, staircase, arch interior) and renderer are not
available; these procedural stand-ins reproduce the shapes that matter for the
hash path: image size, samples per pixel, vertices per path, wavefront record
order, diffuse/glossy mix and radiance distribution.

Each workload is a plain dict.  ``table`` holds the filter configuration
(identical for the oracle and the library); ``gen`` holds the generator
parameters.  ``kappa`` is the camera-distance level scale
(k_s * theta_pix / 2^e_min)^2 computed once here in float32 and handed to both
sides as the same float.
"""
from __future__ import annotations

import math

import numpy as np

from . import Scene

ALPHA_PAPER, ALPHA_CONST, ALPHA_LINEAR = 0, 1, 2


def kappa_for(fov_y_deg: float, height: int, k_s: float, e_min: int) -> float:
    f32 = np.float32
    theta = f32(2.0) * f32(math.tan(math.radians(fov_y_deg) / 2.0)) / f32(height)
    v = f32(k_s) * theta / f32(2.0 ** e_min)
    return float(f32(v * v))


def _table(log2_slots, cam, fov, height, k_s, e_min, alpha_mode=ALPHA_PAPER, alpha=0.2,
           t_max=5.0, rough_thr=0.3, max_level=15, max_probe=64):
    return {
        "log2_slots": log2_slots, "max_probe": max_probe, "cam": tuple(float(c) for c in cam),
        "kappa": kappa_for(fov, height, k_s, e_min), "e_min": e_min, "max_level": max_level,
        "normal_bins_log2": 2, "dir_bins_log2": 3, "rough_thr": rough_thr,
        "alpha_mode": alpha_mode, "alpha": alpha, "t_max": t_max,
    }


def tiny(alpha_mode=ALPHA_CONST, field=0, noise=1):
    """64x64, 1 spp, 2 vertices/path in an open box with a sphere; diffuse;
    2^16 slots; 8 iterations; constant alpha 0.2 (or Eq. 11 with T_max = 5)."""
    cam = (0.5, 0.5, -1.5)
    gen = {"width": 64, "height": 64, "spp": 1, "verts": 2, "seed": 1, "cam": cam,
           "look": (0.0, 0.0, 1.0), "fov_y_deg": 40.0, "field": field, "noise": noise,
           "field_scale": 1.0, "amp": (1.0, 0.8, 0.6), "glossy_lobe": 0}
    return {"name": "tiny-64x64-2v", "scene": dict(kind=Scene.BOX, seed=1), "gen": gen,
            "diffuse_only": True, "iterations": 8,
            "table": _table(16, cam, 40.0, 64, 2.0, -6, alpha_mode=alpha_mode)}


def plain():
    """1280x720, 1 spp, 4 vertices/path; 64 random quads + 16 spheres with
    roughness U[0.05, 1]; directional keys below roughness 0.3; 2^22 slots;
    32 iterations; Eq. 11 with T_max = 5."""
    cam = (0.0, 0.0, -10.0)
    gen = {"width": 1280, "height": 720, "spp": 1, "verts": 4, "seed": 2, "cam": cam,
           "look": (0.0, 0.0, 1.0), "fov_y_deg": 60.0, "field": 0, "noise": 1,
           "field_scale": 4.0, "amp": (1.0, 0.8, 0.6), "glossy_lobe": 1}
    return {"name": "plain-1280x720-4v", "scene": dict(kind=Scene.RANDOM, seed=2, glossy_frac=-1.0),
            "gen": gen, "diffuse_only": False, "iterations": 32,
            "table": _table(22, cam, 60.0, 720, 8.0 * math.sqrt(2.0), -5)}


def precision():
    """1920x1080, 1 spp, 5 vertices/path; half the primitives glossy; HDR
    lognormal(0, 2) noise; 2^24 slots; 64 iterations."""
    cam = (0.0, 0.0, -10.0)
    gen = {"width": 1920, "height": 1080, "spp": 1, "verts": 5, "seed": 3, "cam": cam,
           "look": (0.0, 0.0, 1.0), "fov_y_deg": 60.0, "field": 0, "noise": 2, "sigma": 2.0,
           "field_scale": 4.0, "amp": (1.0, 0.8, 0.6), "glossy_lobe": 1}
    return {"name": "precision-1920x1080-5v", "scene": dict(kind=Scene.RANDOM, seed=3, glossy_frac=0.5),
            "gen": gen, "diffuse_only": False, "iterations": 64,
            "table": _table(24, cam, 60.0, 1080, 8.0 * math.sqrt(2.0), -5)}


BATCH_RES = ((256, 256), (512, 384), (640, 480), (1280, 720), (1920, 1080))


def batched_sessions(n_sessions=16, seed=4):
    """16 sessions of uneven resolutions, 1-4 spp, 3-5 vertices/path, tables of
    2^18..2^23 slots, 32 iterations."""
    from . import philox4x32_10
    out = []
    for i in range(n_sessions):
        w, h = BATCH_RES[i % len(BATCH_RES)]
        r = philox4x32_10((i, 0, 0, 0), (seed, 0x0b47c4ed))
        spp = 1 + int(r[0] % 4)
        verts = 3 + int(r[1] % 3)
        # distinct cells grow with pixels x vertices, not with spp
        log2 = int(min(23, max(18, math.ceil(math.log2(max(1, w * h * verts))))))
        cam = (0.0, 0.0, -10.0)
        gen = {"width": w, "height": h, "spp": spp, "verts": verts, "seed": 100 + i, "cam": cam,
               "look": (0.0, 0.0, 1.0), "fov_y_deg": 60.0, "field": 0, "noise": 1,
               "field_scale": 4.0, "amp": (1.0, 0.8, 0.6), "glossy_lobe": 1}
        out.append({"name": f"session{i}-{w}x{h}-{spp}spp-{verts}v",
                    "scene": dict(kind=Scene.RANDOM, seed=100 + i, glossy_frac=-1.0),
                    "gen": gen, "diffuse_only": False, "iterations": 32,
                    "table": _table(log2, cam, 60.0, h, 8.0 * math.sqrt(2.0), -5)})
    return out


def records_per_iteration(wl) -> int:
    g = wl["gen"]
    return int(g["width"]) * int(g["height"]) * int(g.get("spp", 1)) * int(g["verts"])


def make_scene(wl) -> Scene:
    return Scene(**wl["scene"])


def estimator_inputs(rec: dict, gen: dict) -> tuple:
    """Inputs of the two-field estimators for the records of one iteration
    (depth-major, `gen` the generator parameters that made them).

    The sampled incoming direction at a vertex is the direction to the
    vertex one depth further along the same pixel's path (the last depth
    takes the mirror of the outgoing direction about the normal); the
    vertex's sample g is the next vertex's value (the last depth its own) and
    its weight w / p_perp a deterministic value in [pi/2, 3 pi/2).  Returns
    (args, fl_records): args keyed as the estimator expects, fl_records the
    same vertices keyed on the incoming direction with value g (the samples
    of the f L_i field).  Roughness is passed through; when the records have
    none it is 1 (diffuse under the outgoing field's threshold, directional
    under the f L_i field's infinite one)."""
    n = int(rec["px"].shape[0])
    per = int(gen["width"]) * int(gen["height"]) * int(gen.get("spp", 1))
    verts = n // per
    f64 = np.float64
    p = np.stack([rec["px"], rec["py"], rec["pz"]]).astype(f64)
    nn = np.stack([rec["nx"], rec["ny"], rec["nz"]]).astype(f64)
    wo = np.stack([rec["ox"], rec["oy"], rec["oz"]]).astype(f64)
    wi = np.empty_like(p)
    g = np.stack([rec["r"], rec["g"], rec["b"]]).astype(np.float32)
    for d in range(verts):
        cur = slice(d * per, (d + 1) * per)
        if d + 1 < verts:
            nxt = slice((d + 1) * per, (d + 2) * per)
            v = p[:, nxt] - p[:, cur]
            g[:, cur] = g[:, nxt]
        else:
            v = 2.0 * np.sum(nn[:, cur] * wo[:, cur], axis=0) * nn[:, cur] - wo[:, cur]
        ln = np.sqrt(np.sum(v * v, axis=0))
        bad = ~(ln > 1e-12)
        v[:, bad] = nn[:, cur][:, bad]
        ln[bad] = 1.0
        wi[:, cur] = v / ln
    wi = wi.astype(np.float32)
    k = np.arange(n, dtype=f64)
    wp = (np.pi * (0.5 + np.mod(k * 0.6180339887498949, 1.0))).astype(np.float32)
    rough = rec.get("rough")
    rough = np.ones(n, dtype=np.float32) if rough is None else rough
    args = {"px": rec["px"], "py": rec["py"], "pz": rec["pz"], "nx": rec["nx"], "ny": rec["ny"],
            "nz": rec["nz"], "oox": rec["ox"], "ooy": rec["oy"], "ooz": rec["oz"],
            "oix": wi[0].copy(), "oiy": wi[1].copy(), "oiz": wi[2].copy(), "rough": rough,
            "gr": g[0].copy(), "gg": g[1].copy(), "gb": g[2].copy(), "wp": wp}
    fl = {"px": rec["px"], "py": rec["py"], "pz": rec["pz"], "nx": rec["nx"], "ny": rec["ny"],
          "nz": rec["nz"], "ox": args["oix"], "oy": args["oiy"], "oz": args["oiz"],
          "r": args["gr"], "g": args["gg"], "b": args["gb"], "rough": rough}
    return args, fl


def fl_table(table: dict) -> dict:
    """Configuration of the f L_i field beside a table of the outgoing field:
    the same grid, with the (incoming) direction in every key."""
    return dict(table, rough_thr=float("inf"))


def footprints(rec: dict, wl: dict, spread: float = 1.0) -> np.ndarray:
    """A path-footprint width per record (input of the footprint level rule):
    k_s * pixel angle * camera distance, the width the camera-distance rule
    assumes, times a deterministic factor 2^u with u in [-spread, spread)
    standing in for the footprint growth a renderer tracks along a path."""
    g = wl["gen"]
    cam = np.asarray(g["cam"], dtype=np.float64)
    theta = 2.0 * math.tan(math.radians(g["fov_y_deg"]) / 2.0) / float(g["height"])
    k_s = math.sqrt(wl["table"]["kappa"]) * 2.0 ** wl["table"]["e_min"] / theta if wl["table"]["kappa"] > 0 else 1.0
    p = np.stack([rec["px"], rec["py"], rec["pz"]]).astype(np.float64)
    d = np.sqrt(np.sum((p - cam[:, None]) ** 2, axis=0))
    k = np.arange(d.shape[0], dtype=np.float64)
    u = (np.mod(k * 0.7548776662466927, 1.0) * 2.0 - 1.0) * spread
    return (k_s * theta * d * np.exp2(u)).astype(np.float32)


def furnace_paths(n_paths: int, verts: int, it: int, seed: int = 9, le=(1.0, 0.5, 0.25),
                  albedo=(0.5, 0.6, 0.7)):
    """Paths inside a closed furnace: the unit sphere at the origin, seen from
    its centre, emitting le everywhere and reflecting diffusely with the
    given albedo.  Each path leaves the centre in a uniformly drawn direction
    and bounces `verts` times with cosine-weighted directions, so the
    throughput factor f G w / p of every step is the albedo.  Returns (x,
    nxt, tput, le): the vertices 1..verts as records without values
    (depth-major), the vertices 2..verts+1 as queries, and the per-vertex
    throughput and emission arrays (three each).  Seeded by (seed, it)."""
    rng = np.random.default_rng([seed, it])
    f32 = np.float32
    d = rng.normal(size=(3, n_paths))
    d /= np.linalg.norm(d, axis=0)
    pos = [d.copy()]          # first hit: the sphere point along d from the centre
    wo = [-d]                 # back toward the centre
    cur = d.copy()
    for _ in range(verts):
        nrm = -cur                               # inward normal
        u1, u2 = rng.uniform(size=(2, n_paths))
        r, phi = np.sqrt(u1), 2.0 * np.pi * u2
        lx, ly, lz = r * np.cos(phi), r * np.sin(phi), np.sqrt(np.maximum(0.0, 1.0 - u1))
        # orthonormal frame around the normal (Duff et al. 2017)
        sgn = np.where(nrm[2] >= 0.0, 1.0, -1.0)
        a = -1.0 / (sgn + nrm[2])
        b = nrm[0] * nrm[1] * a
        t1 = np.stack([1.0 + sgn * nrm[0] * nrm[0] * a, sgn * b, -sgn * nrm[0]])
        t2 = np.stack([b, sgn + nrm[1] * nrm[1] * a, -nrm[1]])
        w = lx * t1 + ly * t2 + lz * nrm
        w /= np.linalg.norm(w, axis=0)
        tt = -2.0 * np.sum(cur * w, axis=0)      # second intersection with |p| = 1
        nxt = cur + tt * w
        nxt /= np.linalg.norm(nxt, axis=0)
        pos.append(nxt)
        wo.append(-w)
        cur = nxt
    P = np.stack(pos)        # (verts + 1, 3, n)
    W = np.stack(wo)

    def pack(sl, with_dir):
        p = P[sl].transpose(1, 0, 2).reshape(3, -1)
        o = W[sl].transpose(1, 0, 2).reshape(3, -1)
        n = -p
        out = {"px": p[0], "py": p[1], "pz": p[2], "nx": n[0], "ny": n[1], "nz": n[2]}
        if with_dir:
            out.update(ox=o[0], oy=o[1], oz=o[2])
        return {k: np.ascontiguousarray(v, dtype=f32) for k, v in out.items()}

    x = pack(slice(0, verts), True)
    nx = pack(slice(1, verts + 1), True)
    m = n_paths * verts
    tput = tuple(np.full(m, c, dtype=f32) for c in albedo)
    emit = tuple(np.full(m, c, dtype=f32) for c in le)
    return x, nx, tput, emit


def furnace_table(log2_slots: int = 16) -> dict:
    """Fixed-level table for the furnace (edge 1/8, 4 x 4 normal bins)."""
    return _table(log2_slots, (0.0, 0.0, 0.0), 60.0, 64, 1.0, -3) | {"kappa": 0.0}


def mis_weights(n: int, seed: int = 21, excluded: float = 0.1) -> np.ndarray:
    """Per-record MIS weights standing in for a field fed by some of a
    renderer's sampling techniques: the balance-heuristic weight of one of two
    techniques whose densities at the sample are independent lognormal(0, 1)
    draws, p1 / (p1 + p2), in (0, 1); a fraction `excluded` of the records
    come from a technique the field leaves out (weight 0, rejected by the
    insert).  Seeded, binary32."""
    rng = np.random.default_rng(seed)
    p1 = rng.lognormal(0.0, 1.0, n)
    p2 = rng.lognormal(0.0, 1.0, n)
    w = (p1 / (p1 + p2)).astype(np.float32)
    w[rng.random(n) < excluded] = 0.0
    return w


# --------------------------------------------------------------------------
# Scenes for the GPU path sampler (plain data: primitives and cameras).
def furnace_scene(le=(1.0, 0.5, 0.25), albedo=(0.5, 0.6, 0.7)):
    """The closed furnace: the unit sphere at the origin, emitting le and
    reflecting diffusely with the given albedo; paths start at the centre."""
    return [{"kind": "sphere", "p": (0.0, 0.0, 0.0), "radius": 1.0, "albedo": albedo, "emission": le,
             "rough": 1.0}]


def box_scene(light=(4.0, 4.0, 4.0), albedo=(0.6, 0.6, 0.6)):
    """The tiny workload's open box [0, 1]^3 (floor, ceiling, back, left and
    right unit quads; sphere of radius 0.3 at (0.5, 0.3, 0.5)) with a
    0.5 x 0.5 emitter just below the ceiling; camera at (0.5, 0.5, -1.5)
    looking along +z, vertical field of view 40 degrees."""
    q = lambda p, u, v, a=albedo, r=1.0: {"kind": "quad", "p": p, "u": u, "v": v, "albedo": a, "rough": r}
    prims = [
        q((0.5, 0.0, 0.5), (0.5, 0.0, 0.0), (0.0, 0.0, 0.5)),         # floor
        q((0.5, 1.0, 0.5), (0.5, 0.0, 0.0), (0.0, 0.0, 0.5)),         # ceiling
        q((0.5, 0.5, 1.0), (0.5, 0.0, 0.0), (0.0, 0.5, 0.0)),         # back
        q((0.0, 0.5, 0.5), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5), (0.6, 0.2, 0.2)),  # left
        q((1.0, 0.5, 0.5), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5), (0.2, 0.6, 0.2), 0.2),  # right (glossy key)
        {"kind": "sphere", "p": (0.5, 0.3, 0.5), "radius": 0.3, "albedo": (0.7, 0.7, 0.7), "rough": 1.0},
        {"kind": "quad", "p": (0.5, 0.999, 0.5), "u": (0.25, 0.0, 0.0), "v": (0.0, 0.0, 0.25),
         "albedo": (0.0, 0.0, 0.0), "emission": light, "rough": 1.0},
    ]
    cam = {"pos": (0.5, 0.5, -1.5), "fwd": (0.0, 0.0, 1.0), "up": (0.0, 1.0, 0.0), "fov_y_deg": 40.0}
    return prims, cam


def square_light_scene(h=1.0, s=0.5, light=(3.0, 2.0, 1.0), albedo=(0.8, 0.5, 0.3)):
    """A large diffuse floor (y = 0) under a square emitter of half size s at
    height h centred above the origin; the camera looks straight down at the
    origin from half the height with a narrow field of view, so every first
    vertex is (all but) the floor point below the emitter's centre."""
    prims = [{"kind": "quad", "p": (0.0, 0.0, 0.0), "u": (50.0, 0.0, 0.0), "v": (0.0, 0.0, 50.0),
              "albedo": albedo, "rough": 1.0},
             {"kind": "quad", "p": (0.0, h, 0.0), "u": (s, 0.0, 0.0), "v": (0.0, 0.0, s),
              "albedo": (0.0, 0.0, 0.0), "emission": light, "rough": 1.0}]
    cam = {"pos": (0.0, 0.5 * h, 0.0), "fwd": (0.0, -1.0, 0.0), "up": (0.0, 0.0, 1.0), "fov_y_deg": 0.01}
    return prims, cam
