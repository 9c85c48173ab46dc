"""Seeded synthetic vertex-record generator (inputs only).

Both the oracle and the GPU library consume what this module produces; it
holds none of the filtering arithmetic.  The C++ source ``scenegen.cpp`` traces
procedural scenes (an open box with a sphere, or random quads and spheres) and
emits depth-major SoA float32 records: position, oriented normal, outgoing
direction, RGB sample value and roughness.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scenegen.cpp")
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

FIELDS = ("px", "py", "pz", "nx", "ny", "nz", "ox", "oy", "oz", "r", "g", "b", "rough")
QUERY_FIELDS = ("px", "py", "pz", "nx", "ny", "nz", "ox", "oy", "oz", "rough")


class SynthParams(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("spp", ctypes.c_int32),
        ("verts", ctypes.c_int32), ("seed", ctypes.c_uint32),
        ("cam", ctypes.c_float * 3), ("look", ctypes.c_float * 3), ("fov_y_deg", ctypes.c_float),
        ("field", ctypes.c_int32), ("noise", ctypes.c_int32), ("sigma", ctypes.c_float),
        ("field_scale", ctypes.c_float), ("amp", ctypes.c_float * 3),
        ("lin_a", ctypes.c_float * 9), ("lin_b", ctypes.c_float * 3),
        ("light", ctypes.c_float * 3), ("glossy_thr", ctypes.c_float),
        ("glossy_lobe", ctypes.c_int32),
    ]


class SynthStats(ctypes.Structure):
    _fields_ = [("restarts", ctypes.c_uint64), ("fallbacks", ctypes.c_uint64),
                ("glossy", ctypes.c_uint64)]


def build(force: bool = True) -> str:
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-Wall",
                    _SRC, "-o", tmp], check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.synth_scene_create.restype = ctypes.c_void_p
    lib.synth_scene_create.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_float]
    lib.synth_scene_destroy.argtypes = [ctypes.c_void_p]
    lib.synth_generate.restype = ctypes.c_int
    lib.synth_generate.argtypes = [ctypes.c_void_p, ctypes.POINTER(SynthParams), ctypes.c_uint32,
                                   ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                   ctypes.POINTER(SynthStats)]
    lib.synth_philox.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    _lib = lib
    return lib


def philox4x32_10(ctr, key):
    lib = _load()
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib.synth_philox(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return o


def default_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


class Scene:
    BOX, RANDOM = 0, 1

    def __init__(self, kind: int, seed: int = 0, n_quads: int = 64, n_spheres: int = 16,
                 glossy_frac: float = -1.0):
        self._lib = _load()
        self.kind = kind
        self._h = self._lib.synth_scene_create(int(kind), int(seed) & 0xFFFFFFFF, int(n_quads),
                                               int(n_spheres), float(glossy_frac))

    def __del__(self):
        try:
            if self._h:
                self._lib.synth_scene_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def generate(self, prm: dict, iteration: int, nthreads: int | None = None, out=None):
        """Records of one iteration as a dict of float32 arrays (depth-major).

        ``out`` may supply the 13 destination arrays (e.g. pinned buffers)."""
        p = SynthParams()
        p.width, p.height = int(prm["width"]), int(prm["height"])
        p.spp, p.verts = int(prm.get("spp", 1)), int(prm["verts"])
        p.seed = int(prm.get("seed", 0)) & 0xFFFFFFFF
        p.cam[:] = [float(x) for x in prm["cam"]]
        p.look[:] = [float(x) for x in prm.get("look", (0.0, 0.0, 1.0))]
        p.fov_y_deg = float(prm["fov_y_deg"])
        p.field = int(prm.get("field", 0))
        p.noise = int(prm.get("noise", 1))
        p.sigma = float(prm.get("sigma", 2.0))
        p.field_scale = float(prm.get("field_scale", 1.0))
        p.amp[:] = [float(x) for x in prm.get("amp", (1.0, 0.8, 0.6))]
        p.lin_a[:] = [float(x) for x in prm.get("lin_a", (0.0,) * 9)]
        p.lin_b[:] = [float(x) for x in prm.get("lin_b", (1.0, 1.0, 1.0))]
        p.light[:] = [float(x) for x in prm.get("light", (0.3, 0.8, -0.5))]
        p.glossy_thr = float(prm.get("glossy_thr", 0.3))
        p.glossy_lobe = int(prm.get("glossy_lobe", 1))
        n = p.width * p.height * p.spp * p.verts
        if out is None:
            out = {k: np.empty(n, dtype=np.float32) for k in FIELDS}
        ptrs = (ctypes.c_void_p * 13)(*[out[k].ctypes.data for k in FIELDS])
        st = SynthStats()
        rc = self._lib.synth_generate(self._h, ctypes.byref(p), int(iteration) & 0xFFFFFFFF, ptrs,
                                      int(nthreads or default_threads()), ctypes.byref(st))
        if rc != 0:
            raise ValueError("synth_generate rejected its arguments")
        self.last_stats = {"restarts": st.restarts, "fallbacks": st.fallbacks, "glossy": st.glossy}
        return out
