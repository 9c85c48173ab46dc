"""ctypes binding of libpsf.so (include/psf.h).

Argument marshalling only: every step of the hash path runs in the HIP
kernels of the shared library.  The functions keep the C names; ``Table`` is
a thin convenience wrapper that takes torch CUDA tensors (device memory) and
the current torch stream.  There is no CPU fallback: if the library is
missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsf.so")

PSF_OK, PSF_INVALID_ARGUMENT, PSF_OUT_OF_MEMORY, PSF_BUFFER_TOO_SMALL, PSF_HIP_ERROR, \
    PSF_NOT_SUPPORTED = range(6)
PSF_ALPHA_PAPER, PSF_ALPHA_CONST, PSF_ALPHA_LINEAR = 0, 1, 2
PSF_STATE_F32, PSF_STATE_F16, PSF_STATE_BF16, PSF_STATE_F16_EF, PSF_STATE_BF16_EF = 0, 1, 2, 3, 4
PSF_RESET_COUNTERS, PSF_RESET_CLEAR, PSF_RESET_STATS = 1, 2, 4
PSF_INSERT_AUTO, PSF_INSERT_DIRECT, PSF_INSERT_PARTITIONED = 0, 1, 2
PSF_FLAG_PROBE_STATS = 1
PSF_FLAG_TIMING = 2
PSF_FLAG_TRANSPOSE_RUNS = 4
PSF_FLAG_TRACK_VARIANCE = 8
PSF_FLAG_NO_ACCUMULATORS = 16
PSF_K_COUNT = 11
PSF_EST_CV, PSF_EST_BIASED = 0, 1
PSF_PRIM_QUAD, PSF_PRIM_SPHERE = 0, 1
PSF_PAYLOAD_RGB, PSF_PAYLOAD_SH2_YCOCG = 0, 1
PSF_PATHS_LO, PSF_PATHS_LOE = 0, 1
PSF_ORIGIN_CAMERA, PSF_ORIGIN_POINT = 0, 1

REC_FIELDS = ("px", "py", "pz", "nx", "ny", "nz", "ox", "oy", "oz", "r", "g", "b", "rough", "footprint",
              "weight")
QRY_FIELDS = ("px", "py", "pz", "nx", "ny", "nz", "ox", "oy", "oz", "rough", "footprint")
EST_FIELDS = ("px", "py", "pz", "nx", "ny", "nz", "oox", "ooy", "ooz", "oix", "oiy", "oiz", "rough",
              "gr", "gg", "gb", "wp", "footprint")


class PsfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"psf status {status}: {msg}")
        self.status = status


class psf_config(ctypes.Structure):
    _fields_ = [
        ("log2_slots", ctypes.c_uint32), ("max_probe", ctypes.c_uint32),
        ("cam", ctypes.c_float * 3), ("kappa", ctypes.c_float), ("e_min", ctypes.c_int32),
        ("max_level", ctypes.c_int32), ("normal_bins_log2", ctypes.c_int32),
        ("dir_bins_log2", ctypes.c_int32), ("rough_thr", ctypes.c_float),
        ("alpha_mode", ctypes.c_int32), ("alpha", ctypes.c_float), ("t_max", ctypes.c_float),
        ("state_dtype", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("insert_mode", ctypes.c_int32), ("part_log2", ctypes.c_uint32),
        ("max_batch", ctypes.c_uint64), ("bin_per", ctypes.c_uint32), ("weighted", ctypes.c_uint32),
        ("payload", ctypes.c_uint32),
    ]


class psf_records(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in REC_FIELDS]


class psf_queries(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in QRY_FIELDS]


class psf_estimate_args(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in EST_FIELDS]


class psf_step_args(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in ("le_r", "le_g", "le_b", "t_r", "t_g", "t_b")]


class psf_stats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64), ("skipped", ctypes.c_uint64), ("dropped", ctypes.c_uint64),
        ("coord_overflow", ctypes.c_uint64), ("touched_last", ctypes.c_uint64),
        ("touched_total", ctypes.c_uint64), ("updates", ctypes.c_uint64),
        ("saturated", ctypes.c_uint64), ("occupied", ctypes.c_uint64),
        ("probe_hist", ctypes.c_uint64 * 16),
    ]


class psf_session(ctypes.Structure):
    _fields_ = [
        ("table", ctypes.c_void_p), ("rec", psf_records), ("n", ctypes.c_uint64),
        ("q", psf_queries), ("nq", ctypes.c_uint64), ("d_out_rgb", ctypes.c_void_p),
        ("d_out_found", ctypes.c_void_p),
    ]


class psf_prim(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("p", ctypes.c_float * 3), ("u", ctypes.c_float * 3),
                ("v", ctypes.c_float * 3), ("albedo", ctypes.c_float * 3), ("emission", ctypes.c_float * 3),
                ("rough", ctypes.c_float)]


class psf_camera(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_float * 3), ("fwd", ctypes.c_float * 3), ("up", ctypes.c_float * 3),
                ("fov_y", ctypes.c_float), ("width", ctypes.c_uint32), ("height", ctypes.c_uint32),
                ("spp", ctypes.c_uint32)]


class psf_path_params(ctypes.Structure):
    _fields_ = [("verts", ctypes.c_uint32), ("mode", ctypes.c_int32), ("origin", ctypes.c_int32),
                ("seed", ctypes.c_uint32), ("frame", ctypes.c_uint32)]


PATH_X = ("px", "py", "pz", "nx", "ny", "nz", "ox", "oy", "oz", "rough")
PATH_NEXT = ("qx", "qy", "qz", "qnx", "qny", "qnz", "qox", "qoy", "qoz", "qrough")
PATH_FIELDS = PATH_X + PATH_NEXT + ("t_r", "t_g", "t_b", "le_r", "le_g", "le_b")


class psf_path_out(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in PATH_FIELDS]


# (name, restype, argtypes) of every exported function, in header order
_vp, _u64, _u32, _sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_size_t
_P = ctypes.POINTER
EXPORTS = [
    ("psf_table_bytes", _sz, [_P(psf_config)]),
    ("psf_create_table", ctypes.c_int, [_P(psf_config), _vp, _sz, _vp, _P(_vp)]),
    ("psf_destroy", ctypes.c_int, [_vp]),
    ("psf_insert_samples", ctypes.c_int, [_vp, _P(psf_records), _u64, _vp]),
    ("psf_temporal_update", ctypes.c_int, [_vp, _vp]),
    ("psf_query", ctypes.c_int, [_vp, _P(psf_queries), _u64, _vp, _vp, _vp]),
    ("psf_iterate", ctypes.c_int, [_vp, _P(psf_records), _u64, _P(psf_queries), _u64, _vp, _vp, _vp]),
    ("psf_query_levels", ctypes.c_int, [_vp, _P(psf_queries), _u64, _u32, _vp, _vp, _vp]),
    ("psf_progressive_step", ctypes.c_int, [_vp, _P(psf_records), _P(psf_queries), _P(psf_step_args), _u64,
                                            _vp, _vp]),
    ("psf_reset", ctypes.c_int, [_vp, _u32, _vp]),
    ("psf_reset_region", ctypes.c_int, [_vp, _P(ctypes.c_float), _P(ctypes.c_float), _vp]),
    ("psf_compute_keys", ctypes.c_int, [_vp, _P(psf_records), _u64, _vp, _vp]),
    ("psf_get_stats", ctypes.c_int, [_vp, _P(psf_stats), _vp]),
    ("psf_export_cells", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _u64, _P(_u64), _vp]),
    ("psf_export_cells_noalloc", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _u64, _P(_u64), _vp]),
    ("psf_export_sh_cells", ctypes.c_int, [_vp, _vp, _vp, _vp, _u64, _P(_u64), _vp]),
    ("psf_export_variance", ctypes.c_int, [_vp, _vp, _vp, _u64, _P(_u64), _vp]),
    ("psf_batch_create", ctypes.c_int, [_u32, _P(_vp)]),
    ("psf_batch_destroy", ctypes.c_int, [_vp]),
    ("psf_iterate_batch", ctypes.c_int, [_vp, _P(psf_session), _u32, _vp]),
    ("psf_estimate", ctypes.c_int, [_vp, _vp, _P(psf_estimate_args), _u64, ctypes.c_int32, ctypes.c_float,
                                    _vp, _vp, _vp]),
    ("psf_sample_paths", ctypes.c_int, [_vp, _u32, _P(psf_camera), _P(psf_path_params), _P(psf_path_out), _vp]),
    ("psf_philox", ctypes.c_int, [_vp, _vp, _u64, _vp, _vp]),
    ("psf_kernel_times", ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int]),
    ("psf_kernel_name", ctypes.c_char_p, [_u32]),
    ("psf_last_error", ctypes.c_char_p, []),
    ("psf_version", ctypes.c_char_p, []),
]

_lib = None


def load(path: str = LIB_PATH):
    """Load libpsf.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2005_07547_amd/build.py "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, res, args in EXPORTS:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != PSF_OK:
        raise PsfError(status, load().psf_last_error().decode())


def make_config(log2_slots=16, max_probe=64, cam=(0.0, 0.0, 0.0), kappa=0.0, e_min=0,
                max_level=15, normal_bins_log2=2, dir_bins_log2=3, rough_thr=0.3,
                alpha_mode=PSF_ALPHA_PAPER, alpha=0.2, t_max=5.0, state_dtype=PSF_STATE_F32,
                flags=0, insert_mode=PSF_INSERT_AUTO, part_log2=0, max_batch=0, bin_per=0,
                weighted=0, payload=0, **_ignored):
    c = psf_config()
    c.log2_slots, c.max_probe = int(log2_slots), int(max_probe)
    c.cam[:] = [float(x) for x in cam]
    c.kappa, c.e_min, c.max_level = float(kappa), int(e_min), int(max_level)
    c.normal_bins_log2, c.dir_bins_log2 = int(normal_bins_log2), int(dir_bins_log2)
    c.rough_thr, c.alpha_mode, c.alpha, c.t_max = float(rough_thr), int(alpha_mode), float(alpha), float(t_max)
    c.state_dtype, c.flags, c.insert_mode = int(state_dtype), int(flags), int(insert_mode)
    c.part_log2, c.max_batch, c.bin_per = int(part_log2), int(max_batch), int(bin_per)
    c.weighted = int(weighted)
    c.payload = int(payload)
    return c


def _ptr(t):
    if t is None:
        return None
    return t.data_ptr()


def _device_f32(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise TypeError(f"field {name} must be a contiguous float32 CUDA tensor")
    return t


def make_records(rec: dict):
    s = psf_records()
    for f in REC_FIELDS:
        v = rec.get(f)
        setattr(s, f, None if v is None else _ptr(_device_f32(v, f)))
    return s


def make_queries(q: dict):
    s = psf_queries()
    for f in QRY_FIELDS:
        v = q.get(f)
        setattr(s, f, None if v is None else _ptr(_device_f32(v, f)))
    return s


def current_stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Table:
    """One hash table in device memory (owned by a torch tensor)."""

    def __init__(self, **cfg):
        import torch
        self._lib = load()
        self.cfg = make_config(**cfg)
        nbytes = self._lib.psf_table_bytes(ctypes.byref(self.cfg))
        if nbytes == 0:
            raise PsfError(PSF_INVALID_ARGUMENT, self._lib.psf_last_error().decode())
        self.nbytes = int(nbytes)
        self.buffer = torch.empty(self.nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self.buffer.data_ptr()
        aligned = (base + 255) // 256 * 256
        h = ctypes.c_void_p()
        _check(self._lib.psf_create_table(ctypes.byref(self.cfg), ctypes.c_void_p(aligned),
                                          self.nbytes, current_stream(), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _check(self._lib.psf_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_slots(self):
        return 1 << self.cfg.log2_slots

    def insert(self, rec: dict, n: int | None = None):
        n = int(rec["px"].numel()) if n is None else int(n)
        r = make_records(rec)
        _check(self._lib.psf_insert_samples(self.handle, ctypes.byref(r), n, current_stream()))

    def update(self):
        _check(self._lib.psf_temporal_update(self.handle, current_stream()))

    def query(self, q: dict, n: int | None = None, out=None, found=None):
        import torch
        n = int(q["px"].numel()) if n is None else int(n)
        if out is None:
            out = torch.empty((3, n), dtype=torch.float32, device="cuda")
        if found is None:
            found = torch.empty(n, dtype=torch.uint8, device="cuda")
        qs = make_queries(q)
        _check(self._lib.psf_query(self.handle, ctypes.byref(qs), n, ctypes.c_void_p(_ptr(out)),
                                   ctypes.c_void_p(_ptr(found)), current_stream()))
        return out, found

    def query_levels(self, q: dict, levels_up: int, n: int | None = None, out=None, level=None):
        """psf_query_levels: lookup falling back to coarser levels; returns
        (out (3, n), level (n,): 0 none, else 1 + levels above)."""
        import torch
        n = int(q["px"].numel()) if n is None else int(n)
        if out is None:
            out = torch.empty((3, n), dtype=torch.float32, device="cuda")
        if level is None:
            level = torch.empty(n, dtype=torch.uint8, device="cuda")
        qs = make_queries(q)
        _check(self._lib.psf_query_levels(self.handle, ctypes.byref(qs), n, int(levels_up),
                                          ctypes.c_void_p(_ptr(out)), ctypes.c_void_p(_ptr(level)),
                                          current_stream()))
        return out, level

    def iterate(self, rec: dict, q: dict | None = None, out=None, found=None):
        import torch
        n = int(rec["px"].numel())
        q = rec if q is None else q
        nq = int(q["px"].numel())
        if out is None:
            out = torch.empty((3, nq), dtype=torch.float32, device="cuda")
        if found is None:
            found = torch.empty(nq, dtype=torch.uint8, device="cuda")
        r = make_records(rec)
        qs = make_queries(q)
        _check(self._lib.psf_iterate(self.handle, ctypes.byref(r), n, ctypes.byref(qs), nq,
                                     ctypes.c_void_p(_ptr(out)), ctypes.c_void_p(_ptr(found)),
                                     current_stream()))
        return out, found

    def progressive_step(self, x: dict, nxt: dict, tput, le=None, out=None):
        """psf_progressive_step: samples L_e + L~(next) * tput at the vertices
        x (their r, g, b are not used), inserted and blended.  tput and le are
        sequences of three device arrays (le None: no emission).  Returns the
        samples (3, n)."""
        import torch
        n = int(x["px"].numel())
        if out is None:
            out = torch.empty((3, n), dtype=torch.float32, device="cuda")
        xs = make_records({k: v for k, v in x.items() if k not in ("r", "g", "b")})
        qs = make_queries(nxt)
        a = psf_step_args()
        for f, v in zip(("t_r", "t_g", "t_b"), tput):
            setattr(a, f, _ptr(_device_f32(v, f)))
        if le is not None:
            for f, v in zip(("le_r", "le_g", "le_b"), le):
                setattr(a, f, _ptr(_device_f32(v, f)))
        _check(self._lib.psf_progressive_step(self.handle, ctypes.byref(xs), ctypes.byref(qs), ctypes.byref(a), n,
                                              ctypes.c_void_p(_ptr(out)), current_stream()))
        return out

    def reset_region(self, lo, hi):
        """psf_reset_region: zero c_old of every cell meeting the box [lo, hi]."""
        a = (ctypes.c_float * 3)(*[float(v) for v in lo])
        b = (ctypes.c_float * 3)(*[float(v) for v in hi])
        _check(self._lib.psf_reset_region(self.handle, a, b, current_stream()))

    def keys(self, rec: dict):
        import torch
        n = int(rec["px"].numel())
        out = torch.empty(n, dtype=torch.int64, device="cuda")
        r = make_records({k: v for k, v in rec.items() if k in REC_FIELDS})
        _check(self._lib.psf_compute_keys(self.handle, ctypes.byref(r), n,
                                          ctypes.c_void_p(_ptr(out)), current_stream()))
        return out

    def reset(self, what: int):
        _check(self._lib.psf_reset(self.handle, int(what), current_stream()))

    def stats(self) -> dict:
        s = psf_stats()
        _check(self._lib.psf_get_stats(self.handle, ctypes.byref(s), current_stream()))
        d = {f: getattr(s, f) for f, _ in psf_stats._fields_ if f != "probe_hist"}
        d["probe_hist"] = list(s.probe_hist)
        return d

    def kernel_times(self, reset=False) -> dict:
        """{kernel name: (launches, total ms)} for tables made with PSF_FLAG_TIMING."""
        import numpy as np
        launches = np.zeros(PSF_K_COUNT, dtype=np.uint64)
        ms = np.zeros(PSF_K_COUNT, dtype=np.float64)
        _check(self._lib.psf_kernel_times(self.handle, launches.ctypes.data, ms.ctypes.data,
                                          1 if reset else 0))
        return {self._lib.psf_kernel_name(k).decode(): (int(launches[k]), float(ms[k]))
                for k in range(PSF_K_COUNT) if launches[k]}

    def export_variance(self):
        return export_variance(self)

    def export(self, noalloc: bool = False):
        """Occupied cells as numpy arrays: keys (uint64), n_new, c_old (uint32
        counts; float32 weight sums for a weighted table), L (3 x C).
        noalloc: through psf_export_cells_noalloc (the library's fixed device
        array instead of a per-call allocation)."""
        import numpy as np
        st = self.stats()
        cap = max(1, int(st["occupied"]))
        keys = np.zeros(cap, dtype=np.uint64)
        n_new = np.zeros(cap, dtype=np.uint32)
        c_old = np.zeros(cap, dtype=np.uint32)
        rgb = np.zeros((3, cap), dtype=np.float32)
        count = ctypes.c_uint64()
        fn = self._lib.psf_export_cells_noalloc if noalloc else self._lib.psf_export_cells
        _check(fn(self.handle, keys.ctypes.data, n_new.ctypes.data, c_old.ctypes.data, rgb.ctypes.data, cap,
                  ctypes.byref(count), current_stream()))
        c = int(count.value)
        order = np.argsort(keys[:c], kind="stable")
        if self.cfg.weighted:
            n_new, c_old = n_new.view(np.float32), c_old.view(np.float32)
        return {"keys": keys[:c][order], "n_new": n_new[:c][order], "c_old": c_old[:c][order],
                "L": rgb[:, :c][:, order]}


def export_sh(t):
    """Occupied cells of an SH payload table: keys (uint64), c_old (uint32
    counts; float32 weight sums for a weighted table), coeff (6 x C float32:
    four luminance SH coefficients, Co, Cg), sorted by key."""
    import numpy as np
    st = t.stats()
    cap = max(1, int(st["occupied"]))
    keys = np.zeros(cap, dtype=np.uint64)
    c_old = np.zeros(cap, dtype=np.uint32)
    coeff = np.zeros((6, cap), dtype=np.float32)
    count = ctypes.c_uint64()
    _check(t._lib.psf_export_sh_cells(t.handle, keys.ctypes.data, c_old.ctypes.data, coeff.ctypes.data, cap,
                                      ctypes.byref(count), current_stream()))
    c = int(count.value)
    order = np.argsort(keys[:c], kind="stable")
    if t.cfg.weighted:
        c_old = c_old.view(np.float32)
    return {"keys": keys[:c][order], "c_old": c_old[:c][order], "coeff": coeff[:, :c][:, order]}


def export_variance(t):
    """Occupied cells of a table created with PSF_FLAG_TRACK_VARIANCE: keys
    (uint64) and each cell's luminance variance (float32), sorted by key."""
    import numpy as np
    st = t.stats()
    cap = max(1, int(st["occupied"]))
    keys = np.zeros(cap, dtype=np.uint64)
    var = np.zeros(cap, dtype=np.float32)
    count = ctypes.c_uint64()
    _check(t._lib.psf_export_variance(t.handle, keys.ctypes.data, var.ctypes.data, cap, ctypes.byref(count),
                                      current_stream()))
    c = int(count.value)
    order = np.argsort(keys[:c], kind="stable")
    return keys[:c][order], var[:c][order]


def estimate(t_oe, t_fli, a: dict, mode: int, param: float, out=None, applied=None):
    """psf_estimate: control-variate (mode PSF_EST_CV, param beta) or biased
    (PSF_EST_BIASED, param gamma) estimate at every vertex of a (device
    float32 arrays keyed as EST_FIELDS; rough may be None).  Returns
    (out (3, n), applied (n,))."""
    import torch
    n = int(a["px"].numel())
    if out is None:
        out = torch.empty((3, n), dtype=torch.float32, device="cuda")
    if applied is None:
        applied = torch.empty(n, dtype=torch.uint8, device="cuda")
    s = psf_estimate_args()
    for f in EST_FIELDS:
        v = a.get(f)
        setattr(s, f, None if v is None else _ptr(_device_f32(v, f)))
    lib = load()
    _check(lib.psf_estimate(t_oe.handle, t_fli.handle, ctypes.byref(s), n, int(mode), float(param),
                            ctypes.c_void_p(_ptr(out)), ctypes.c_void_p(_ptr(applied)), current_stream()))
    return out, applied


class Batch:
    """A batch context (psf_batch) for batched iterations over several tables."""

    def __init__(self, max_sessions: int = 64):
        self._lib = load()
        h = ctypes.c_void_p()
        _check(self._lib.psf_batch_create(int(max_sessions), ctypes.byref(h)))
        self.handle = h
        self.max_sessions = int(max_sessions)

    def close(self):
        if getattr(self, "handle", None):
            _check(self._lib.psf_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def iterate(self, tables, recs, queries=None, outs=None, founds=None):
        """One batched iteration; queries default to the records.  Returns
        the (out, found) pairs."""
        import torch
        k = len(tables)
        queries = recs if queries is None else queries
        if outs is None:
            outs = [torch.empty((3, int(q["px"].numel())), dtype=torch.float32, device="cuda")
                    for q in queries]
        if founds is None:
            founds = [torch.empty(int(q["px"].numel()), dtype=torch.uint8, device="cuda")
                      for q in queries]
        arr = (psf_session * k)()
        for i in range(k):
            s = arr[i]
            s.table = tables[i].handle
            s.rec = make_records(recs[i])
            s.n = int(recs[i]["px"].numel())
            s.q = make_queries(queries[i])
            s.nq = int(queries[i]["px"].numel())
            s.d_out_rgb = _ptr(outs[i])
            s.d_out_found = _ptr(founds[i]) if founds[i] is not None else None
        _check(self._lib.psf_iterate_batch(self.handle, arr, k, current_stream()))
        return list(zip(outs, founds))


def version() -> str:
    return load().psf_version().decode()


class Scene:
    """Scene primitives for psf_sample_paths, copied once to device memory.
    prims: dicts with kind ("quad" or "sphere"), p, u, v (quad half edges;
    sphere: radius), albedo, emission, rough."""

    def __init__(self, prims):
        import torch
        arr = (psf_prim * max(1, len(prims)))()
        for i, q in enumerate(prims):
            arr[i].kind = PSF_PRIM_SPHERE if q["kind"] == "sphere" else PSF_PRIM_QUAD
            arr[i].p[:] = [float(c) for c in q["p"]]
            if q["kind"] == "sphere":
                arr[i].u[:] = [float(q["radius"]), 0.0, 0.0]
            else:
                arr[i].u[:] = [float(c) for c in q["u"]]
                arr[i].v[:] = [float(c) for c in q["v"]]
            arr[i].albedo[:] = [float(c) for c in q.get("albedo", (0.0, 0.0, 0.0))]
            arr[i].emission[:] = [float(c) for c in q.get("emission", (0.0, 0.0, 0.0))]
            arr[i].rough = float(q.get("rough", 1.0))
        raw = bytes(arr)
        self.n = len(prims)
        self.dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).cuda()


def camera(pos, fwd, up, fov_y_deg, width, height, spp=1):
    c = psf_camera()
    c.pos[:], c.fwd[:], c.up[:] = [float(v) for v in pos], [float(v) for v in fwd], [float(v) for v in up]
    import math
    c.fov_y = math.radians(float(fov_y_deg))
    c.width, c.height, c.spp = int(width), int(height), int(spp)
    return c


def sample_paths(scene: Scene, cam, verts: int, mode: int = PSF_PATHS_LO, origin: int = PSF_ORIGIN_CAMERA,
                 seed: int = 1, frame: int = 0, out: dict | None = None):
    """psf_sample_paths: returns (x, next, t, le) -- the vertices as a record
    dict (without values), their next vertices as a query dict, and the
    throughput and emission triples, all device float32 arrays of
    paths * verts entries (depth-major).  out: a dict of PATH_FIELDS arrays
    to reuse."""
    import torch
    n = int(cam.width) * int(cam.height) * int(cam.spp) * int(verts)
    if out is None:
        out = {f: torch.empty(n, dtype=torch.float32, device="cuda") for f in PATH_FIELDS}
    po = psf_path_out()
    for f in PATH_FIELDS:
        setattr(po, f, _ptr(_device_f32(out[f], f)))
    prm = psf_path_params(int(verts), int(mode), int(origin), int(seed) & 0xFFFFFFFF, int(frame) & 0xFFFFFFFF)
    _check(load().psf_sample_paths(ctypes.c_void_p(scene.dev.data_ptr()), scene.n, ctypes.byref(cam),
                                   ctypes.byref(prm), ctypes.byref(po), current_stream()))
    x = {k: out[k] for k in PATH_X}
    nxt = {"px": out["qx"], "py": out["qy"], "pz": out["qz"], "nx": out["qnx"], "ny": out["qny"],
           "nz": out["qnz"], "ox": out["qox"], "oy": out["qoy"], "oz": out["qoz"], "rough": out["qrough"]}
    return x, nxt, (out["t_r"], out["t_g"], out["t_b"]), (out["le_r"], out["le_g"], out["le_b"])


def philox(ctr, key):
    """psf_philox on the device: ctr (n, 4) and key (n, 2) uint32 numpy
    arrays; returns (n, 4) uint32."""
    import numpy as np
    import torch
    c = torch.from_numpy(np.ascontiguousarray(ctr, dtype=np.uint32).view(np.int32)).cuda()
    k = torch.from_numpy(np.ascontiguousarray(key, dtype=np.uint32).view(np.int32)).cuda()
    n = int(c.shape[0])
    o = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    _check(load().psf_philox(ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(k.data_ptr()), n,
                             ctypes.c_void_p(o.data_ptr()), current_stream()))
    return o.cpu().numpy().view(np.uint32)

