"""CPU oracle for the progressive spatio-temporal filtering hash path.

TEST INFRASTRUCTURE ONLY: tests, the smoke entry point and the benchmark's
CPU-baseline leg may use it; the library never does.  The arithmetic lives in
``psf_oracle.cpp`` (binary64, ``std::map``); this module only marshals numpy
arrays through ctypes.  It imports nothing from the HIP package.

Sections followed: Sec. 2.1 Eq. 5-6 (counters and weighted means per basis
function, with optional per-record MIS weights: Sec. 2.5), Sec. 2.4 Eq. 10-11
(temporal blend, counter reset), Sec. 2.6 (spatio-directional hashing; the key specification is this project's, written
out in ``psf_oracle.cpp``), Algorithm 1 (lookups read the last blended state),
and, for the two-field estimators, Sec. 2.5, Sec. 4.2 (Eq. 25) and Sec. 5
(Eq. 28) in ``estimate`` below (plain numpy in binary64 over the lookups);
``ShOracle`` holds the two-band SH YCoCg cell payload of Sec. 2.6.  Every
cell also keeps a luminance variance around its approximant (the paper
defines none; the reading is stated in ``psf_oracle.cpp`` and pinned in
``tests/test_oracle_variance.py``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libpsf_oracle.so")
_lib = None

ALPHA_PAPER, ALPHA_CONST, ALPHA_LINEAR = 0, 1, 2
RESET_COUNTERS, RESET_CLEAR = 1, 2
FIELDS = ("px", "py", "pz", "nx", "ny", "nz", "ox", "oy", "oz", "r", "g", "b", "rough", "footprint",
          "weight")


class _Records(ctypes.Structure):
    _fields_ = [("f", ctypes.c_void_p * 15)]


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (no GPU code involved)."""
    import importlib
    return importlib.import_module(__name__ + ".build").build(force=force)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    lib.orc_create.restype = vp
    lib.orc_create.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_float, ctypes.c_int,
                               ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_float,
                               ctypes.c_int, ctypes.c_float, ctypes.c_float]
    lib.orc_destroy.argtypes = [vp]
    lib.orc_keys.argtypes = [vp, ctypes.POINTER(_Records), u64, vp, vp]
    lib.orc_set_filter.argtypes = [vp, vp, u64]
    lib.orc_insert.argtypes = [vp, ctypes.POINTER(_Records), u64]
    lib.orc_update.restype = u64
    lib.orc_update.argtypes = [vp]
    lib.orc_query.argtypes = [vp, ctypes.POINTER(_Records), u64, vp, vp]
    lib.orc_reset.argtypes = [vp, u32]
    lib.orc_query_levels.argtypes = [vp, ctypes.POINTER(_Records), u64, ctypes.c_int, vp, vp]
    lib.orc_reset_region.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]
    lib.orc_count.restype = u64
    lib.orc_count.argtypes = [vp]
    lib.orc_export.restype = u64
    lib.orc_export.argtypes = [vp, vp, vp, vp, vp, vp, u64]
    lib.orc_counters.argtypes = [vp, vp, vp, vp]
    lib.orc_export_variance.restype = u64
    lib.orc_export_variance.argtypes = [vp, vp, vp, u64]
    lib.orc_sharded_export_variance.restype = u64
    lib.orc_sharded_export_variance.argtypes = [vp, vp, vp, u64]
    lib.orc_sharded_create.restype = vp
    lib.orc_sharded_create.argtypes = [u32] + lib.orc_create.argtypes
    lib.orc_sharded_destroy.argtypes = [vp]
    lib.orc_sharded_set_filter.argtypes = [vp, vp, u64]
    lib.orc_sharded_insert.argtypes = [vp, ctypes.POINTER(_Records), u64]
    lib.orc_sharded_update.restype = u64
    lib.orc_sharded_update.argtypes = [vp]
    lib.orc_sharded_query.argtypes = [vp, ctypes.POINTER(_Records), u64, vp, vp]
    lib.orc_sharded_count.restype = u64
    lib.orc_sharded_count.argtypes = [vp]
    lib.orc_sharded_export.restype = u64
    lib.orc_sharded_export.argtypes = [vp, vp, vp, vp, vp, vp, u64]
    lib.orc_sharded_counters.argtypes = [vp, vp, vp, vp]
    lib.orc_sh_create.restype = vp
    lib.orc_sh_create.argtypes = lib.orc_create.argtypes
    lib.orc_sh_destroy.argtypes = [vp]
    lib.orc_sh_insert.argtypes = [vp, ctypes.POINTER(_Records), u64]
    lib.orc_sh_update.restype = u64
    lib.orc_sh_update.argtypes = [vp]
    lib.orc_sh_query.argtypes = [vp, ctypes.POINTER(_Records), u64, vp, vp]
    lib.orc_sh_count.restype = u64
    lib.orc_sh_count.argtypes = [vp]
    lib.orc_sh_export.restype = u64
    lib.orc_sh_export.argtypes = [vp, vp, vp, vp, u64]
    _lib = lib
    return lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


class _Pack:
    """Holds contiguous float32 copies alive while the C call runs."""

    def __init__(self, rec: dict, n: int):
        self.keep = []
        self.s = _Records()
        for i, name in enumerate(FIELDS):
            a = rec.get(name)
            if a is None:
                self.s.f[i] = None
                continue
            a = _f32(a)
            if a.shape[0] < n:
                raise ValueError(f"field {name} shorter than n")
            self.keep.append(a)
            self.s.f[i] = a.ctypes.data


class Oracle:
    """One hash table, mirrored in binary64 on the host."""

    def __init__(self, cam=(0.0, 0.0, 0.0), kappa=0.0, e_min=0, max_level=15,
                 normal_bins_log2=2, dir_bins_log2=3, rough_thr=0.3,
                 alpha_mode=ALPHA_PAPER, alpha=0.2, t_max=5.0, weighted=0, **_ignored):
        # weighted: records may carry MIS weights and the exported counters
        # are float64 weight sums; otherwise they are integer counts (uint64)
        # and a weight array is refused, as the library refuses it
        self.weighted = bool(weighted)
        self._lib = _load()
        cam_arr = (ctypes.c_float * 3)(*[float(c) for c in cam])
        self._h = self._lib.orc_create(cam_arr, float(np.float32(kappa)), int(e_min),
                                       int(max_level), int(normal_bins_log2),
                                       int(dir_bins_log2), float(np.float32(rough_thr)),
                                       int(alpha_mode), float(np.float32(alpha)),
                                       float(np.float32(t_max)))

    def close(self):
        if self._h:
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _n(rec):
        return int(np.asarray(rec["px"]).shape[0])

    def keys(self, rec):
        n = self._n(rec)
        p = _Pack(rec, n)
        out = np.empty(n, dtype=np.uint64)
        ovf = np.empty(n, dtype=np.uint8)
        self._lib.orc_keys(self._h, ctypes.byref(p.s), n, out.ctypes.data, ovf.ctypes.data)
        return out, ovf

    def set_filter(self, keys):
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        self._lib.orc_set_filter(self._h, k.ctypes.data if k.size else None, int(k.size))

    def insert(self, rec):
        if rec.get("weight") is not None and not self.weighted:
            raise ValueError("weights need a weighted table")
        n = self._n(rec)
        p = _Pack(rec, n)
        self._lib.orc_insert(self._h, ctypes.byref(p.s), n)

    def update(self) -> int:
        return int(self._lib.orc_update(self._h))

    def query(self, rec):
        n = self._n(rec)
        p = _Pack(rec, n)
        out = np.zeros((3, n), dtype=np.float64)
        found = np.zeros(n, dtype=np.uint8)
        self._lib.orc_query(self._h, ctypes.byref(p.s), n, out.ctypes.data, found.ctypes.data)
        return out, found

    def query_levels(self, rec, up: int):
        """Lookup falling back to up to `up` coarser levels (Sec. 2.3);
        returns (rgb (3, n), level (n,): 0 none, else 1 + levels above)."""
        n = self._n(rec)
        p = _Pack(rec, n)
        out = np.zeros((3, n), dtype=np.float64)
        lv = np.zeros(n, dtype=np.uint8)
        self._lib.orc_query_levels(self._h, ctypes.byref(p.s), n, int(up), out.ctypes.data, lv.ctypes.data)
        return out, lv

    def reset(self, what: int):
        self._lib.orc_reset(self._h, int(what))

    def reset_region(self, lo, hi):
        """Zero c_old of every cell whose box meets [lo, hi] (Sec. 2.4, local
        counter reset)."""
        a = (ctypes.c_float * 3)(*[float(np.float32(v)) for v in lo])
        b = (ctypes.c_float * 3)(*[float(np.float32(v)) for v in hi])
        self._lib.orc_reset_region(self._h, a, b)

    def count(self) -> int:
        return int(self._lib.orc_count(self._h))

    def export(self):
        cap = self.count()
        keys = np.zeros(cap, dtype=np.uint64)
        n_new = np.zeros(cap, dtype=np.float64)
        c_old = np.zeros(cap, dtype=np.float64)
        L = np.zeros((3, cap), dtype=np.float64)
        s = np.zeros((3, cap), dtype=np.float64)
        if cap:
            got = self._lib.orc_export(self._h, keys.ctypes.data, n_new.ctypes.data,
                                       c_old.ctypes.data, L.ctypes.data, s.ctypes.data, cap)
            assert got == cap
        if not self.weighted:
            # unit weights: the counters are integers, exact in binary64
            n_new, c_old = n_new.astype(np.uint64), c_old.astype(np.uint64)
        return {"keys": keys, "n_new": n_new, "c_old": c_old, "L": L, "s": s}

    def export_variance(self):
        """Keys (ascending) and each cell's luminance variance around its
        approximant (the mixture variance under the blend's weights)."""
        cap = self.count()
        keys = np.zeros(cap, dtype=np.uint64)
        var = np.zeros(cap, dtype=np.float64)
        if cap:
            assert self._export_variance(keys.ctypes.data, var.ctypes.data, cap) == cap
        return keys, var

    def _export_variance(self, keys, var, cap):
        return self._lib.orc_export_variance(self._h, keys, var, cap)

    def counters(self):
        a = np.zeros(3, dtype=np.uint64)
        self._lib.orc_counters(self._h, a[0:].ctypes.data, a[1:].ctypes.data, a[2:].ctypes.data)
        return {"skipped": int(a[0]), "coord_overflow": int(a[1]), "inserted": int(a[2])}


class ShardedOracle(Oracle):
    """The same table split by key over `threads` host threads (one std::map
    per thread; a cell's samples arrive in array order on its own thread, so
    the results equal the single-threaded oracle's bit for bit).  Supports
    insert, update, query, set_filter, export, export_variance, count,
    counters and keys."""

    def __init__(self, threads: int, cam=(0.0, 0.0, 0.0), kappa=0.0, e_min=0, max_level=15,
                 normal_bins_log2=2, dir_bins_log2=3, rough_thr=0.3,
                 alpha_mode=ALPHA_PAPER, alpha=0.2, t_max=5.0, weighted=0, **_ignored):
        # a single oracle of the same configuration answers keys()
        super().__init__(cam=cam, kappa=kappa, e_min=e_min, max_level=max_level,
                         normal_bins_log2=normal_bins_log2, dir_bins_log2=dir_bins_log2, rough_thr=rough_thr,
                         alpha_mode=alpha_mode, alpha=alpha, t_max=t_max, weighted=weighted)
        self.threads = max(1, int(threads))
        cam_arr = (ctypes.c_float * 3)(*[float(c) for c in cam])
        self._s = self._lib.orc_sharded_create(self.threads, cam_arr, float(np.float32(kappa)), int(e_min),
                                               int(max_level), int(normal_bins_log2), int(dir_bins_log2),
                                               float(np.float32(rough_thr)), int(alpha_mode),
                                               float(np.float32(alpha)), float(np.float32(t_max)))

    def close(self):
        if getattr(self, "_s", None):
            self._lib.orc_sharded_destroy(self._s)
            self._s = None
        super().close()

    def set_filter(self, keys):
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        self._lib.orc_sharded_set_filter(self._s, k.ctypes.data if k.size else None, int(k.size))

    def insert(self, rec):
        if rec.get("weight") is not None and not self.weighted:
            raise ValueError("weights need a weighted table")
        n = self._n(rec)
        p = _Pack(rec, n)
        self._lib.orc_sharded_insert(self._s, ctypes.byref(p.s), n)

    def update(self) -> int:
        return int(self._lib.orc_sharded_update(self._s))

    def query(self, rec):
        n = self._n(rec)
        p = _Pack(rec, n)
        out = np.zeros((3, n), dtype=np.float64)
        found = np.zeros(n, dtype=np.uint8)
        self._lib.orc_sharded_query(self._s, ctypes.byref(p.s), n, out.ctypes.data, found.ctypes.data)
        return out, found

    def count(self) -> int:
        return int(self._lib.orc_sharded_count(self._s))

    def export(self):
        cap = self.count()
        keys = np.zeros(cap, dtype=np.uint64)
        n_new = np.zeros(cap, dtype=np.float64)
        c_old = np.zeros(cap, dtype=np.float64)
        L = np.zeros((3, cap), dtype=np.float64)
        s = np.zeros((3, cap), dtype=np.float64)
        if cap:
            got = self._lib.orc_sharded_export(self._s, keys.ctypes.data, n_new.ctypes.data, c_old.ctypes.data,
                                               L.ctypes.data, s.ctypes.data, cap)
            assert got == cap
        if not self.weighted:
            n_new, c_old = n_new.astype(np.uint64), c_old.astype(np.uint64)
        return {"keys": keys, "n_new": n_new, "c_old": c_old, "L": L, "s": s}

    def _export_variance(self, keys, var, cap):
        return self._lib.orc_sharded_export_variance(self._s, keys, var, cap)

    def counters(self):
        a = np.zeros(3, dtype=np.uint64)
        self._lib.orc_sharded_counters(self._s, a[0:].ctypes.data, a[1:].ctypes.data, a[2:].ctypes.data)
        return {"skipped": int(a[0]), "coord_overflow": int(a[1]), "inserted": int(a[2])}

    def query_levels(self, rec, up: int):
        raise NotImplementedError("the sharded oracle answers plain lookups only")

    def reset(self, what: int):
        raise NotImplementedError("the sharded oracle has no reset")

    def reset_region(self, lo, hi):
        raise NotImplementedError("the sharded oracle has no reset")


class ShOracle:
    """A table whose cells hold the two-band SH luminance and the YCoCg
    chroma (Sec. 2.6; the reading is written out in psf_oracle.cpp): per
    frame a ridge least-squares fit of the four luminance coefficients over
    the samples' normals and the chroma means, blended by Eq. 10-11; a
    lookup evaluates the luminance at the query's normal.  Binary64."""

    def __init__(self, cam=(0.0, 0.0, 0.0), kappa=0.0, e_min=0, max_level=15, normal_bins_log2=0,
                 dir_bins_log2=3, rough_thr=0.3, alpha_mode=ALPHA_PAPER, alpha=0.2, t_max=5.0, **_ignored):
        self._lib = _load()
        cam_arr = (ctypes.c_float * 3)(*[float(c) for c in cam])
        self._h = self._lib.orc_sh_create(cam_arr, float(np.float32(kappa)), int(e_min), int(max_level),
                                          int(normal_bins_log2), int(dir_bins_log2), float(np.float32(rough_thr)),
                                          int(alpha_mode), float(np.float32(alpha)), float(np.float32(t_max)))

    def close(self):
        if self._h:
            self._lib.orc_sh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def insert(self, rec):
        n = Oracle._n(rec)
        p = _Pack(rec, n)
        self._lib.orc_sh_insert(self._h, ctypes.byref(p.s), n)

    def update(self) -> int:
        return int(self._lib.orc_sh_update(self._h))

    def query(self, rec):
        n = Oracle._n(rec)
        p = _Pack(rec, n)
        out = np.zeros((3, n), dtype=np.float64)
        found = np.zeros(n, dtype=np.uint8)
        self._lib.orc_sh_query(self._h, ctypes.byref(p.s), n, out.ctypes.data, found.ctypes.data)
        return out, found

    def export(self):
        cap = int(self._lib.orc_sh_count(self._h))
        keys = np.zeros(cap, dtype=np.uint64)
        c_old = np.zeros(cap, dtype=np.float64)
        coeff = np.zeros((6, cap), dtype=np.float64)
        if cap:
            got = self._lib.orc_sh_export(self._h, keys.ctypes.data, c_old.ctypes.data, coeff.ctypes.data, cap)
            assert got == cap
        return {"keys": keys, "c_old": c_old, "coeff": coeff}


# --------------------------------------------------------------------------
# Estimators on two fields (Sec. 4.2, Eq. 25; Sec. 5, Eq. 28).
EST_CV, EST_BIASED = 0, 1


def estimate(orc_oe: Oracle, orc_fli: Oracle, a: dict, mode: int, param: float):
    """Control-variate (mode EST_CV, param = beta) or biased (EST_BIASED,
    param = gamma) estimate of the outgoing radiance minus emission at every
    vertex of `a`.

    At a vertex x with outgoing direction w_o and sampled incoming direction
    w_i the control variate is h = f~L_i(x, w_i) (looked up in orc_fli, keyed
    on w_i) and its known integral is L~o\\e(x, w_o) (looked up in orc_oe,
    keyed on w_o).  With the vertex's sample g = L_i f and weight
    wp = w / p_perp:

      Sec. 4.2 (Eq. 25):  wp (g - beta h) + beta L~o\\e
      Sec. 5 (Eq. 28):    gamma wp (g - h) + L~o\\e   (beta = 1, corrector scaled)

    Reading: the known integral is added once, outside the wp factor (the
    estimate is then unbiased for any beta; the printed formulas place it
    inside the bracket that is divided by the density).  Where either cell
    is missing or not yet blended the vertex keeps the plain estimate wp g.
    Binary64 throughout; param is taken at binary32, as the library receives
    it.  Returns (estimate (3, n) float64, applied (n,) uint8).
    """
    n = int(np.asarray(a["px"]).shape[0])
    base = {k: a[k] for k in ("px", "py", "pz", "nx", "ny", "nz")}
    base["rough"] = a.get("rough")
    base["footprint"] = a.get("footprint")
    zeros = np.zeros(n, dtype=np.float32)
    qo = dict(base, ox=a.get("oox", zeros), oy=a.get("ooy", zeros), oz=a.get("ooz", zeros))
    qi = dict(base, ox=a.get("oix", zeros), oy=a.get("oiy", zeros), oz=a.get("oiz", zeros))
    L, fo = orc_oe.query(qo)
    h, fi = orc_fli.query(qi)
    g = np.stack([np.asarray(a[k], dtype=np.float64) for k in ("gr", "gg", "gb")])
    w = np.asarray(a["wp"], dtype=np.float64)
    p = float(np.float32(param))
    if mode == EST_CV:
        e = w * (g - p * h) + p * L
    elif mode == EST_BIASED:
        e = p * (w * (g - h)) + L
    else:
        raise ValueError("mode must be EST_CV or EST_BIASED")
    both = (fo != 0) & (fi != 0)
    e = np.where(both[None, :], e, w * g)
    return e, both.astype(np.uint8)


# --------------------------------------------------------------------------
# Progressive solver (Sec. 2.2, Eq. 8-9; Algorithm 1).
def progressive_step(orc: Oracle, x: dict, nxt: dict, tput, le=None):
    """One frame of the progressive solver: the sample at each vertex x_i is
    L_e(x_i) + L~(x_{i+1}) t_i, with L~ the approximant at the path's next
    vertex as the last completed blend left it (0 where it has no blended
    cell) and t_i = f G w / p of the sampled step; the samples are projected
    onto the cells at x (Eq. 8, as insert) and blended (Eq. 10-11).  The
    samples are formed in binary64 and handed to the insert as binary32
    records, as a caller's renderer would.  Returns the samples (3, n)."""
    L, _ = orc.query(nxt)
    t = np.stack([np.asarray(v, dtype=np.float64) for v in tput])
    e = np.zeros_like(t) if le is None else np.stack([np.asarray(v, dtype=np.float64) for v in le])
    lbar = e + L * t
    rec = {k: v for k, v in x.items() if k not in ("r", "g", "b")}
    rec["r"], rec["g"], rec["b"] = (lbar[c].astype(np.float32) for c in range(3))
    orc.insert(rec)
    orc.update()
    return lbar
