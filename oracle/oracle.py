"""ctypes front end of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module.  It wraps oracle/libcinr_oracle.so (plain C, FP64 value plane,
binary32 decision plane) with NumPy-friendly calls.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcinr_oracle.so")

MAX_LEVELS = 32
MAX_LAYERS = 8

CACHED, UNCACHED_DIRECT, UNCACHED_LATTICE = 0, 1, 2


class Inr(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("n_levels", C.c_int32), ("n_features", C.c_int32),
                ("log2_table", C.c_int32), ("level_res", C.c_int32 * MAX_LEVELS), ("n_layers", C.c_int32),
                ("widths", C.c_int32 * (MAX_LAYERS + 1)), ("value_scale", C.c_float),
                ("value_offset", C.c_float), ("table", C.c_void_p), ("weights", C.c_void_p),
                ("grid", C.c_void_p)]


class Camera(C.Structure):
    _fields_ = [("projection", C.c_int32), ("width", C.c_int32), ("height", C.c_int32),
                ("eye", C.c_float * 3), ("forward", C.c_float * 3), ("right", C.c_float * 3),
                ("up", C.c_float * 3), ("tan_half_x", C.c_float), ("tan_half_y", C.c_float),
                ("ortho_w", C.c_float), ("ortho_h", C.c_float)]


class Params(C.Structure):
    _fields_ = [("step", C.c_float), ("lod_scale", C.c_float), ("ert_threshold", C.c_float),
                ("seed", C.c_uint32), ("frame_index", C.c_int32), ("samples_per_iter", C.c_int32),
                ("mode", C.c_int32), ("macro_cell", C.c_int32), ("macro_minmax", C.c_void_p),
                ("adapt_max_exp", C.c_int32),
                ("pipeline", C.c_int32), ("pt_density", C.c_float), ("pt_light_dir", C.c_float * 3),
                ("pt_light", C.c_float * 3), ("pt_ambient", C.c_float * 3), ("pt_max_bounces", C.c_int32),
                ("pt_spp", C.c_int32), ("pt_seed", C.c_uint32), ("lod_context", C.c_float),
                ("ert_replay", C.c_void_p), ("ert_record", C.c_void_p), ("ert_slack", C.c_double)]


class CacheDesc(C.Structure):
    _fields_ = [("brick", C.c_int32), ("n_lods", C.c_int32), ("pool_bricks", C.c_int32),
                ("max_requests", C.c_int32), ("rank_window", C.c_int32), ("ranking", C.c_int32),
                ("preload_period", C.c_int32), ("pool_f16", C.c_int32), ("f16_lods", C.c_uint32),
                ("pool_bricks_f16", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("rays", "samples", "hits", "fallbacks", "misses", "skipped",
                                          "requested", "selected", "evicted", "ert_violations")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        i64, i32, u32 = C.c_int64, C.c_int32, C.c_uint32
        sig = {
            "orc_splitmix64": (C.c_uint64, [C.c_uint64]),
            "orc_xorshift32": (u32, [u32]),
            "orc_frame_seed": (u32, [u32, u32]),
            "orc_philox4x32_10": (None, [P, P, P]),
            "orc_level_size": (i64, [P, C.c_int]),
            "orc_table_entries": (i64, [P]),
            "orc_encode": (None, [P, P, i64, P]),
            "orc_mlp": (None, [P, P, i64, P]),
            "orc_value": (None, [P, P, i64, P]),
            "orc_lod_geometry": (C.c_int, [P, i32, i32, P, P, P]),
            "orc_brick_origin_literal": (None, [P, i32, i32, P]),
            "orc_decode_bricks": (C.c_int, [P, P, i64, i32, i32, P]),
            "orc_macrocells": (None, [P, i32, P]),
            "orc_macrocell_flags": (None, [P, i64, P, P]),
            "orc_step_exp": (i32, [C.c_float, i32]),
            "orc_round_half": (C.c_double, [C.c_double]),
            "orc_pt_uniform": (C.c_float, [C.c_uint32]),
            "orc_pt_free_flight": (C.c_float, [C.c_uint32]),
            "orc_pt_free_flights": (None, [P, i64, P]),
            "orc_pt_direction": (C.c_uint32, [C.c_uint32, C.c_uint32, P, P]),
            "orc_pt_segment_exit": (C.c_float, [P, P, P]),
            "orc_tf_alpha32": (C.c_float, [P, C.c_float]),
            "orc_select_lod_scaled": (i32, [P, P, C.c_float, C.c_float, C.c_uint32, i32, i32]),
            "orc_macrocell_step_codes": (None, [P, i64, P, i32, P]),
            "orc_ray_setup": (C.c_int, [P, P, i32, i32, P, P, P, P]),
            "orc_select_lod": (i32, [P, P, C.c_float, u32, i32, i32]),
            "orc_lod_floor": (i32, [i32, i32, i32]),
            "orc_render_uncached": (C.c_int, [P, P, P, P, P, P]),
            "orc_render_pixels": (C.c_int, [P, P, P, P, P, P, i64, P]),
            "orc_cache_create": (P, [P, P]),
            "orc_cache_create_multi": (P, [P, i32, P]),
            "orc_cache_render_views": (C.c_int, [P, i32, P, P, P, P, P, P]),
            "orc_train_points": (None, [C.c_uint64, i64, i64, P]),
            "orc_grid_trilinear": (None, [P, P, P, i64, P]),
            "orc_cache_destroy": (None, [P]),
            "orc_cache_render": (C.c_int, [P, P, P, P, P, P]),
            "orc_cache_prefill": (C.c_int, [P, P, i64, i32]),
            "orc_cache_n_keys": (i64, [P]),
            "orc_cache_inject_requests": (C.c_int, [P, P, P, i64]),
            "orc_cache_touch": (C.c_int, [P, i32, i32]),
            "orc_cache_end_frame": (C.c_int, [P, i32, P]),
            "orc_cache_page_table": (None, [P, P]),
            "orc_cache_owner": (None, [P, P]),
            "orc_cache_last_used": (None, [P, P]),
            "orc_cache_rank": (None, [P, P]),
            "orc_cache_req_count": (None, [P, P]),
            "orc_cache_request_list": (i64, [P, P]),
            "orc_cache_miss_list": (i64, [P, P, P, i64]),
            "orc_cache_evict_log": (i64, [P, P, i64]),
            "orc_cache_pool": (None, [P, P]),
            "orc_cache_set_miss_logging": (None, [P, C.c_int]),
            "orc_cache_set_ert_trace": (None, [P, C.c_int]),
            "orc_cache_ert_trace": (i64, [P, P, i64]),
            "orc_loss_grad": (C.c_double, [P, P, P, i64, P, P]),
            "orc_loss_grad_prec": (C.c_double, [P, P, P, i64, P, P, C.c_int]),
            "orc_round_bf16": (C.c_double, [C.c_double]),
            "orc_adam_step": (None, [P, P, P, P, i64, i64, C.c_double, C.c_double, C.c_double, C.c_double]),
            "orc_set_threads": (None, [C.c_int]),
            "orc_get_threads": (C.c_int, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


# ----------------------------------------------------------------------------
# INR
# ----------------------------------------------------------------------------


class OracleInr:
    """Holds the float32 parameters (kept alive) and the C descriptor."""

    def __init__(self, arch, table, weights, value_scale=1.0, value_offset=0.0, dims=None):
        self.arch = arch
        self.table = np.ascontiguousarray(table, dtype=np.float32)
        self.weights = np.ascontiguousarray(weights, dtype=np.float32)
        d = Inr()
        dims = arch.dims if dims is None else dims
        for a in range(3):
            d.dims[a] = int(dims[a])
        d.n_levels, d.n_features, d.log2_table = arch.n_levels, arch.n_features, arch.log2_table
        for l, n in enumerate(arch.level_res):
            d.level_res[l] = n
        d.n_layers = len(arch.widths) - 1
        for i, w in enumerate(arch.widths):
            d.widths[i] = w
        d.value_scale = float(value_scale)
        d.value_offset = float(value_offset)
        d.table = self.table.ctypes.data
        d.weights = self.weights.ctypes.data
        self.desc = d
        self.dims = tuple(int(x) for x in dims)
        assert lib().orc_table_entries(C.byref(d)) == self.table.shape[0]

    def ref(self):
        return C.byref(self.desc)

    @classmethod
    def from_grid(cls, grid, value_scale=1.0, value_offset=0.0):
        """A value source backed by an explicit grid (float32 [Vz][Vy][Vx]):
        trilinear at voxel coordinates, then the same normalisation."""
        self = cls.__new__(cls)
        self.arch = None
        self.grid = np.ascontiguousarray(grid, dtype=np.float32)
        d = Inr()
        dims = (self.grid.shape[2], self.grid.shape[1], self.grid.shape[0])
        for a in range(3):
            d.dims[a] = int(dims[a])
        d.value_scale, d.value_offset = float(value_scale), float(value_offset)
        d.grid = self.grid.ctypes.data
        self.desc = d
        self.dims = tuple(int(x) for x in dims)
        return self

    def encode(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
        out = np.empty((u.shape[0], self.arch.n_levels * self.arch.n_features), np.float64)
        lib().orc_encode(self.ref(), _ptr(u), u.shape[0], _ptr(out))
        return out

    def mlp(self, feat):
        feat = np.ascontiguousarray(feat, dtype=np.float64)
        out = np.empty(feat.shape[0], np.float64)
        lib().orc_mlp(self.ref(), _ptr(feat), feat.shape[0], _ptr(out))
        return out

    def value(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        out = np.empty(x.shape[0], np.float64)
        lib().orc_value(self.ref(), _ptr(x), x.shape[0], _ptr(out))
        return out

    def decode_bricks(self, reqs, brick, n_lods):
        reqs = np.ascontiguousarray(reqs, dtype=np.int32).reshape(-1, 4)
        out = np.empty((reqs.shape[0], brick, brick, brick), np.float64)
        rc = lib().orc_decode_bricks(self.ref(), _ptr(reqs), reqs.shape[0], brick, n_lods, _ptr(out))
        if rc != 0:
            raise ValueError("invalid brick request")
        return out

    def macrocells(self, cell):
        M = [(d + cell - 1) // cell for d in self.dims]
        out = np.empty((M[2], M[1], M[0], 2), np.float32)
        lib().orc_macrocells(self.ref(), cell, _ptr(out))
        return out


def value_normalization(arch, table, weights, n_probe=1 << 16):
    """Scale/offset mapping the 2nd and 98th percentiles of the raw network
    output over a fixed Halton probe set to 0 and 1 (the stored value range
    of Section 4.1 for a random-init network)."""
    from paper_2504_18001_amd.synth import halton_points
    m = OracleInr(arch, table, weights)
    y = m.mlp(m.encode(halton_points(n_probe)))
    lo, hi = np.percentile(y, [2.0, 98.0])
    scale = 1.0 / (hi - lo)
    return float(np.float32(scale)), float(np.float32(-lo * scale))


# ----------------------------------------------------------------------------
# Geometry and decision-plane helpers
# ----------------------------------------------------------------------------


def lod_geometry(dims, brick, n_lods):
    K = np.zeros((n_lods, 3), np.int32)
    nb = np.zeros((n_lods, 3), np.int32)
    off = np.zeros(n_lods + 1, np.int64)
    d = np.asarray(dims, np.int32)
    rc = lib().orc_lod_geometry(_ptr(d), brick, n_lods, _ptr(K), _ptr(nb), _ptr(off))
    assert rc == 0
    return K, nb, off


def brick_origin_literal(b, lod, brick):
    bb = np.asarray(b, np.int32)
    out = np.zeros(3, np.int64)
    lib().orc_brick_origin_literal(_ptr(bb), lod, brick, _ptr(out))
    return tuple(int(x) for x in out)


def camera_struct(cam) -> Camera:
    c = Camera()
    c.projection = cam.projection
    c.width, c.height = cam.width, cam.height
    for a in range(3):
        c.eye[a] = float(cam.eye[a])
        c.forward[a] = float(cam.forward[a])
        c.right[a] = float(cam.right[a])
        c.up[a] = float(cam.up[a])
    c.tan_half_x, c.tan_half_y = cam.tan_half_x, cam.tan_half_y
    c.ortho_w, c.ortho_h = cam.ortho_w, cam.ortho_h
    return c


def ray_setup(cam, dims, i, j):
    c = camera_struct(cam)
    d = np.asarray(dims, np.int32)
    o = np.zeros(3, np.float32)
    dd = np.zeros(3, np.float32)
    ts = np.zeros(1, np.float32)
    te = np.zeros(1, np.float32)
    ok = lib().orc_ray_setup(C.byref(c), _ptr(d), i, j, _ptr(o), _ptr(dd), _ptr(ts), _ptr(te))
    return bool(ok), o, dd, float(ts[0]), float(te[0])


def select_lod(p, eye, lod_scale, frame_seed, lod_floor, n_lods):
    pp = np.asarray(p, np.float32)
    ee = np.asarray(eye, np.float32)
    return int(lib().orc_select_lod(_ptr(pp), _ptr(ee), float(lod_scale), int(frame_seed) & 0xFFFFFFFF,
                                    lod_floor, n_lods))


def select_lod_scaled(p, eye, lod_scale, factor, frame_seed, lod_floor, n_lods):
    pp = np.asarray(p, np.float32)
    ee = np.asarray(eye, np.float32)
    return int(lib().orc_select_lod_scaled(_ptr(pp), _ptr(ee), float(lod_scale), float(factor),
                                           int(frame_seed) & 0xFFFFFFFF, lod_floor, n_lods))


def macrocell_flags(minmax, tf):
    mm = np.ascontiguousarray(minmax, np.float32)
    n = mm.size // 2
    out = np.zeros(n, np.uint8)
    t = np.ascontiguousarray(tf, np.float32)
    lib().orc_macrocell_flags(_ptr(mm), n, _ptr(t), _ptr(out))
    return out


PT_MAX_EVENTS = 8000


def pt_uniform(r):
    return float(lib().orc_pt_uniform(int(r) & 0xFFFFFFFF))


def pt_free_flight(r):
    return float(lib().orc_pt_free_flight(int(r) & 0xFFFFFFFF))


def pt_free_flights(words):
    """Free-flight lengths of an array of random words (vectorised)."""
    w = np.ascontiguousarray(words, np.uint32)
    out = np.empty(w.shape, np.float32)
    lib().orc_pt_free_flights(_ptr(w), w.size, _ptr(out))
    return out


def pt_direction(pix, n0, key):
    """Isotropic direction from events n0, n0+1, ... of pixel `pix` (Philox
    key (key[0], key[1])): (direction, first unused event)."""
    k = np.asarray(key, np.uint32)
    d = np.zeros(3, np.float32)
    n = lib().orc_pt_direction(pix, n0, _ptr(k), _ptr(d))
    return d, int(n)


def pt_segment_exit(p, d, vm1):
    p = np.asarray(p, np.float32)
    d = np.asarray(d, np.float32)
    v = np.asarray(vm1, np.float32)
    return float(lib().orc_pt_segment_exit(_ptr(p), _ptr(d), _ptr(v)))


def tf_alpha32(tf, v):
    t = np.ascontiguousarray(tf, np.float32)
    return float(lib().orc_tf_alpha32(_ptr(t), float(v)))


def round_half(x):
    """x rounded to the nearest binary16 value, ties to even (IEEE 754)."""
    return float(lib().orc_round_half(float(x)))


def step_exp(mu, E):
    """Step exponent of a macro-cell of maximum opacity mu > 0 (adaptive sampling)."""
    return int(lib().orc_step_exp(float(mu), int(E)))


def macrocell_step_codes(minmax, tf, E):
    """Per-cell codes of the adaptive sampler: 255 transparent, else the step exponent."""
    mm = np.ascontiguousarray(minmax, np.float32)
    n = mm.size // 2
    out = np.zeros(n, np.uint8)
    t = np.ascontiguousarray(tf, np.float32)
    lib().orc_macrocell_step_codes(_ptr(mm), n, _ptr(t), int(E), _ptr(out))
    return out


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, np.uint32)
    k = np.asarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return [int(x) for x in out]


def make_params(step, lod_scale, seed=0, frame_index=0, ert_threshold=2.0, samples_per_iter=8, mode=CACHED,
                macro_cell=0, macro_minmax=None, adapt_max_exp=-1, path=None, lod_context=0.0, ert_replay=None,
                ert_slack=1e-4):
    """adapt_max_exp: adaptive sampling rate with steps of up to 2^E sample
    spacings (Section 5.2); -1 (or 0) for the fixed step.  path: None for ray
    marching, else a dict of path-tracing parameters (density, light_dir,
    light, ambient, max_bounces, spp, seed).  lod_context: context-aware
    LoD weight in [0, 1] (needs macro-cells)."""
    p = Params()
    p.adapt_max_exp = adapt_max_exp
    p.lod_context = lod_context
    if path is not None:
        p.pipeline = 1
        p.pt_density = path.get("density", 0.05)
        for a in range(3):
            p.pt_light_dir[a] = path.get("light_dir", (0.0, 0.0, 1.0))[a]
            p.pt_light[a] = path.get("light", (1.0, 1.0, 1.0))[a]
            p.pt_ambient[a] = path.get("ambient", (0.0, 0.0, 0.0))[a]
        p.pt_max_bounces = path.get("max_bounces", 1)
        p.pt_spp = path.get("spp", 1)
        p.pt_seed = path.get("seed", 0) & 0xFFFFFFFF
    p.step, p.lod_scale, p.ert_threshold = step, lod_scale, ert_threshold
    p.seed, p.frame_index, p.samples_per_iter, p.mode = seed & 0xFFFFFFFF, frame_index, samples_per_iter, mode
    p.macro_cell = macro_cell if macro_minmax is not None else 0
    p._mm = None if macro_minmax is None else np.ascontiguousarray(macro_minmax, np.float32)
    p.macro_minmax = p._mm.ctypes.data if p._mm is not None else None
    # ert_replay: int32 [H][W] sample-grid index just past each ray's early
    # termination in the renderer being checked, -1 where it did not end early
    p._replay = None if ert_replay is None else np.ascontiguousarray(ert_replay, np.int32)
    p.ert_replay = p._replay.ctypes.data if p._replay is not None else None
    # opacity margin of the replay check: the checked renderer's value
    # tolerance (its reduced-precision MLP may move an opacity by that much)
    p.ert_slack = ert_slack
    p._record = None
    return p


def record_ert(params, width, height):
    """Makes frames rendered with `params` record each ray's early
    termination (see ert_replay); returns the int32 [height][width] array the
    next render fills."""
    params._record = np.full((height, width), -1, np.int32)
    params.ert_record = params._record.ctypes.data
    return params._record


def render_uncached(inr: OracleInr, cam, tf, params: Params):
    c = camera_struct(cam)
    t = np.ascontiguousarray(tf, np.float32)
    out = np.zeros((cam.height, cam.width, 4), np.float64)
    st = Stats()
    rc = lib().orc_render_uncached(inr.ref(), C.byref(c), _ptr(t), C.byref(params), _ptr(out), C.byref(st))
    assert rc == 0
    return out, st.as_dict()


def render_pixels(inr: OracleInr, cam, tf, params: Params, pixels, cache=None):
    """Colours of the listed pixels (j*W + i), against `cache`'s residency
    (None for the uncached modes), leaving all state untouched."""
    c = camera_struct(cam)
    t = np.ascontiguousarray(tf, np.float32)
    px = np.ascontiguousarray(pixels, np.int32)
    out = np.zeros((px.size, 4), np.float64)
    rc = lib().orc_render_pixels(inr.ref(), cache.h if cache is not None else None, C.byref(c), _ptr(t),
                                 C.byref(params), _ptr(px), px.size, _ptr(out))
    assert rc == 0
    return out


class OracleCache:
    """Oracle brick cache of one volume, or shared by a list of volumes of
    equal dimensions (volume i owns keys [i K, (i+1) K))."""

    def __init__(self, inr, brick, n_lods, pool_bricks, max_requests, rank_window=1000, ranking=1,
                 preload_period=0, log_misses=False, trace_ert=False, pool_f16=False, f16_lods=0,
                 pool_bricks_f16=0):
        inrs = list(inr) if isinstance(inr, (list, tuple)) else [inr]
        self.inrs = inrs
        self.inr = inrs[0]
        d = CacheDesc()
        d.brick, d.n_lods, d.pool_bricks, d.max_requests = brick, n_lods, pool_bricks, max_requests
        d.rank_window, d.ranking, d.preload_period = rank_window, ranking, preload_period
        d.pool_f16 = 1 if pool_f16 else 0
        d.f16_lods, d.pool_bricks_f16 = f16_lods, pool_bricks_f16
        self.desc = d
        self._descs = (Inr * len(inrs))(*[m.desc for m in inrs])
        self.h = lib().orc_cache_create_multi(C.cast(self._descs, C.c_void_p), len(inrs), C.byref(d))
        if not self.h:
            raise ValueError("invalid cache description, or not enough host memory for it")
        self.n_keys = int(lib().orc_cache_n_keys(self.h))
        lib().orc_cache_set_miss_logging(self.h, 1 if log_misses else 0)
        lib().orc_cache_set_ert_trace(self.h, 1 if trace_ert else 0)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_cache_destroy(self.h)
            self.h = None

    def render(self, cam, tf, params: Params):
        c = camera_struct(cam)
        t = np.ascontiguousarray(tf, np.float32)
        out = np.zeros((cam.height, cam.width, 4), np.float64)
        st = Stats()
        rc = lib().orc_cache_render(self.h, C.byref(c), _ptr(t), C.byref(params), _ptr(out), C.byref(st))
        assert rc == 0
        return out, st.as_dict()

    def render_views(self, views, params):
        """One frame of several views: views = [(volume index, camera, tf)],
        params = [Params] (one per view).  Returns [(image, stats)]."""
        n = len(views)
        vol = np.array([v[0] for v in views], np.int32)
        cams = (Camera * n)(*[camera_struct(v[1]) for v in views])
        tfs = np.ascontiguousarray(np.stack([np.asarray(v[2], np.float32) for v in views]), np.float32)
        ps = (Params * n)(*params)
        sizes = [v[1].width * v[1].height for v in views]
        out = np.zeros(4 * sum(sizes), np.float64)
        sts = (Stats * n)()
        rc = lib().orc_cache_render_views(self.h, n, _ptr(vol), C.cast(cams, C.c_void_p), _ptr(tfs),
                                          C.cast(ps, C.c_void_p), _ptr(out), C.cast(sts, C.c_void_p))
        assert rc == 0
        res, o = [], 0
        for (vi, cam, tf), sz, st in zip(views, sizes, sts):
            res.append((out[4 * o:4 * (o + sz)].reshape(cam.height, cam.width, 4), st.as_dict()))
            o += sz
        return res

    def prefill(self, keys, stamp=0):
        k = np.ascontiguousarray(keys, np.int32)
        rc = lib().orc_cache_prefill(self.h, _ptr(k), k.size, stamp)
        if rc != 0:
            raise ValueError("invalid prefill")

    def inject_requests(self, keys, counts):
        k = np.ascontiguousarray(keys, np.int32)
        c = np.ascontiguousarray(counts, np.uint32)
        if lib().orc_cache_inject_requests(self.h, _ptr(k), _ptr(c), k.size) != 0:
            raise ValueError("invalid request injection")

    def touch(self, slot, frame):
        if lib().orc_cache_touch(self.h, slot, frame) != 0:
            raise ValueError("invalid slot")

    def end_frame(self, frame):
        st = Stats()
        lib().orc_cache_end_frame(self.h, frame, C.byref(st))
        return st.as_dict()

    def page_table(self):
        out = np.empty(self.n_keys, np.int32)
        lib().orc_cache_page_table(self.h, _ptr(out))
        return out

    def owner(self):
        out = np.empty(self.desc.pool_bricks, np.int32)
        lib().orc_cache_owner(self.h, _ptr(out))
        return out

    def last_used(self):
        out = np.empty(self.desc.pool_bricks, np.int32)
        lib().orc_cache_last_used(self.h, _ptr(out))
        return out

    def rank(self):
        out = np.empty(self.n_keys, np.int64)
        lib().orc_cache_rank(self.h, _ptr(out))
        return out

    def req_count(self):
        out = np.empty(self.n_keys, np.uint32)
        lib().orc_cache_req_count(self.h, _ptr(out))
        return out

    def request_list(self):
        n = lib().orc_cache_request_list(self.h, None)
        out = np.empty(max(n, 1), np.int32)
        lib().orc_cache_request_list(self.h, _ptr(out))
        return out[:n]

    def miss_list(self):
        n = lib().orc_cache_miss_list(self.h, None, None, 0)
        pk = np.empty((max(n, 1), 2), np.int32)
        pos = np.empty((max(n, 1), 3), np.float32)
        lib().orc_cache_miss_list(self.h, _ptr(pk), _ptr(pos), n)
        return pk[:n], pos[:n]

    def evict_log(self):
        n = lib().orc_cache_evict_log(self.h, None, 0)
        out = np.empty((max(n, 1), 4), np.int32)
        lib().orc_cache_evict_log(self.h, _ptr(out), n)
        return out[:n]

    def pool(self):
        B = self.desc.brick
        out = np.empty((self.desc.pool_bricks, B, B, B), np.float64)
        lib().orc_cache_pool(self.h, _ptr(out))
        return out

    def ert_trace(self):
        n = lib().orc_cache_ert_trace(self.h, None, 0)
        out = np.empty(max(n, 1), np.int32)
        lib().orc_cache_ert_trace(self.h, _ptr(out), n)
        return out[:n]


def loss_grad(inr: OracleInr, u, target, bf16_operands=False):
    """Mean squared error and its gradients (table, weights); with
    bf16_operands the hidden layers' product operands are rounded to bfloat16."""
    u = np.ascontiguousarray(u, np.float64).reshape(-1, 3)
    t = np.ascontiguousarray(target, np.float64)
    gt = np.zeros(inr.table.shape, np.float64)
    gw = np.zeros(inr.weights.shape, np.float64)
    loss = lib().orc_loss_grad_prec(inr.ref(), _ptr(u), _ptr(t), u.shape[0], _ptr(gt), _ptr(gw),
                                    1 if bf16_operands else 0)
    return loss, gt, gw


def round_bf16(x):
    return lib().orc_round_bf16(float(x))


def train_points(seed, step, n):
    """Training batch `step` (n points in [0,1)^3), float64 [n][3]."""
    u = np.zeros((n, 3), np.float64)
    lib().orc_train_points(C.c_uint64(seed), C.c_int64(step), C.c_int64(n), _ptr(u))
    return u


def grid_trilinear(grid, u):
    """Trilinear ground truth of points u in the explicit grid (float32 [Vz][Vy][Vx])."""
    g = np.ascontiguousarray(grid, np.float32)
    dims = np.array([g.shape[2], g.shape[1], g.shape[0]], np.int32)
    uu = np.ascontiguousarray(u, np.float64).reshape(-1, 3)
    out = np.zeros(uu.shape[0], np.float64)
    lib().orc_grid_trilinear(_ptr(g), _ptr(dims), _ptr(uu), C.c_int64(uu.shape[0]), _ptr(out))
    return out


def set_threads(n):
    lib().orc_set_threads(int(n))


def get_threads():
    return int(lib().orc_get_threads())
