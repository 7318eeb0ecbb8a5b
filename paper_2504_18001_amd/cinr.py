"""Thin Python binding of libcinr (include/cinr.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch provides device memory and the current stream.  The
library is loaded from this package directory; importing this module on a
machine where it is missing raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcinr.so")

MAX_LEVELS, MAX_LAYERS, MAX_LODS = 32, 8, 16
F32, BF16, F16, BF16X3 = 0, 1, 2, 3
CACHED, UNCACHED_DIRECT, UNCACHED_LATTICE = 0, 1, 2
RANK_TIMESTAMP, RANK_PRIORITY = 0, 1
PERSPECTIVE, ORTHOGRAPHIC = 0, 1
DUMP_PAGE_TABLE, DUMP_SLOT_OWNER, DUMP_LAST_USED, DUMP_RANK, DUMP_REQ_COUNT = 0, 1, 2, 3, 4
DUMP_REQUEST_LIST, DUMP_MISS_LIST, DUMP_EVICTION_LOG, DUMP_POOL = 5, 6, 7, 8
DUMP_PT_DIRECTORY, DUMP_PT_BLOCKS, DUMP_PT_STATE = 9, 10, 11
# bytes of the fixed device array of cinr_render_frame_noalloc (the last 256
# hold its control words)
NOALLOC_SCRATCH_BYTES = 64 << 20

DTYPES = {"f32": F32, "fp32": F32, "bf16": BF16, "f16": F16, "fp16": F16, "bf16x3": BF16X3}


class CinrError(RuntimeError):
    pass


class VolumeDesc(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("n_levels", C.c_int32), ("n_features", C.c_int32),
                ("log2_table", C.c_int32), ("level_res", C.c_int32 * MAX_LEVELS), ("n_layers", C.c_int32),
                ("widths", C.c_int32 * (MAX_LAYERS + 1)), ("value_scale", C.c_float), ("value_offset", C.c_float),
                ("d_table", C.c_void_p), ("d_weights", C.c_void_p), ("d_macrocells", C.c_void_p),
                ("macrocell_size", C.c_int32)]


class CacheDesc(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("brick", "n_lods", "pool_bricks", "max_requests", "rank_window", "ranking",
                                          "preload_period", "miss_log_capacity", "evict_log_capacity",
                                          "keep_request_counts", "pool_dtype")] + [
        ("f16_lods", C.c_uint32), ("pool_bricks_f16", C.c_int32), ("virtual_page_table", C.c_int32),
        ("pt_blocks", C.c_int32)]


# Largest rounding error of binary16 for the pool's values in [0, 1]: half
# the spacing 2^-11 of [0.5, 1).
F16_POOL_ERROR = 2.0 ** -12


def f16_lods_for_bounds(bounds):
    """The f16_lods mask of a mixed pool from per-LoD error bounds: LoD L
    is stored in binary16 when bounds[L] admits binary16 rounding."""
    return sum(1 << L for L, b in enumerate(bounds) if b >= F16_POOL_ERROR)


class CameraDesc(C.Structure):
    _fields_ = [("projection", C.c_int32), ("width", C.c_int32), ("height", C.c_int32), ("eye", C.c_float * 3),
                ("forward", C.c_float * 3), ("right", C.c_float * 3), ("up", C.c_float * 3),
                ("tan_half_x", C.c_float), ("tan_half_y", C.c_float), ("ortho_w", C.c_float), ("ortho_h", C.c_float)]


class RenderParams(C.Structure):
    _fields_ = [("step", C.c_float), ("lod_scale", C.c_float), ("ert_threshold", C.c_float), ("seed", C.c_uint32),
                ("frame_index", C.c_int32), ("samples_per_iter", C.c_int32), ("mode", C.c_int32),
                ("mlp_dtype", C.c_int32), ("pipe_depth", C.c_int32), ("xcd_bands", C.c_int32),
                ("adapt_max_exp", C.c_int32), ("waves_per_simd", C.c_int32),
                ("pipeline", C.c_int32), ("pt_density", C.c_float), ("pt_light_dir", C.c_float * 3),
                ("pt_light", C.c_float * 3), ("pt_ambient", C.c_float * 3), ("pt_max_bounces", C.c_int32),
                ("pt_spp", C.c_int32), ("pt_seed", C.c_uint32), ("lod_context", C.c_float),
                ("ert_record", C.c_void_p)]


RAY_MARCH, PATH_TRACE = 0, 1


def _set_path(p, path):
    """Path-tracing fields of RenderParams p from a dict (density, light_dir,
    light, ambient, max_bounces, spp, seed), or ray marching for None."""
    if path is None:
        p.pipeline = RAY_MARCH
        return
    p.pipeline = PATH_TRACE
    p.pt_density = float(path.get("density", 0.05))
    for a in range(3):
        p.pt_light_dir[a] = float(path.get("light_dir", (0.0, 0.0, 1.0))[a])
        p.pt_light[a] = float(path.get("light", (1.0, 1.0, 1.0))[a])
        p.pt_ambient[a] = float(path.get("ambient", (0.0, 0.0, 0.0))[a])
    p.pt_max_bounces = int(path.get("max_bounces", 1))
    p.pt_spp = int(path.get("spp", 1))
    p.pt_seed = int(path.get("seed", 0)) & 0xFFFFFFFF


def _ert_record(rec, cam):
    """Device pointer of an early-termination record tensor (int32 [H][W] on
    the GPU), or None."""
    if rec is None:
        return None
    if rec.dtype != torch.int32 or not rec.is_cuda or not rec.is_contiguous() or \
            tuple(rec.shape) != (cam.height, cam.width):
        raise ValueError("ert_record must be a contiguous int32 CUDA tensor of shape (height, width)")
    return rec.data_ptr()


def _workspace_size(vol, width, height, samples_per_iter, path):
    need = C.c_size_t()
    fn = lib().cinr_path_workspace_size if path is not None else lib().cinr_render_workspace_size
    _check(fn(vol.h, width, height, samples_per_iter, C.byref(need)))
    return need.value


def pt_free_flight(words):
    """The path tracer's free-flight lengths for a device tensor of 32-bit
    random words (int32 bit patterns), on the GPU."""
    w = words.to(torch.int32).contiguous()
    out = torch.empty(w.shape, dtype=torch.float32, device=w.device)
    _check(lib().cinr_pt_free_flight(_ptr(w), w.numel(), _ptr(out), _stream()))
    return out


class GridDesc(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("d_grid", C.c_void_p), ("value_scale", C.c_float),
                ("value_offset", C.c_float), ("d_macrocells", C.c_void_p), ("macrocell_size", C.c_int32)]


class TrainDesc(C.Structure):
    _fields_ = [("batch", C.c_int64), ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("seed", C.c_uint64), ("mlp_dtype", C.c_int32)]


STAGES = ("setup", "march", "infer", "shade", "cm", "decode")
STAT_FIELDS = ("rays", "samples", "hits", "fallbacks", "misses", "skipped", "requested", "selected", "evicted",
               "iterations")

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CinrError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        sig = {
            "cinr_create_volume_inr": [P, P],
            "cinr_create_volume_grid": [P, P],
            "cinr_destroy_volume": [P],
            "cinr_lod_geometry": [P, i32, i32, P, P],
            "cinr_infer_points": [P, P, i64, P, i32, P],
            "cinr_decode_bricks": [P, P, i32, i32, P, i32, P],
            "cinr_decode_bricks_shaped": [P, P, i32, i32, P, i32, i32, i32, P],
            "cinr_set_decode_shape": [P, i32, i32],
            "cinr_tune_decode": [P, P, i32, i32, P, i32, i32, P, P, P],
            "cinr_build_macrocells": [P, i32, P, i32, P],
            "cinr_cache_workspace_size": [P, P, P],
            "cinr_create_cache": [P, P, P, sz, P, sz, P, P],
            "cinr_destroy_cache": [P],
            "cinr_cache_prefill": [P, P, i32, i32, i32, P],
            "cinr_render_workspace_size": [P, i32, i32, i32, P],
            "cinr_render_frame": [P, P, P, P, P, P, P, P, sz, P],
            "cinr_render_frame_noalloc": [P, P, P, P, P, P, P, P],
            "cinr_cache_dump": [P, i32, P, sz, P, P],
            "cinr_last_error": [],
            "cinr_set_timing": [P, i32],
            "cinr_collect_timing": [P, P, P],
            "cinr_train_workspace_size": [P, P, P],
            "cinr_train_create": [P, P, P, sz, P, P],
            "cinr_train_destroy": [P],
            "cinr_train_points": [P, P, P, i64, P, P, P],
            "cinr_train_gradients": [P, P, P, i64, P, P, P, P],
            "cinr_train_step": [P, P, P, i64, P, P],
            "cinr_adam_update": [P, P, P, P, i64, i64, C.c_float, C.c_float, C.c_float, C.c_float, i32, P],
            "cinr_train_set_lr": [P, C.c_float],
            "cinr_cache_workspace_size_multi": [P, i32, P, P],
            "cinr_create_cache_multi": [P, i32, P, P, sz, P, sz, P, P],
            "cinr_render_views": [P, i32, P, P],
            "cinr_tuned_launch": [P, i32, i32, P, P, P, P],
            "cinr_frame_graph_create": [P, i32, P, P],
            "cinr_path_workspace_size": [P, i32, i32, i32, P],
            "cinr_pt_free_flight": [P, i64, P, P],
            "cinr_frame_graph_render": [P, P, i32, P],
            "cinr_frame_graph_counts": [P, P, P, P],
            "cinr_frame_graph_set_device_iterations": [P, i32],
            "cinr_frame_graph_destroy": [P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.cinr_destroy_volume.restype = None
        L.cinr_destroy_cache.restype = None
        L.cinr_train_destroy.restype = None
        L.cinr_frame_graph_destroy.restype = None
        L.cinr_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise CinrError(f"libcinr error {rc}: {lib().cinr_last_error().decode()}")


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dtype(d):
    return DTYPES[d] if isinstance(d, str) else int(d)


class _VolumeOps:
    """Operations shared by INR and grid volumes (handle `h`, `dims`, `device`)."""

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.cinr_destroy_volume(self.h)
            self.h = None

    def geometry(self, brick, n_lods):
        nb = np.zeros((n_lods, 3), np.int32)
        off = np.zeros(n_lods + 1, np.int64)
        _check(lib().cinr_lod_geometry(self.h, brick, n_lods, nb.ctypes.data_as(C.c_void_p),
                                       off.ctypes.data_as(C.c_void_p)))
        return nb, off

    def infer_points(self, pos, dtype="f32", out=None):
        pos = pos.contiguous()
        n = pos.shape[0]
        out = torch.empty(n, dtype=torch.float32, device=pos.device) if out is None else out
        _check(lib().cinr_infer_points(self.h, _ptr(pos), n, _ptr(out), _dtype(dtype), _stream()))
        return out

    def decode_bricks(self, reqs, brick, dtype="f32", out=None):
        reqs = reqs.to(torch.int32).contiguous()
        n = reqs.shape[0]
        out = torch.empty((n, brick, brick, brick), dtype=torch.float32, device=reqs.device) if out is None else out
        _check(lib().cinr_decode_bricks(self.h, _ptr(reqs), n, brick, _ptr(out), _dtype(dtype), _stream()))
        return out

    def decode_bricks_shaped(self, reqs, brick, dtype="f32", parts=0, stage_kib=64, out=None):
        """decode_bricks with an explicit launch shape (parts per brick, LDS
        budget of the staged corner boxes)."""
        reqs = reqs.to(torch.int32).contiguous()
        n = reqs.shape[0]
        out = torch.empty((n, brick, brick, brick), dtype=torch.float32, device=reqs.device) if out is None else out
        _check(lib().cinr_decode_bricks_shaped(self.h, _ptr(reqs), n, brick, _ptr(out), _dtype(dtype), int(parts),
                                               int(stage_kib), _stream()))
        return out

    DECODE_SHAPES = ((0, 0),) + tuple((p, k) for p in (1, 2, 4, 8, 16) for k in (0, 32, 64))

    def tune_decode(self, reqs, brick, dtype="f32", reps=3):
        """Times every decoding launch shape on the requests `reqs` and keeps
        the fastest for this volume; returns (chosen shape, {shape: ms})."""
        reqs = reqs.to(torch.int32).contiguous()
        n = reqs.shape[0]
        out = torch.empty((n, brick, brick, brick), dtype=torch.float32, device=reqs.device)
        ms = np.zeros(len(self.DECODE_SHAPES), np.float32)
        chosen = C.c_int32()
        _check(lib().cinr_tune_decode(self.h, _ptr(reqs), n, brick, _ptr(out), _dtype(dtype), int(reps),
                                      ms.ctypes.data_as(C.c_void_p), C.byref(chosen), _stream()))
        return self.DECODE_SHAPES[chosen.value], {s: float(t) for s, t in zip(self.DECODE_SHAPES, ms) if t >= 0}

    def set_decode_shape(self, parts, stage_kib=64):
        """Launch shape of this volume's brick decoding (decode_bricks and caches)."""
        _check(lib().cinr_set_decode_shape(self.h, int(parts), int(stage_kib)))

    def set_timing(self, on, march_only=False):
        """Stage timing off, on (every stage) or, with march_only, on the march launches only."""
        _check(lib().cinr_set_timing(self.h, (2 if march_only else 1) if on else 0))

    def collect_timing(self):
        """{stage: (milliseconds, launches)} since the last collection."""
        ms = np.zeros(len(STAGES), np.float64)
        n = np.zeros(len(STAGES), np.int64)
        _check(lib().cinr_collect_timing(self.h, ms.ctypes.data_as(C.c_void_p), n.ctypes.data_as(C.c_void_p)))
        return {s: (float(ms[i]), int(n[i])) for i, s in enumerate(STAGES)}

    def build_macrocells(self, cell, dtype="f32"):
        M = [(d + cell - 1) // cell for d in self.dims]
        out = torch.empty((M[2], M[1], M[0], 2), dtype=torch.float32, device=self.device)
        _check(lib().cinr_build_macrocells(self.h, cell, _ptr(out), _dtype(dtype), _stream()))
        return out


class GridVolume(_VolumeOps):
    """A volume defined by an explicit voxel grid (f32 [Vz][Vy][Vx] on the GPU)."""

    def __init__(self, grid, value_scale=1.0, value_offset=0.0, macrocells=None, macro_cell=0):
        self.grid = grid.to(torch.float32).contiguous()
        self.device = self.grid.device
        self.dims = (int(grid.shape[2]), int(grid.shape[1]), int(grid.shape[0]))
        self.macrocells = None
        if macrocells is not None:
            self.macrocells = macrocells.to(device=self.device, dtype=torch.float32).contiguous()
        d = GridDesc()
        for a in range(3):
            d.dims[a] = self.dims[a]
        d.d_grid = self.grid.data_ptr()
        d.value_scale, d.value_offset = float(value_scale), float(value_offset)
        d.d_macrocells = self.macrocells.data_ptr() if self.macrocells is not None else None
        d.macrocell_size = int(macro_cell) if self.macrocells is not None else 0
        self.desc = d
        h = C.c_void_p()
        _check(lib().cinr_create_volume_grid(C.byref(d), C.byref(h)))
        self.h = h


class Volume(_VolumeOps):
    """A volume defined by a hash-grid INR whose parameters live on the GPU."""

    def __init__(self, arch, table, weights, value_scale=1.0, value_offset=0.0, macrocells=None, macro_cell=0,
                 dims=None, device="cuda"):
        self.arch = arch
        self.dims = tuple(int(x) for x in (arch.dims if dims is None else dims))
        self.table = torch.as_tensor(np.asarray(table, np.float32)).to(device).contiguous() \
            if not torch.is_tensor(table) else table.to(device=device, dtype=torch.float32).contiguous()
        self.weights = torch.as_tensor(np.asarray(weights, np.float32)).to(device).contiguous() \
            if not torch.is_tensor(weights) else weights.to(device=device, dtype=torch.float32).contiguous()
        self.macrocells = None
        if macrocells is not None:
            mc = macrocells if torch.is_tensor(macrocells) else torch.as_tensor(np.asarray(macrocells, np.float32))
            self.macrocells = mc.to(device=device, dtype=torch.float32).contiguous()
        d = VolumeDesc()
        for a in range(3):
            d.dims[a] = self.dims[a]
        d.n_levels, d.n_features, d.log2_table = arch.n_levels, arch.n_features, arch.log2_table
        for l, n in enumerate(arch.level_res):
            d.level_res[l] = n
        d.n_layers = len(arch.widths) - 1
        for i, w in enumerate(arch.widths):
            d.widths[i] = w
        d.value_scale, d.value_offset = float(value_scale), float(value_offset)
        d.d_table = self.table.data_ptr()
        d.d_weights = self.weights.data_ptr()
        d.d_macrocells = self.macrocells.data_ptr() if self.macrocells is not None else None
        d.macrocell_size = int(macro_cell) if self.macrocells is not None else 0
        self.desc = d
        h = C.c_void_p()
        _check(lib().cinr_create_volume_inr(C.byref(d), C.byref(h)))
        self.h = h

    @property
    def device(self):
        return self.table.device


class Cache:
    """Multi-resolution brick cache over a torch-allocated pool and workspace,
    for one volume or shared by a list of volumes of the same shape (volume i
    owns keys [i K, (i+1) K), K = keys of one volume)."""

    def __init__(self, volume, brick, n_lods, pool_bricks, max_requests, rank_window=1000,
                 ranking=RANK_PRIORITY, preload_period=0, miss_log_capacity=0, evict_log_capacity=4096,
                 keep_request_counts=False, pool_dtype="f32", f16_lods=0, pool_bricks_f16=0,
                 virtual_page_table=False, pt_blocks=0):
        vols = list(volume) if isinstance(volume, (list, tuple)) else [volume]
        self.volumes = vols
        volume = vols[0]
        self.volume = volume
        d = CacheDesc()
        d.brick, d.n_lods, d.pool_bricks, d.max_requests = brick, n_lods, pool_bricks, max_requests
        d.rank_window, d.ranking, d.preload_period = rank_window, ranking, preload_period
        d.miss_log_capacity, d.evict_log_capacity = miss_log_capacity, evict_log_capacity
        d.keep_request_counts = 1 if keep_request_counts else 0
        if pool_dtype not in ("f32", "f16"):
            raise ValueError(f"pool_dtype {pool_dtype!r}: 'f32' or 'f16'")
        d.pool_dtype = _dtype(pool_dtype)
        d.f16_lods, d.pool_bricks_f16 = int(f16_lods), int(pool_bricks_f16)
        d.virtual_page_table, d.pt_blocks = int(bool(virtual_page_table)), int(pt_blocks)
        self.pool_dtype = pool_dtype if not f16_lods else "mixed"
        # binary32 slots [0, split), then binary16 slots [split, pool_bricks)
        self.split = pool_bricks - pool_bricks_f16 if f16_lods else pool_bricks
        self.desc = d
        ws = C.c_size_t()
        hs = (C.c_void_p * len(vols))(*[v.h.value for v in vols])
        _check(lib().cinr_cache_workspace_size_multi(hs, len(vols), C.byref(d), C.byref(ws)))
        dev = volume.device
        if f16_lods:
            nbytes = (self.split * 4 + (pool_bricks - self.split) * 2) * brick ** 3
            self.pool = torch.empty((nbytes + 3) // 4, dtype=torch.float32, device=dev)
        else:
            tdt = torch.float16 if pool_dtype == "f16" else torch.float32
            self.pool = torch.empty(max(pool_bricks, 1) * brick ** 3, dtype=tdt, device=dev)
        self.workspace = torch.empty(ws.value, dtype=torch.uint8, device=dev)
        h = C.c_void_p()
        _check(lib().cinr_create_cache_multi(hs, len(vols), C.byref(d), _ptr(self.pool),
                                             self.pool.numel() * self.pool.element_size(),
                                             _ptr(self.workspace), ws.value, _stream(), C.byref(h)))
        self.h = h
        nb, off = volume.geometry(brick, n_lods)
        self.nb, self.key_offset = nb, off
        self.keys_per_volume = int(off[-1])
        self.n_keys = self.keys_per_volume * len(vols)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.cinr_destroy_cache(self.h)
            self.h = None

    def prefill(self, keys, stamp=0, dtype="f32"):
        k = keys.to(torch.int32).contiguous()
        _check(lib().cinr_cache_prefill(self.h, _ptr(k), k.numel(), stamp, _dtype(dtype), _stream()))

    def dump(self, kind):
        need = C.c_size_t()
        rc = lib().cinr_cache_dump(self.h, kind, None, 0, C.byref(need), _stream())
        if rc not in (0, -2):
            _check(rc)
        buf = np.empty(max(need.value, 1), np.uint8)
        _check(lib().cinr_cache_dump(self.h, kind, buf.ctypes.data_as(C.c_void_p), buf.size, C.byref(need),
                                     _stream()))
        buf = buf[:need.value]
        if kind in (DUMP_PAGE_TABLE, DUMP_SLOT_OWNER, DUMP_LAST_USED, DUMP_REQUEST_LIST, DUMP_PT_DIRECTORY):
            return buf.view(np.int32)
        if kind == DUMP_PT_BLOCKS:
            return buf.view(np.int32).reshape(-1, 512)
        if kind == DUMP_PT_STATE:
            b = buf.view(np.int32)
            return {"blocks": int(b[0]), "free_blocks": int(b[1]), "unmapped_for_want_of_a_block": int(b[2]),
                    "directory_per_volume": int(b[3])}
        if kind == DUMP_RANK:
            return buf.view(np.int64)
        if kind == DUMP_REQ_COUNT:
            return buf.view(np.uint32)
        if kind == DUMP_MISS_LIST:
            rec = buf.view(np.int32).reshape(-1, 5)
            return rec[:, :2].copy(), rec[:, 2:].copy().view(np.float32)
        if kind == DUMP_EVICTION_LOG:
            return buf.view(np.int32).reshape(-1, 4)
        if kind == DUMP_POOL:
            B = self.desc.brick
            if self.pool_dtype == "mixed":
                # both classes as float32 (binary16 values widen exactly)
                n32 = self.split * B ** 3 * 4
                with np.errstate(invalid="ignore"):  # free slots hold arbitrary bits
                    hi = buf[n32:].view(np.float16).astype(np.float32)
                return np.concatenate([buf[:n32].view(np.float32), hi]).reshape(-1, B, B, B)
            return buf.view(np.float16 if self.pool_dtype == "f16" else np.float32).reshape(-1, B, B, B)
        return buf


def camera_desc(cam) -> CameraDesc:
    c = CameraDesc()
    c.projection, c.width, c.height = int(cam.projection), int(cam.width), int(cam.height)
    for a in range(3):
        c.eye[a] = float(cam.eye[a])
        c.forward[a] = float(cam.forward[a])
        c.right[a] = float(cam.right[a])
        c.up[a] = float(cam.up[a])
    c.tan_half_x, c.tan_half_y = float(cam.tan_half_x), float(cam.tan_half_y)
    c.ortho_w, c.ortho_h = float(cam.ortho_w), float(cam.ortho_h)
    return c


class Renderer:
    """Owns the per-call render workspace (grown on demand)."""

    def __init__(self, device="cuda"):
        self.device = device
        self.ws = None
        self.stats = torch.zeros(len(STAT_FIELDS), dtype=torch.int64, device=device)

    def render(self, volume: Volume, cam, tf, step, lod_scale=0.0, frame_index=0, seed=0, ert_threshold=2.0,
               samples_per_iter=32, mode=CACHED, dtype="f32", cache: Cache = None, out=None, stats=None,
               pipe_depth=0, xcd_bands=0, adapt_max_exp=0, path=None, lod_context=0.0, waves_per_simd=0,
               ert_record=None):
        """path: None for ray marching, else the path tracer's parameters
        (dict: density, light_dir, light, ambient, max_bounces, spp, seed).
        lod_context: context-aware LoD weight in [0, 1].
        ert_record: optional int32 [H][W] CUDA tensor that receives, per pixel,
        the sample-grid index just past the sample that ended the ray early
        (-1: not ended early)."""
        need = _workspace_size(volume, cam.width, cam.height, samples_per_iter, path)
        if self.ws is None or self.ws.numel() < need:
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        out, tf, p, cd, st = self._call_args(cam, tf, step, lod_scale, frame_index, seed, ert_threshold,
                                             samples_per_iter, mode, dtype, out, stats, pipe_depth, xcd_bands,
                                             adapt_max_exp, path, lod_context, waves_per_simd, ert_record)
        _check(lib().cinr_render_frame(cache.h if cache is not None else None, volume.h, C.byref(cd), _ptr(tf),
                                       C.byref(p), _ptr(out), _ptr(st), _ptr(self.ws), self.ws.numel(),
                                       _stream()))
        self._last_stats = st
        return out

    def render_noalloc(self, volume: Volume, cam, tf, step, lod_scale=0.0, frame_index=0, seed=0,
                       ert_threshold=2.0, samples_per_iter=32, mode=CACHED, dtype="f32", cache: Cache = None,
                       out=None, stats=None, pipe_depth=0, xcd_bands=0, adapt_max_exp=0, path=None,
                       lod_context=0.0, waves_per_simd=0, ert_record=None):
        """render() through cinr_render_frame_noalloc: no render workspace, the
        library's fixed device array instead (NOALLOC_SCRATCH_BYTES); the call
        returns once the frame has finished.  `out` and the TF must already be
        CUDA tensors for the call itself to allocate nothing."""
        out, tf, p, cd, st = self._call_args(cam, tf, step, lod_scale, frame_index, seed, ert_threshold,
                                             samples_per_iter, mode, dtype, out, stats, pipe_depth, xcd_bands,
                                             adapt_max_exp, path, lod_context, waves_per_simd, ert_record)
        _check(lib().cinr_render_frame_noalloc(cache.h if cache is not None else None, volume.h, C.byref(cd),
                                               _ptr(tf), C.byref(p), _ptr(out), _ptr(st), _stream()))
        self._last_stats = st
        return out

    def _call_args(self, cam, tf, step, lod_scale, frame_index, seed, ert_threshold, samples_per_iter, mode, dtype,
                   out, stats, pipe_depth, xcd_bands, adapt_max_exp, path, lod_context, waves_per_simd, ert_record):
        out = torch.empty((cam.height, cam.width, 4), dtype=torch.float32, device=self.device) if out is None else out
        tf = tf if torch.is_tensor(tf) else torch.as_tensor(np.asarray(tf, np.float32))
        tf = tf.to(device=self.device, dtype=torch.float32).contiguous()
        self._tf = tf
        p = RenderParams()
        p.step, p.lod_scale, p.ert_threshold = float(step), float(lod_scale), float(ert_threshold)
        p.seed, p.frame_index, p.samples_per_iter = int(seed) & 0xFFFFFFFF, int(frame_index), int(samples_per_iter)
        p.mode, p.mlp_dtype = int(mode), _dtype(dtype)
        p.pipe_depth, p.xcd_bands = int(pipe_depth), int(xcd_bands)
        p.adapt_max_exp = int(adapt_max_exp)
        p.lod_context = float(lod_context)
        p.waves_per_simd = int(waves_per_simd)
        _set_path(p, path)
        p.ert_record = _ert_record(ert_record, cam)
        cd = camera_desc(cam)
        st = self.stats if stats is None else stats
        return out, tf, p, cd, st

    def last_stats(self):
        v = self._last_stats.cpu().numpy()
        return {k: int(v[i]) for i, k in enumerate(STAT_FIELDS)}


class Trainer:
    """GPU training of a Volume's INR (its table and weights are updated in
    place) against an explicit grid; Adam state lives in a torch workspace."""

    def __init__(self, volume: Volume, batch=1 << 18, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15, seed=0,
                 dtype="bf16"):
        self.volume = volume
        d = TrainDesc()
        d.batch, d.lr, d.beta1, d.beta2, d.eps = int(batch), float(lr), float(beta1), float(beta2), float(eps)
        d.seed, d.mlp_dtype = int(seed) & 0xFFFFFFFFFFFFFFFF, _dtype(dtype)
        self.desc = d
        ws = C.c_size_t()
        _check(lib().cinr_train_workspace_size(volume.h, C.byref(d), C.byref(ws)))
        self.workspace = torch.empty(ws.value, dtype=torch.uint8, device=volume.table.device)
        h = C.c_void_p()
        _check(lib().cinr_train_create(volume.h, C.byref(d), _ptr(self.workspace), ws.value, _stream(), C.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.cinr_train_destroy(self.h)
            self.h = None

    @staticmethod
    def _grid(grid):
        if grid is None:
            return None, None
        dims = np.array([grid.shape[2], grid.shape[1], grid.shape[0]], np.int32)
        return grid.contiguous(), dims

    def points(self, step, grid=None):
        """(u [batch][3], target [batch] or None) of training step `step`."""
        g, dims = self._grid(grid)
        dev = self.volume.table.device
        u = torch.empty((self.desc.batch, 3), dtype=torch.float32, device=dev)
        t = torch.empty(self.desc.batch, dtype=torch.float32, device=dev) if g is not None else None
        _check(lib().cinr_train_points(self.h, _ptr(g), dims.ctypes.data_as(C.c_void_p) if dims is not None else None,
                                       int(step), _ptr(u), _ptr(t), _stream()))
        return u, t

    def gradients(self, u, target):
        """(loss, table gradient [entries][F], weight gradient) of the given points."""
        u = u.contiguous()
        target = target.contiguous()
        v = self.volume
        gt = torch.empty_like(v.table)
        gw = torch.empty_like(v.weights)
        loss = torch.empty(1, dtype=torch.float32, device=u.device)
        _check(lib().cinr_train_gradients(self.h, _ptr(u), _ptr(target), u.shape[0], _ptr(loss), _ptr(gt), _ptr(gw),
                                          _stream()))
        return loss, gt, gw

    def set_lr(self, lr):
        _check(lib().cinr_train_set_lr(self.h, float(lr)))

    def step(self, grid, step, loss=None):
        """One Adam step on batch `step`; `loss` (f32 [1] tensor) receives the batch loss."""
        g, dims = self._grid(grid)
        _check(lib().cinr_train_step(self.h, _ptr(g), dims.ctypes.data_as(C.c_void_p), int(step), _ptr(loss),
                                     _stream()))


def adam_update(p, m, v, g, step, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15, clear_grad=False):
    """In-place Adam update of float32 tensors (the trainer's optimiser)."""
    _check(lib().cinr_adam_update(_ptr(p), _ptr(m), _ptr(v), _ptr(g), p.numel(), int(step), float(lr), float(beta1),
                                  float(beta2), float(eps), 1 if clear_grad else 0, _stream()))


class ViewDesc(C.Structure):
    _fields_ = [("volume", C.c_void_p), ("camera", CameraDesc), ("d_tf", C.c_void_p), ("params", RenderParams),
                ("d_rgba", C.c_void_p), ("d_stats", C.c_void_p), ("d_workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t)]


class MultiViewRenderer:
    """Renders frames of several views through one shared cache
    (cinr_render_views); owns each view's render workspace and statistics."""

    def __init__(self, n_views, device="cuda"):
        self.device = device
        self.ws = [None] * n_views
        self.stats = torch.zeros((n_views, len(STAT_FIELDS)), dtype=torch.int64, device=device)
        self._keep = []

    def describe(self, views, step, lod_scale=0.0, frame_index=0, seed=0, ert_threshold=2.0, samples_per_iter=32,
                 dtype="f32", outs=None, pipe_depth=0, xcd_bands=0, adapt_max_exp=0, path=None, lod_context=0.0,
                 waves_per_simd=0, ert_records=None):
        """The cinr_view array of `views` (list of (volume, camera, tf)) and
        their output images; the TF tensors are kept alive by the renderer.
        ert_records: optional list of per-view early-termination records."""
        n = len(views)
        arr = (ViewDesc * n)()
        outs = outs or [None] * n
        keep = []
        for i, (vol, cam, tf) in enumerate(views):
            need = _workspace_size(vol, cam.width, cam.height, samples_per_iter, path)
            if self.ws[i] is None or self.ws[i].numel() < need:
                self.ws[i] = torch.empty(need, dtype=torch.uint8, device=self.device)
            if outs[i] is None:
                outs[i] = torch.empty((cam.height, cam.width, 4), dtype=torch.float32, device=self.device)
            t = tf if torch.is_tensor(tf) else torch.as_tensor(np.asarray(tf, np.float32))
            t = t.to(device=self.device, dtype=torch.float32).contiguous()
            keep.append(t)
            v = arr[i]
            v.volume = vol.h.value
            v.camera = camera_desc(cam)
            v.d_tf = t.data_ptr()
            p = v.params
            p.step, p.lod_scale, p.ert_threshold = float(step), float(lod_scale), float(ert_threshold)
            p.seed, p.frame_index, p.samples_per_iter = int(seed) & 0xFFFFFFFF, int(frame_index), int(samples_per_iter)
            p.mode, p.mlp_dtype = CACHED, _dtype(dtype)
            p.pipe_depth, p.xcd_bands = int(pipe_depth), int(xcd_bands)
            p.adapt_max_exp = int(adapt_max_exp)
            p.lod_context = float(lod_context)
            p.waves_per_simd = int(waves_per_simd)
            _set_path(p, path)
            p.ert_record = _ert_record(None if ert_records is None else ert_records[i], cam)
            v.d_rgba = outs[i].data_ptr()
            v.d_stats = self.stats[i].data_ptr()
            v.d_workspace = self.ws[i].data_ptr()
            v.workspace_bytes = self.ws[i].numel()
        self._keep = keep
        return arr, outs

    def render(self, cache: Cache, views, step, lod_scale=0.0, frame_index=0, seed=0, ert_threshold=2.0,
               samples_per_iter=32, dtype="f32", outs=None, pipe_depth=0, xcd_bands=0, adapt_max_exp=0, path=None,
               lod_context=0.0, waves_per_simd=0, ert_records=None):
        """views: list of (volume, camera, tf); returns the list of RGBA images."""
        arr, outs = self.describe(views, step, lod_scale, frame_index, seed, ert_threshold, samples_per_iter, dtype,
                                  outs, pipe_depth, xcd_bands, adapt_max_exp, path, lod_context, waves_per_simd,
                                  ert_records)
        _check(lib().cinr_render_views(cache.h, len(views), arr, _stream()))
        return outs

    def last_stats(self):
        v = self.stats.cpu().numpy()
        return [{k: int(row[i]) for i, k in enumerate(STAT_FIELDS)} for row in v]


class FrameGraph:
    """Captured multi-view frames (cinr_frame_graph_*): made once for a fixed
    set of views (list of (volume, camera, tf)) and parameters; each render()
    replays the frame with new cameras (same sizes and projections) and a new
    frame index.  The TF tensors (`tfs`) may be updated in place between
    frames.  Owns the views' workspaces, images and statistics."""

    def __init__(self, cache: Cache, views, step, lod_scale=0.0, seed=0, ert_threshold=2.0, samples_per_iter=32,
                 dtype="f32", pipe_depth=0, xcd_bands=0, adapt_max_exp=0, device="cuda", path=None, lod_context=0.0,
                 waves_per_simd=0):
        self.cache = cache
        self.volumes = [v for v, _, _ in views]
        self.mv = MultiViewRenderer(len(views), device)
        arr, self.outs = self.mv.describe(views, step, lod_scale, 0, seed, ert_threshold, samples_per_iter, dtype,
                                          None, pipe_depth, xcd_bands, adapt_max_exp, path, lod_context,
                                          waves_per_simd)
        self.tfs = list(self.mv._keep)
        self.n = len(views)
        h = C.c_void_p()
        _check(lib().cinr_frame_graph_create(cache.h, self.n, arr, C.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.cinr_frame_graph_destroy(self.h)
            self.h = None

    def render(self, cameras, frame_index):
        """Renders one frame; returns the list of RGBA images (the same tensors every frame)."""
        if len(cameras) != self.n:
            raise ValueError(f"{len(cameras)} cameras for {self.n} views")
        arr = (CameraDesc * self.n)(*[camera_desc(c) for c in cameras])
        _check(lib().cinr_frame_graph_render(self.h, arr, int(frame_index), _stream()))
        return self.outs

    def set_device_iterations(self, k):
        """Wavefront iterations after the first march queued in the graph (0 to 16)."""
        _check(lib().cinr_frame_graph_set_device_iterations(self.h, int(k)))

    def counts(self):
        """(graph frames, eager frames, graph frames with further iterations)."""
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().cinr_frame_graph_counts(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def last_stats(self):
        return self.mv.last_stats()


def tuned_launch(volume, width, height):
    """(pipe_depth, xcd_bands, trials_left, waves_per_simd) of the online
    launch tuning."""
    p, b, w, t = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().cinr_tuned_launch(volume.h, int(width), int(height), C.byref(p), C.byref(b), C.byref(w),
                                   C.byref(t)))
    return p.value, b.value, t.value, w.value
