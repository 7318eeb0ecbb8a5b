"""The C ABI on the CPU: the library loads, exports every function that
include/cinr.h declares, and its host-side logic (argument validation,
LoD/brick geometry, workspace sizing) behaves as documented.

No call in this file launches a kernel or touches device memory: volume
creation only records the parameter pointers, so placeholder addresses are
passed for them.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2504_18001_amd import cinr, configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cinr.h")

OK, INVALID_ARG = 0, -1


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cinr_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 16
    L = cinr.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert missing == []
    # and the binding declares a signature for each of them
    for n in names:
        assert getattr(L, n).argtypes is not None or n == "cinr_last_error", n


def fake_volume(arch, macro_cell=0):
    """Creates a volume with placeholder parameter addresses (never read)."""
    d = cinr.VolumeDesc()
    for a in range(3):
        d.dims[a] = arch.dims[a]
    d.n_levels, d.n_features, d.log2_table = arch.n_levels, arch.n_features, arch.log2_table
    for l, n in enumerate(arch.level_res):
        d.level_res[l] = n
    d.n_layers = len(arch.widths) - 1
    for i, w in enumerate(arch.widths):
        d.widths[i] = w
    d.value_scale, d.value_offset = 1.0, 0.0
    d.d_table = C.c_void_p(0x10000)
    d.d_weights = C.c_void_p(0x20000)
    if macro_cell:
        d.d_macrocells = C.c_void_p(0x30000)
        d.macrocell_size = macro_cell
    h = C.c_void_p()
    rc = cinr.lib().cinr_create_volume_inr(C.byref(d), C.byref(h))
    return rc, h, d


def test_null_arguments_are_rejected_with_a_message():
    L = cinr.lib()
    h = C.c_void_p()
    assert L.cinr_create_volume_inr(None, C.byref(h)) == INVALID_ARG
    assert b"null" in L.cinr_last_error()
    assert L.cinr_lod_geometry(None, 16, 4, None, None) == INVALID_ARG
    assert L.cinr_render_frame(None, None, None, None, None, None, None, None, 0, None) == INVALID_ARG


@pytest.mark.parametrize("field,value", [("n_levels", 0), ("n_levels", 33), ("n_features", 3), ("log2_table", 3),
                                         ("n_layers", 0)])
def test_invalid_volume_descriptors(field, value):
    rc, h, d = fake_volume(configs.ARCH_SMALL)
    assert rc == OK
    cinr.lib().cinr_destroy_volume(h)
    setattr(d, field, value)
    h2 = C.c_void_p()
    assert cinr.lib().cinr_create_volume_inr(C.byref(d), C.byref(h2)) == INVALID_ARG
    assert len(cinr.lib().cinr_last_error()) > 0


def test_first_width_must_match_the_encoding():
    _, h, d = fake_volume(configs.ARCH_SMALL)
    cinr.lib().cinr_destroy_volume(h)
    d.widths[0] = d.widths[0] + 1
    h2 = C.c_void_p()
    assert cinr.lib().cinr_create_volume_inr(C.byref(d), C.byref(h2)) == INVALID_ARG


@pytest.mark.parametrize("arch,brick,n_lods", [(configs.ARCH_SMALL, 8, 2), (configs.ARCH_512, 16, 4),
                                               (configs.ARCH_TERA, 16, 6)])
def test_lod_geometry_matches_the_oracle(arch, brick, n_lods):
    rc, h, _ = fake_volume(arch)
    assert rc == OK
    try:
        nb = np.zeros((n_lods, 3), np.int32)
        off = np.zeros(n_lods + 1, np.int64)
        rc = cinr.lib().cinr_lod_geometry(h, brick, n_lods, nb.ctypes.data_as(C.c_void_p),
                                          off.ctypes.data_as(C.c_void_p))
        assert rc == OK
        _, onb, ooff = O.lod_geometry(arch.dims, brick, n_lods)
        assert np.array_equal(nb, np.asarray(onb).reshape(n_lods, 3))
        assert np.array_equal(off, np.asarray(ooff))
    finally:
        cinr.lib().cinr_destroy_volume(h)


def test_brick_key_counts_of_the_two_small_configurations():
    # Section 4.3.2 geometry, stride B-1: 9^3 + 5^3 and 35^3 + 18^3 + 9^3 + 5^3 keys
    for arch, brick, n_lods, keys in ((configs.ARCH_SMALL, 8, 2, 854), (configs.ARCH_512, 16, 4, 49561)):
        _, h, _ = fake_volume(arch)
        off = np.zeros(n_lods + 1, np.int64)
        assert cinr.lib().cinr_lod_geometry(h, brick, n_lods, None, off.ctypes.data_as(C.c_void_p)) == OK
        assert off[-1] == keys
        cinr.lib().cinr_destroy_volume(h)


def test_invalid_brick_geometry_is_rejected():
    _, h, _ = fake_volume(configs.ARCH_SMALL)
    try:
        for brick, n_lods in ((1, 2), (8, 0), (8, cinr.MAX_LODS + 1)):
            assert cinr.lib().cinr_lod_geometry(h, brick, n_lods, None, None) == INVALID_ARG
    finally:
        cinr.lib().cinr_destroy_volume(h)


def cache_desc(brick=8, n_lods=2, pool=96, max_requests=16, pool_dtype=cinr.F32):
    d = cinr.CacheDesc()
    d.brick, d.n_lods, d.pool_bricks, d.max_requests = brick, n_lods, pool, max_requests
    d.rank_window, d.ranking = 1000, cinr.RANK_PRIORITY
    d.pool_dtype = pool_dtype
    return d


def test_cache_workspace_grows_with_the_pool_and_rejects_bad_descriptors():
    _, h, _ = fake_volume(configs.ARCH_SMALL)
    L = cinr.lib()
    try:
        sizes = []
        for pool in (16, 96, 4096):
            b = C.c_size_t()
            assert L.cinr_cache_workspace_size(h, C.byref(cache_desc(pool=pool)), C.byref(b)) == OK
            sizes.append(b.value)
        assert sizes[0] < sizes[1] < sizes[2]
        b = C.c_size_t()
        # 0 <= max_requests <= 256, pool_bricks >= 0
        assert L.cinr_cache_workspace_size(h, C.byref(cache_desc(max_requests=0)), C.byref(b)) == OK
        assert L.cinr_cache_workspace_size(h, C.byref(cache_desc(max_requests=-1)), C.byref(b)) == INVALID_ARG
        assert L.cinr_cache_workspace_size(h, C.byref(cache_desc(max_requests=257)), C.byref(b)) == INVALID_ARG
        assert L.cinr_cache_workspace_size(h, C.byref(cache_desc(pool=-1)), C.byref(b)) == INVALID_ARG
        # the pool holds binary32 or binary16 values, nothing else
        assert L.cinr_cache_workspace_size(h, C.byref(cache_desc(pool_dtype=cinr.F16)), C.byref(b)) == OK
        for bad in (cinr.BF16, cinr.BF16X3, -1):
            assert L.cinr_cache_workspace_size(h, C.byref(cache_desc(pool_dtype=bad)), C.byref(b)) == INVALID_ARG
    finally:
        L.cinr_destroy_volume(h)


def test_mixed_pool_descriptors():
    _, h, _ = fake_volume(configs.ARCH_SMALL)
    L = cinr.lib()

    def size(**kw):
        d = cache_desc(pool=40, max_requests=8)
        for k, v in kw.items():
            setattr(d, k, v)
        b = C.c_size_t()
        return L.cinr_cache_workspace_size(h, C.byref(d), C.byref(b))

    try:
        assert size(f16_lods=0b10, pool_bricks_f16=16) == OK
        assert size(f16_lods=0b01, pool_bricks_f16=32) == OK
        assert size(f16_lods=0b10, pool_bricks_f16=16, pool_dtype=cinr.F16) == INVALID_ARG  # classes need F32
        assert size(f16_lods=0b11, pool_bricks_f16=16) == INVALID_ARG   # every LoD binary16: one class
        assert size(f16_lods=0b100, pool_bricks_f16=16) == INVALID_ARG  # LoD 2 does not exist
        assert size(f16_lods=0b10, pool_bricks_f16=0) == INVALID_ARG
        assert size(f16_lods=0b10, pool_bricks_f16=40) == INVALID_ARG   # no binary32 slot
        assert size(f16_lods=0b10, pool_bricks_f16=7) == INVALID_ARG    # fewer slots than max_requests
        assert size(f16_lods=0b10, pool_bricks_f16=33) == INVALID_ARG
    finally:
        L.cinr_destroy_volume(h)


def test_f16_lods_from_error_bounds():
    assert cinr.f16_lods_for_bounds([1e-5, 2.0 ** -12, 1e-3, 0.0]) == 0b0110
    assert cinr.f16_lods_for_bounds([0.0, 0.0]) == 0


def test_render_workspace_covers_the_per_ray_buffers():
    _, h, _ = fake_volume(configs.ARCH_512, macro_cell=16)
    L = cinr.lib()
    try:
        b = C.c_size_t()
        assert L.cinr_render_workspace_size(h, 1920, 1080, 32, C.byref(b)) == OK
        npix = 1920 * 1080
        # per pixel at least: two live lists, k, pending pixel and count, S values, S miss records
        assert b.value >= npix * (5 * 4 + 32 * 4 + 32 * 16)
        assert L.cinr_render_workspace_size(h, 1920, 1080, 65, C.byref(b)) == INVALID_ARG
        assert L.cinr_render_workspace_size(h, 0, 1080, 32, C.byref(b)) == INVALID_ARG
    finally:
        L.cinr_destroy_volume(h)


def test_noalloc_frame_checks_its_arguments_before_any_device_work():
    """The allocation-free frame call rejects null arguments and frames whose
    workspace exceeds its fixed device array (before touching the device)."""
    L = cinr.lib()
    assert L.cinr_render_frame_noalloc(None, None, None, None, None, None, None, None) == INVALID_ARG
    _, h, _ = fake_volume(configs.ARCH_512, macro_cell=16)
    try:
        cam = cinr.CameraDesc()
        cam.projection, cam.width, cam.height = cinr.PERSPECTIVE, 1920, 1080
        p = cinr.RenderParams()
        p.step, p.samples_per_iter, p.mode = 0.5, 8, cinr.UNCACHED_DIRECT
        rc = L.cinr_render_frame_noalloc(None, h, C.byref(cam), C.c_void_p(0x40000), C.byref(p),
                                         C.c_void_p(0x50000), None, None)
        assert rc == -2  # CINR_OUT_OF_MEMORY
        assert b"fixed scratch array" in L.cinr_last_error()
        b = C.c_size_t()
        assert L.cinr_render_workspace_size(h, 1920, 1080, 8, C.byref(b)) == OK
        assert b.value > cinr.NOALLOC_SCRATCH_BYTES
        p.samples_per_iter = 0
        assert L.cinr_render_frame_noalloc(None, h, C.byref(cam), C.c_void_p(0x40000), C.byref(p),
                                           C.c_void_p(0x50000), None, None) == INVALID_ARG
    finally:
        L.cinr_destroy_volume(h)


def test_timing_modes():
    _, h, _ = fake_volume(configs.ARCH_SMALL)
    L = cinr.lib()
    try:
        for mode in (0, 1, 2, 0):
            assert L.cinr_set_timing(h, mode) == OK
        assert L.cinr_set_timing(h, 3) == INVALID_ARG
        assert L.cinr_set_timing(h, -1) == INVALID_ARG
        assert b"timing mode" in L.cinr_last_error()
        assert L.cinr_set_timing(None, 1) == INVALID_ARG
    finally:
        L.cinr_destroy_volume(h)


def test_frame_graph_arguments_are_checked_before_any_device_work():
    L = cinr.lib()
    g = C.c_void_p()
    assert L.cinr_frame_graph_create(None, 1, None, C.byref(g)) == INVALID_ARG
    assert L.cinr_frame_graph_render(None, None, 0, None) == INVALID_ARG
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    assert L.cinr_frame_graph_counts(None, C.byref(a), C.byref(b), C.byref(c)) == INVALID_ARG


def test_path_tracer_workspace_and_arguments():
    _, h, _ = fake_volume(configs.ARCH_SMALL)
    L = cinr.lib()
    try:
        rb, pb = C.c_size_t(), C.c_size_t()
        assert L.cinr_render_workspace_size(h, 64, 48, 8, C.byref(rb)) == OK
        assert L.cinr_path_workspace_size(h, 64, 48, 8, C.byref(pb)) == OK
        # 128 bytes of path state per pixel on top of the ray marcher's workspace
        assert 64 * 48 * 128 <= pb.value - rb.value < 64 * 48 * 128 + 512
        assert L.cinr_path_workspace_size(h, 1 << 14, 1 << 13, 1, C.byref(pb)) == INVALID_ARG  # 2^27 pixels
        assert L.cinr_pt_free_flight(None, -1, None, None) == INVALID_ARG
        assert L.cinr_pt_free_flight(None, 0, None, None) == OK
        cam = configs.SMALL.camera(0)
        cam.width, cam.height = 64, 48
        cd = cinr.camera_desc(cam)
        ws = C.c_void_p(0x40000)  # placeholders: every call below fails before any device work

        def params(**kw):
            p = cinr.RenderParams()
            p.step, p.lod_scale, p.ert_threshold, p.samples_per_iter = 0.5, 0.01, 2.0, 8
            p.mode, p.mlp_dtype = cinr.UNCACHED_DIRECT, cinr.F32
            cinr._set_path(p, dict(density=0.05, spp=2, max_bounces=2))
            for k, v in kw.items():
                setattr(p, k, v)
            return p

        def render(p, ws_bytes):
            return L.cinr_render_frame(None, h, C.byref(cd), C.c_void_p(0x50000), C.byref(p), C.c_void_p(0x60000),
                                       None, ws, ws_bytes, None)

        big = pb.value * 4
        for bad in (dict(pipeline=2), dict(pt_density=0.0), dict(pt_density=float("nan")), dict(pt_spp=0),
                    dict(pt_spp=65536), dict(pt_max_bounces=0), dict(adapt_max_exp=1), dict(waves_per_simd=5),
                    dict(waves_per_simd=-1), dict(lod_context=-0.5), dict(lod_context=2.0)):
            assert render(params(**bad), big) == INVALID_ARG, bad
        # a ray-marching workspace is too small for the path tracer
        assert render(params(), rb.value) == -2
    finally:
        L.cinr_destroy_volume(h)
