"""GPU parity against the CPU oracle (through the C ABI).

Tolerances: value-plane results (INR values, images) within max abs 2e-3 for
the FP32 MLP and 8e-3 for BF16/FP16 (images: max abs RGBA); decision-plane
results (page table, slot owners, stamps, ranks, request counts, request
lists, miss lists, eviction logs) bit-exact.
"""
import math

import numpy as np
import pytest
import torch

from paper_2504_18001_amd import configs, synth
from tests.helpers import inr_params, oracle_inr, value_range

pytestmark = pytest.mark.gpu

TOL = {"f32": 2e-3, "bf16": 8e-3, "f16": 8e-3, "bf16x3": 8e-3}
# per-value (INR output) tolerances: FP32 only suffers reordering; split
# BF16 carries about 16 significant bits per operand
VTOL = {"f32": 1e-4, "bf16": 8e-3, "f16": 2e-3, "bf16x3": 2e-4}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_18001_amd import cinr
    cinr.lib()  # fails loudly if the library is missing


def gpu_volume(arch, seed, dims=None, macrocells=None, macro_cell=0):
    from paper_2504_18001_amd import cinr
    t, w = inr_params(arch, seed)
    s, o = value_range(arch, seed)
    return cinr.Volume(arch, t, w, s, o, macrocells=macrocells, macro_cell=macro_cell, dims=dims)


ARCHS = [("small", configs.ARCH_SMALL), ("inr512", configs.ARCH_512), ("tera", configs.ARCH_TERA)]


@pytest.mark.parametrize("name,arch", ARCHS)
@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16", "bf16x3"])
def test_infer_points(name, arch, dtype):
    vol = gpu_volume(arch, 0)
    m = oracle_inr(arch, 0)
    rng = np.random.default_rng(7)
    n = 4099  # several workgroup rounds plus a ragged tail
    V = np.asarray(arch.dims, np.float64)
    x = (rng.uniform(-0.5, 1.0, size=(n, 3)) * (V - 1)).astype(np.float32)  # includes positions clamped to the box
    got = vol.infer_points(torch.from_numpy(x).cuda(), dtype).cpu().numpy()
    ref = m.value(x.astype(np.float64))
    err = np.abs(got - ref)
    print(name, dtype, "max", err.max(), "mean", err.mean())
    assert err.max() <= VTOL[dtype]


@pytest.mark.parametrize("name,arch,B,n_lods", [("small", configs.ARCH_SMALL, 8, 2), ("inr512", configs.ARCH_512, 16, 4)])
@pytest.mark.parametrize("dtype", ["f32", "bf16", "bf16x3"])
def test_decode_bricks(name, arch, B, n_lods, dtype):
    vol = gpu_volume(arch, 1)
    m = oracle_inr(arch, 1)
    nb, _ = vol.geometry(B, n_lods)
    reqs = synth.random_requests(nb.tolist(), 37, seed=3)
    # include the last brick of every LoD (clamped samples) and the origin brick
    extra = [[L, *(nb[L] - 1)] for L in range(n_lods)] + [[0, 0, 0, 0]]
    reqs = np.concatenate([reqs, np.asarray(extra, np.int32)])
    got = vol.decode_bricks(torch.from_numpy(reqs).cuda(), B, dtype).cpu().numpy()
    ref = m.decode_bricks(reqs, B, n_lods)
    err = np.abs(got - ref)
    print(name, dtype, "max", err.max())
    assert err.max() <= VTOL[dtype]


STAGED = [(1, 0), (1, 64), (2, 32), (4, 0), (4, 64), (8, 32), (16, 0), (16, 64)]


@pytest.mark.parametrize("name,arch,B,n_lods", [("small", configs.ARCH_SMALL, 8, 2), ("inr512", configs.ARCH_512, 16, 4),
                                                ("tera", configs.ARCH_TERA, 16, 6)])
@pytest.mark.parametrize("dtype", ["f32", "bf16x3"])
def test_decode_bricks_staged_is_bit_identical(name, arch, B, n_lods, dtype):
    """Decoding with LDS-staged corner boxes, every launch shape, against the
    unstaged decode (bit for bit: same cells, weights and order) and the
    oracle; random requests of every LoD plus the clamped last brick of each
    LoD, the origin brick and two invalid requests (NaN bricks)."""
    vol = gpu_volume(arch, 1)
    m = oracle_inr(arch, 1)
    nb, _ = vol.geometry(B, n_lods)
    reqs = synth.random_requests(nb.tolist(), 45, seed=4)
    extra = [[L, *(nb[L] - 1)] for L in range(n_lods)] + [[0, 0, 0, 0], [0, int(nb[0][0]), 0, 0], [-1, 0, 0, 0]]
    reqs = torch.from_numpy(np.concatenate([reqs, np.asarray(extra, np.int32)])).cuda()
    base = vol.decode_bricks_shaped(reqs, B, dtype, parts=0).cpu().numpy()
    ref = m.decode_bricks(reqs[:-2].cpu().numpy(), B, n_lods)
    assert np.abs(base[:-2] - ref).max() <= VTOL[dtype]
    assert np.isnan(base[-2:]).all() and np.isfinite(base[:-2]).all()
    for parts, kib in STAGED:
        if B % parts:
            continue
        got = vol.decode_bricks_shaped(reqs, B, dtype, parts=parts, stage_kib=kib).cpu().numpy()
        assert np.array_equal(got, base, equal_nan=True), (parts, kib, np.nanmax(np.abs(got - base)))
    # a short list is split into more parts on the device; a list of 1536
    # requests (two per resident workgroup) keeps each shape's own parts
    big = torch.from_numpy(synth.random_requests(nb.tolist(), 1536, seed=5)).cuda()
    bbase = vol.decode_bricks_shaped(big, B, dtype, parts=0).cpu().numpy()
    for parts, kib in STAGED:
        if B % parts:
            continue
        got = vol.decode_bricks_shaped(big, B, dtype, parts=parts, stage_kib=kib).cpu().numpy()
        assert np.array_equal(got, bbase), ("1536 requests", parts, kib)


def test_decode_shape_arguments():
    from paper_2504_18001_amd import cinr
    vol = gpu_volume(configs.ARCH_SMALL, 0)
    reqs = torch.zeros((1, 4), dtype=torch.int32, device="cuda")
    for parts, kib in ((3, 64), (4, 48), (-1, 64), (2, -32)):
        with pytest.raises(cinr.CinrError):
            vol.decode_bricks_shaped(reqs, 8, parts=parts, stage_kib=kib)
    with pytest.raises(cinr.CinrError, match="multiple"):
        vol.decode_bricks_shaped(reqs, 8, parts=16, stage_kib=64)
    vol.set_decode_shape(4, 32)
    a = vol.decode_bricks(reqs, 8).cpu().numpy()
    vol.set_decode_shape(0)
    assert np.array_equal(a, vol.decode_bricks(reqs, 8).cpu().numpy())


def test_decode_invalid_request_gives_nan():
    vol = gpu_volume(configs.ARCH_SMALL, 0)
    reqs = torch.tensor([[0, 0, 0, 0], [0, 99, 0, 0], [17, 0, 0, 0]], dtype=torch.int32, device="cuda")
    out = vol.decode_bricks(reqs, 8).cpu().numpy()
    assert np.isfinite(out[0]).all() and np.isnan(out[1]).all() and np.isnan(out[2]).all()


def test_macrocells_match_oracle():
    vol = gpu_volume(configs.ARCH_SMALL, 0)
    m = oracle_inr(configs.ARCH_SMALL, 0)
    got = vol.build_macrocells(16).cpu().numpy()
    ref = m.macrocells(16)
    assert np.abs(got - ref).max() <= 1e-4


def _render_gpu(vol, cam, tf, w, frame, mode, dtype="f32", cache=None, ert=2.0, S=None, renderer=None, adapt=0,
                step=None, lod_context=0.0):
    from paper_2504_18001_amd import cinr
    r = renderer or cinr.Renderer()
    img = r.render(vol, cam, tf, step or w.step, w.lod_scale, frame_index=frame, seed=w.seed, ert_threshold=ert,
                   samples_per_iter=S or w.samples_per_iter, mode=mode, dtype=dtype, cache=cache, adapt_max_exp=adapt,
                   lod_context=lod_context)
    return img.cpu().numpy().astype(np.float64), r.last_stats()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_uncached_render_small(dtype):
    from oracle import oracle as O
    from paper_2504_18001_amd import cinr
    w = configs.SMALL
    vol = gpu_volume(w.arch, 0)
    m = oracle_inr(w.arch, 0)
    for frame in (0, 3):
        cam = w.camera(frame)
        cam.width, cam.height = 72, 56  # ragged 8x8 tiles
        tf = w.tf(frame)
        img, st = _render_gpu(vol, cam, tf, w, frame, cinr.UNCACHED_DIRECT, dtype)
        p = O.make_params(w.step, w.lod_scale, seed=w.seed, frame_index=frame, samples_per_iter=w.samples_per_iter,
                          mode=O.UNCACHED_DIRECT)
        ref, rst = O.render_uncached(m, cam, tf, p)
        err = np.abs(img - ref).max()
        print("uncached", dtype, frame, err, st, rst)
        assert err <= TOL[dtype]
        assert st["rays"] == rst["rays"] and st["samples"] == rst["samples"] and st["misses"] == rst["misses"]


@pytest.mark.parametrize("dtype", ["f32", "bf16x3"])
def test_uncached_lattice_render_small(dtype):
    """The lattice mode (each sample interpolated from the INR's values at its
    8 LoD-0 lattice points) against the oracle's: images within the
    tolerance, statistics equal.  Then the invariant that a cache holding
    every LoD-0 brick renders the lattice image bit for bit (the same lattice
    values, interpolation, compositing and early termination)."""
    from oracle import oracle as O
    from paper_2504_18001_amd import cinr
    w = configs.SMALL
    vol = gpu_volume(w.arch, 0)
    m = oracle_inr(w.arch, 0)
    B = 8
    nb, off = vol.geometry(B, 1)
    n0 = int(off[1])
    cache = cinr.Cache(vol, B, 1, n0, 16)
    cache.prefill(torch.arange(n0, dtype=torch.int32, device="cuda"), dtype=dtype)
    for frame in (0, 3):
        cam = w.camera(frame)
        cam.width, cam.height = 72, 56  # ragged 8x8 tiles
        tf = w.tf(frame)
        img, st = _render_gpu(vol, cam, tf, w, frame, cinr.UNCACHED_LATTICE, dtype, S=32)
        p = O.make_params(w.step, w.lod_scale, seed=w.seed, frame_index=frame, samples_per_iter=32,
                          mode=O.UNCACHED_LATTICE)
        ref, rst = O.render_uncached(m, cam, tf, p)
        err = np.abs(img - ref).max()
        print("lattice", dtype, frame, err, st, rst)
        assert err <= TOL[dtype]
        for k in ("rays", "samples", "hits", "misses", "skipped"):
            assert st[k] == rst[k], (k, st[k], rst[k])
        for ert in (2.0, 0.95):
            a, _ = _render_gpu(vol, cam, tf, w, frame, cinr.UNCACHED_LATTICE, dtype, S=32, ert=ert)
            c, cst = _render_gpu(vol, cam, tf, w, frame, cinr.CACHED, dtype, cache=cache, S=32, ert=ert)
            np.testing.assert_array_equal(c, a, err_msg=f"frame {frame} ert {ert}")
            assert cst["misses"] == 0 and cst["fallbacks"] == 0


@pytest.mark.parametrize("ranking", [1, 0])
def test_selection_among_many_candidates(ranking):
    """Frames requesting far more bricks than one 2048-entry chunk of the
    selection (the 512^3 architecture with 8^3 bricks: 389,017 keys, a
    four-pass selection run in one launch): the request list must be the
    first max_requests requested keys by (rank desc, key asc), or by key for
    the timestamp variant, recomputed on the host from the dumped counts and
    ranks.  Two frames, so that the second adds to ranks of the first."""
    from paper_2504_18001_amd import cinr
    w = configs.HD512
    vol = gpu_volume(w.arch, 0)
    cache = cinr.Cache(vol, 8, 1, 4096, 256, ranking=ranking, keep_request_counts=True)
    r = cinr.Renderer()
    for f in range(2):
        cam = w.camera(f)
        cam.width, cam.height = 256, 144
        r.render(vol, cam, w.tf(f), w.step, 0.0, frame_index=f, seed=w.seed, mode=cinr.CACHED, dtype="f32",
                 cache=cache)
        req = cache.dump(cinr.DUMP_REQ_COUNT)
        rank = cache.dump(cinr.DUMP_RANK)
        got = cache.dump(cinr.DUMP_REQUEST_LIST)
        touched = np.nonzero(req)[0]
        print("frame", f, "requested bricks", len(touched), "selected", len(got))
        assert len(touched) > 4 * 2048
        if ranking:
            order = np.lexsort((touched, -rank[touched]))
            want = touched[order][:256]
        else:
            want = np.sort(touched)[:256]
        np.testing.assert_array_equal(got, want.astype(np.int32), err_msg=f"frame {f}")
        # ranks of this frame's requests: a new brick f + c - 1, an old one rank + c (clamped)
        assert (rank[touched] >= f).all()


def test_uncached_lattice_arguments():
    from paper_2504_18001_amd import cinr
    w = configs.SMALL
    vol = gpu_volume(w.arch, 0)
    cam = w.camera(0)
    with pytest.raises(cinr.CinrError, match="samples_per_iter >= 8"):
        _render_gpu(vol, cam, w.tf(0), w, 0, cinr.UNCACHED_LATTICE, S=4)


def _compare_state(gc, oc, frame, check_misses=True):
    from paper_2504_18001_amd import cinr
    np.testing.assert_array_equal(gc.dump(cinr.DUMP_PAGE_TABLE), oc.page_table(), err_msg=f"page table f{frame}")
    np.testing.assert_array_equal(gc.dump(cinr.DUMP_SLOT_OWNER), oc.owner(), err_msg=f"owner f{frame}")
    np.testing.assert_array_equal(gc.dump(cinr.DUMP_LAST_USED), oc.last_used(), err_msg=f"last_used f{frame}")
    np.testing.assert_array_equal(gc.dump(cinr.DUMP_RANK), oc.rank(), err_msg=f"rank f{frame}")
    np.testing.assert_array_equal(gc.dump(cinr.DUMP_REQ_COUNT), oc.req_count(), err_msg=f"req f{frame}")
    np.testing.assert_array_equal(gc.dump(cinr.DUMP_REQUEST_LIST), oc.request_list(), err_msg=f"list f{frame}")
    np.testing.assert_array_equal(gc.dump(cinr.DUMP_EVICTION_LOG), oc.evict_log(), err_msg=f"evlog f{frame}")
    if check_misses:
        gpk, gpos = gc.dump(cinr.DUMP_MISS_LIST)
        opk, opos = oc.miss_list()
        np.testing.assert_array_equal(gpk, opk, err_msg=f"miss list f{frame}")
        np.testing.assert_array_equal(gpos.view(np.uint32), opos.view(np.uint32), err_msg=f"miss pos f{frame}")


def run_cached_sequence(w, frames, width, height, dtype="f32", dims=None, pool=None, max_req=None, ranking=1,
                        preload=None, S=None, macro=False, tf_fn=None, n_lods=None, brick=None, adapt=0,
                        pool_dtype="f32", lod_context=0.0, f16_lods=0, pool_bricks_f16=0, caches=None,
                        virtual_pt=False):
    from oracle import oracle as O
    from paper_2504_18001_amd import cinr
    arch = w.arch
    cs = w.cache
    B = brick or cs.brick
    nl = n_lods or cs.n_lods
    pool = pool if pool is not None else cs.pool_bricks
    max_req = max_req if max_req is not None else cs.max_requests
    preload = cs.preload_period if preload is None else preload
    m = oracle_inr(arch, 0, dims=dims)
    mm = m.macrocells(w.macro_cell) if macro else None
    vol = gpu_volume(arch, 0, dims=dims, macrocells=mm, macro_cell=w.macro_cell if macro else 0)
    gc = cinr.Cache(vol, B, nl, pool, max_req, ranking=ranking, preload_period=preload, miss_log_capacity=1 << 22,
                    evict_log_capacity=1 << 16, keep_request_counts=True, pool_dtype=pool_dtype, f16_lods=f16_lods,
                    pool_bricks_f16=pool_bricks_f16, virtual_page_table=virtual_pt)
    oc = O.OracleCache(m, brick=B, n_lods=nl, pool_bricks=pool, max_requests=max_req, ranking=ranking,
                       preload_period=preload, log_misses=True, pool_f16=pool_dtype == "f16", f16_lods=f16_lods,
                       pool_bricks_f16=pool_bricks_f16)
    if caches is not None:
        caches.extend([gc, oc])
    r = cinr.Renderer()
    worst = 0.0
    for f in frames:
        cam = w.camera(f, dims)
        cam.width, cam.height = width, height
        tf = tf_fn(f) if tf_fn else w.tf(f)
        img, st = _render_gpu(vol, cam, tf, w, f, cinr.CACHED, dtype, cache=gc, S=S, renderer=r, adapt=adapt,
                              lod_context=lod_context)
        p = O.make_params(w.step, w.lod_scale, seed=w.seed, frame_index=f, samples_per_iter=S or w.samples_per_iter,
                          mode=O.CACHED, macro_cell=w.macro_cell if macro else 0, macro_minmax=mm,
                          adapt_max_exp=adapt, lod_context=lod_context)
        ref, rst = oc.render(cam, tf, p)
        err = np.abs(img - ref).max()
        worst = max(worst, err)
        print(f"frame {f}: err {err:.2e} gpu {st} oracle {rst}", flush=True)
        for k in ("rays", "samples", "hits", "fallbacks", "misses", "skipped", "requested", "selected", "evicted"):
            assert st[k] == rst[k], (f, k, st[k], rst[k])
        _compare_state(gc, oc, f)
        assert err <= TOL[dtype], (f, err)
    return worst


def test_cached_sequence_small_parity():
    # 64^3, 128x128, B = 8, 2 LoDs, 96-slot pool, 16 requests per frame:
    # the pool fills after 6 frames and LRU eviction runs from then on.
    w = configs.SMALL
    run_cached_sequence(w, range(12), 128, 128)


def test_cached_sequence_small_bf16_with_macrocells_and_key_order():
    w = configs.SMALL
    run_cached_sequence(w, range(6), 64, 48, dtype="bf16", ranking=0, macro=True,
                        tf_fn=lambda f: synth.tf_window(60, 255))


def test_cached_sequence_512_arch_reduced():
    # the 512^3 architecture (16 levels x 2, T = 2^19, 32-64-64-1) on a
    # 120x104x96 virtual volume, 4 LoDs, B = 16, pre-load of the coarsest LoD
    w = configs.scaled(configs.HD512, 80, 45, orbit_radius=260.0, lod_scale=1.0 / 180.0)
    run_cached_sequence(w, range(8), 80, 45, dims=(120, 104, 96), pool=300, max_req=12, preload=2)


def test_cached_sequence_two_pass_selection():
    # 128x120x112 virtual volume, B = 8, 2 LoDs: about 5,800 keys, so the
    # selection takes two passes (one fused launch); the 160-slot pool fills
    # after 7 frames, then the LRU pass and a separate insertion run
    w = configs.SMALL
    run_cached_sequence(w, range(12), 96, 96, dims=(128, 120, 112), pool=160, max_req=24)
