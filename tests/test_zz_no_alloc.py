"""The allocation-free frame call (cinr_render_frame_noalloc) against
cinr_render_frame, through the C ABI: identical images, frame statistics and
cache state (page table, slot owners, stamps, request list, eviction log), bit
for bit, over consecutive calls whose images shrink.  The fixed device array
keeps whatever the previous call left in it, so a smaller second call checks
that every frame clears what it reads as zero.
"""
import numpy as np
import pytest
import torch

from paper_2504_18001_amd import configs, synth
from tests.helpers import inr_params, value_range

pytestmark = pytest.mark.gpu

# an explicit launch shape: both calls then run the same kernels (the
# allocation-free call times no launch-shape trial)
SHAPE = dict(pipe_depth=1, xcd_bands=1, waves_per_simd=3)
PATH = dict(density=0.06, light_dir=(0.48, 0.6, 0.64), light=(2.5, 2.5, 2.5), ambient=(0.3, 0.35, 0.4),
            max_bounces=3, spp=2, seed=17)
DUMPS = ("DUMP_PAGE_TABLE", "DUMP_SLOT_OWNER", "DUMP_LAST_USED", "DUMP_REQUEST_LIST", "DUMP_EVICTION_LOG")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_18001_amd import cinr
    cinr.lib()  # fails loudly if the library is missing


def _volume(w):
    from paper_2504_18001_amd import cinr
    t, wt = inr_params(w.arch, w.inr_seed)
    s, o = value_range(w.arch, w.inr_seed)
    base = cinr.Volume(w.arch, t, wt, s, o)
    mm = base.build_macrocells(w.macro_cell, "f32")
    return cinr.Volume(w.arch, base.table, base.weights, s, o, macrocells=mm, macro_cell=w.macro_cell)


def _cache(vol, w, pool=None):
    from paper_2504_18001_amd import cinr
    cs = w.cache
    return cinr.Cache(vol, cs.brick, cs.n_lods, pool or cs.pool_bricks, cs.max_requests, rank_window=cs.rank_window,
                      ranking=cs.ranking, preload_period=cs.preload_period, keep_request_counts=True)


def _same_state(a, b, tag):
    from paper_2504_18001_amd import cinr
    for k in DUMPS:
        da, db = a.dump(getattr(cinr, k)), b.dump(getattr(cinr, k))
        assert np.array_equal(np.asarray(da), np.asarray(db)), f"{tag}: {k} differs"


def _frames(w, sizes, mode, dtype, path=None, ert=0.999, pool=None):
    """Renders the same frame sequence through both entry points (each with
    its own cache) and compares every frame."""
    from paper_2504_18001_amd import cinr
    vol = _volume(w)
    ca = _cache(vol, w, pool) if mode == cinr.CACHED else None
    cb = _cache(vol, w, pool) if mode == cinr.CACHED else None
    ra, rb = cinr.Renderer(), cinr.Renderer()
    for f, (W, H) in enumerate(sizes):
        cam = w.camera(f)
        cam.width, cam.height = W, H
        tf = torch.as_tensor(w.tf(f)).cuda()
        sa = torch.zeros(len(cinr.STAT_FIELDS), dtype=torch.int64, device="cuda")
        sb = torch.zeros_like(sa)
        ob = torch.full((H, W, 4), -7.0, dtype=torch.float32, device="cuda")
        kw = dict(lod_scale=w.lod_scale, frame_index=f, seed=w.seed, ert_threshold=ert,
                  samples_per_iter=w.samples_per_iter, mode=mode, dtype=dtype, path=path, **SHAPE)
        print(f"[noalloc] frame {f} {W}x{H} mode {mode} dtype {dtype} path {path is not None}", flush=True)
        ia = ra.render(vol, cam, tf, w.step, cache=ca, stats=sa, **kw)
        ib = rb.render_noalloc(vol, cam, tf, w.step, cache=cb, stats=sb, out=ob, **kw)
        torch.cuda.synchronize()
        assert torch.equal(ia, ib), f"frame {f} ({W}x{H}): images differ, max abs {(ia - ib).abs().max().item()}"
        assert torch.equal(sa, sb), f"frame {f}: statistics differ {sa.tolist()} vs {sb.tolist()}"
        if ca is not None:
            _same_state(ca, cb, f"frame {f}")
    return sa.cpu().numpy()


def test_cached_frames_shrinking():
    """Cached ray-marched frames with early termination and true misses (the
    readback loop of later iterations), a 96-slot pool that evicts; the second
    and fourth frames are smaller than the ones before."""
    from paper_2504_18001_amd import cinr
    w = configs.SMALL
    st = _frames(w, [(128, 128), (72, 40), (128, 96), (33, 17), (128, 128)], cinr.CACHED, "f32")
    assert st[cinr.STAT_FIELDS.index("rays")] > 0


def test_cached_preload_frames_bf16():
    """The pre-load schedule (coarsest LoD forced, no early termination)
    through both calls, BF16 MLP, decreasing sizes."""
    from paper_2504_18001_amd import cinr
    w = configs.scaled(configs.SMALL, 128, 128, cache=configs.CacheShape(brick=8, n_lods=2, pool_bricks=96,
                                                                           max_requests=16, preload_period=2))
    _frames(w, [(128, 128), (100, 64), (64, 64), (48, 24)], cinr.CACHED, "bf16")


def test_uncached_frames_shrinking():
    from paper_2504_18001_amd import cinr
    w = configs.SMALL
    _frames(w, [(96, 96), (40, 24)], cinr.UNCACHED_DIRECT, "bf16x3")


def test_path_traced_frames_shrinking():
    from paper_2504_18001_amd import cinr
    w = configs.scaled(configs.SMALL, 64, 64, samples_per_iter=4)
    _frames(w, [(64, 64), (48, 32), (31, 9)], cinr.CACHED, "f32", path=PATH, ert=2.0)


def test_too_large_a_frame_is_rejected_before_any_launch():
    from paper_2504_18001_amd import cinr
    w = configs.SMALL
    vol = _volume(w)
    r = cinr.Renderer()
    cam = w.camera(0)
    cam.width, cam.height = 1920, 1080  # about 0.36 GB of workspace at 8 samples per iteration
    out = torch.zeros((1080, 1920, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(cinr.CinrError, match="fixed scratch array"):
        r.render_noalloc(vol, cam, w.tf(0), w.step, mode=cinr.UNCACHED_DIRECT, samples_per_iter=8, out=out, **SHAPE)
    assert float(out.abs().max()) == 0.0
