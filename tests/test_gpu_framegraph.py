"""Captured multi-view frames (cinr_frame_graph_*) against eager frames
(cinr_render_views, bit for bit) and against the oracle: images, statistics
and every piece of cache state, over a sequence with a cold start (true
misses, so further iterations after the captured first marches), evictions
(the end graph with the LRU pass) and a TF that changes between frames."""
import numpy as np
import pytest
import torch

from paper_2504_18001_amd import configs
from tests.helpers import inr_params, oracle_inr, value_range
from tests.test_gpu_parity import TOL

pytestmark = pytest.mark.gpu

W = configs.SMALL
SIZES = [(48, 40), (32, 32), (64, 48), (40, 40), (24, 56)]
VOLS = [0, 1, 2, 0, 1]
STATE = ("DUMP_PAGE_TABLE", "DUMP_SLOT_OWNER", "DUMP_LAST_USED", "DUMP_RANK", "DUMP_REQ_COUNT", "DUMP_REQUEST_LIST",
         "DUMP_EVICTION_LOG")


def gpu_volume(seed):
    from paper_2504_18001_amd import cinr
    t, w = inr_params(W.arch, seed)
    s, o = value_range(W.arch, seed)
    return cinr.Volume(W.arch, t, w, s, o)


def view_cam(i, f):
    c = W.camera(f + 3 * i)
    c.width, c.height = SIZES[i]
    return c


def make_cache(vols, **kw):
    from paper_2504_18001_amd import cinr
    return cinr.Cache(vols, 8, 2, 150, 24, miss_log_capacity=1 << 20, evict_log_capacity=1 << 14,
                      keep_request_counts=True, **kw)


def miss_set(cache):
    from paper_2504_18001_amd import cinr
    pk, pos = cache.dump(cinr.DUMP_MISS_LIST)
    g = np.concatenate([pk, pos.view(np.int32)], axis=1)
    return g[np.lexsort(g.T[::-1])]


@pytest.mark.parametrize("n_views,mixed,dev_iters", [(5, False, 0), (1, False, 0), (5, True, 0), (5, False, 3),
                                                     (1, False, 3)])
def test_graph_frames_equal_eager_frames_and_oracle(n_views, mixed, dev_iters):
    """dev_iters: wavefront iterations after the first marches queued in the
    graph, so that frames of at most dev_iters + 1 iterations need no host
    round trip before their end."""
    from oracle import oracle as O
    from paper_2504_18001_amd import cinr
    vols = [gpu_volume(s) for s in range(3)]
    ms = [oracle_inr(W.arch, s) for s in range(3)]
    # mixed: LoD 1 in a binary16 class of 75 slots, LoD 0 in 75 binary32
    # slots, at a LoD scale that requests both LoDs
    pool_kw = dict(f16_lods=0b10, pool_bricks_f16=75) if mixed else {}
    ls = W.lod_scale * (0.3 if mixed else 1.0)
    ge, gg = make_cache(vols, **pool_kw), make_cache(vols, **pool_kw)
    oc = O.OracleCache(ms, brick=8, n_lods=2, pool_bricks=150, max_requests=24, log_misses=True, **pool_kw)
    idx = list(range(n_views))
    kw = dict(lod_scale=ls, seed=W.seed, samples_per_iter=W.samples_per_iter, pipe_depth=2, xcd_bands=4)
    mv = cinr.MultiViewRenderer(n_views)
    fg = cinr.FrameGraph(gg, [(vols[VOLS[i]], view_cam(i, 0), W.tf(0)) for i in idx], W.step, **kw)
    fg.set_device_iterations(dev_iters)
    iters = []  # most iterations of a view, per frame
    for f in range(12):
        print(f"frame {f}, {n_views} views", flush=True)
        eager = mv.render(ge, [(vols[VOLS[i]], view_cam(i, f), W.tf(f)) for i in idx], W.step, frame_index=f, **kw)
        for i in idx:
            fg.tfs[i].copy_(torch.as_tensor(np.asarray(W.tf(f), np.float32)))
        imgs = fg.render([view_cam(i, f) for i in idx], f)
        se, sg = mv.last_stats(), fg.last_stats()
        iters.append(max(sg[i]["iterations"] for i in idx))
        ps = [O.make_params(W.step, ls, seed=W.seed, frame_index=f, samples_per_iter=W.samples_per_iter)
              for _ in idx]
        ref = oc.render_views([(VOLS[i], view_cam(i, f), W.tf(f)) for i in idx], ps)
        for i in idx:
            a, b = eager[i].cpu().numpy(), imgs[i].cpu().numpy()
            np.testing.assert_array_equal(b, a, err_msg=f"frame {f} view {i}")
            assert sg[i] == se[i], (f, i, sg[i], se[i])
            rimg, rst = ref[i]
            for k in ("rays", "samples", "hits", "fallbacks", "misses", "skipped", "requested", "selected", "evicted"):
                assert sg[i][k] == rst[k], (f, i, k, sg[i][k], rst[k])
            assert np.abs(b.astype(np.float64) - rimg).max() <= TOL["f32"], (f, i)
        for name in STATE:
            kind = getattr(cinr, name)
            np.testing.assert_array_equal(gg.dump(kind), ge.dump(kind), err_msg=f"frame {f} {name}")
        np.testing.assert_array_equal(miss_set(gg), miss_set(ge))
        np.testing.assert_array_equal(gg.dump(cinr.DUMP_PAGE_TABLE), oc.page_table())
        np.testing.assert_array_equal(gg.dump(cinr.DUMP_LAST_USED), oc.last_used())
    n_graph, n_eager, n_tail = fg.counts()
    print("graph frames", n_graph, "eager", n_eager, "with further iterations", n_tail, "iterations", iters)
    assert n_graph == 12 and n_eager == 0
    # the cold start leaves true misses after the first marches; frames of more
    # iterations than the graph queues finish with host round trips
    assert max(iters) > 1
    assert n_tail == sum(1 for k in iters if k > 1 + dev_iters)
    ev = gg.dump(cinr.DUMP_EVICTION_LOG)
    assert (ev[:, 2] >= 0).any()  # bricks were evicted (LRU pass in the end graph)
    if mixed:  # in both classes
        assert ((ev[:, 2] >= 0) & (ev[:, 1] < 75)).any() and ((ev[:, 2] >= 0) & (ev[:, 1] >= 75)).any()


def test_graph_frames_wait_for_online_tuning():
    from paper_2504_18001_amd import cinr
    # separate volumes (same INRs): each path tunes its own launch shapes
    ve, vg = [gpu_volume(s) for s in range(3)], [gpu_volume(s) for s in range(3)]
    ge, gg = make_cache(ve), make_cache(vg)
    idx = list(range(3))
    kw = dict(lod_scale=W.lod_scale, seed=W.seed, samples_per_iter=W.samples_per_iter)
    mv = cinr.MultiViewRenderer(3)
    fg = cinr.FrameGraph(gg, [(vg[VOLS[i]], view_cam(i, 0), W.tf(0)) for i in idx], W.step, **kw)
    # 48 counted trials, plus up to 96 frames cut short by true misses and the
    # frames under a pre-load LoD floor, which are not counted
    n_frames = 160
    for f in range(n_frames):
        eager = mv.render(ge, [(ve[VOLS[i]], view_cam(i, f), W.tf(0)) for i in idx], W.step, frame_index=f, **kw)
        imgs = fg.render([view_cam(i, f) for i in idx], f)
        for i in idx:
            np.testing.assert_array_equal(imgs[i].cpu().numpy(), eager[i].cpu().numpy())
        np.testing.assert_array_equal(gg.dump(cinr.DUMP_LAST_USED), ge.dump(cinr.DUMP_LAST_USED))
    n_graph, n_eager, _ = fg.counts()
    print("graph frames", n_graph, "eager", n_eager)
    # the 24 candidate shapes x 2 rounds are tried eagerly, then frames replay
    assert all(cinr.tuned_launch(vg[VOLS[i]], *SIZES[i])[2] == 0 for i in idx)
    assert n_eager >= 48 and n_graph > 0 and n_graph + n_eager == n_frames


def test_graph_rejects_a_camera_of_another_size():
    from paper_2504_18001_amd import cinr
    vols = [gpu_volume(0)]
    cache = make_cache(vols)
    fg = cinr.FrameGraph(cache, [(vols[0], view_cam(0, 0), W.tf(0))], W.step, lod_scale=W.lod_scale, pipe_depth=2,
                         xcd_bands=4)
    cam = view_cam(0, 1)
    cam.width += 8
    with pytest.raises(cinr.CinrError, match="size and projection"):
        fg.render([cam], 1)
