"""Frames of several views through one cache shared by several INRs
(cinr_render_views) against the oracle, and the online launch tuner."""
import numpy as np
import pytest
import torch

from paper_2504_18001_amd import configs, synth
from tests.helpers import inr_params, oracle_inr, value_range
from tests.test_gpu_parity import TOL

pytestmark = pytest.mark.gpu

W = configs.SMALL
SIZES = [(48, 40), (32, 32), (64, 48), (40, 40)]
VOLS = [0, 1, 2, 0]


def gpu_volume(seed):
    from paper_2504_18001_amd import cinr
    t, w = inr_params(W.arch, seed)
    s, o = value_range(W.arch, seed)
    return cinr.Volume(W.arch, t, w, s, o)


def view_cam(i, f):
    c = W.camera(f + 3 * i)  # every view on its own point of the orbit
    c.width, c.height = SIZES[i]
    return c


@pytest.mark.parametrize("pool_dtype,staged", [("f32", False), ("f16", False), ("mixed", False), ("f32", True)])
def test_shared_cache_views_match_oracle(pool_dtype, staged):
    """staged: the shared cache decodes its bricks of the 3 INRs with
    LDS-staged corner boxes (4 parts per brick, 32 KiB)."""
    from oracle import oracle as O
    from paper_2504_18001_amd import cinr
    vols = [gpu_volume(s) for s in range(3)]
    if staged:
        vols[0].set_decode_shape(4, 32)
    ms = [oracle_inr(W.arch, s) for s in range(3)]
    B, nl, pool, req = 8, 2, 150, 24
    # mixed: LoD 1 in a binary16 class of 75 slots, LoD 0 in 75 binary32 slots,
    # at a LoD scale that requests both LoDs (both classes evict)
    mixed = dict(f16_lods=0b10, pool_bricks_f16=75) if pool_dtype == "mixed" else {}
    ls = W.lod_scale * (0.3 if mixed else 1.0)
    gc = cinr.Cache(vols, B, nl, pool, req, miss_log_capacity=1 << 20, evict_log_capacity=1 << 14,
                    keep_request_counts=True, pool_dtype="f16" if pool_dtype == "f16" else "f32", **mixed)
    oc = O.OracleCache(ms, brick=B, n_lods=nl, pool_bricks=pool, max_requests=req, log_misses=True,
                       pool_f16=pool_dtype == "f16", **mixed)
    assert gc.n_keys == oc.n_keys == 3 * gc.keys_per_volume
    mv = cinr.MultiViewRenderer(len(SIZES))
    for f in range(10):
        views = [(vols[VOLS[i]], view_cam(i, f), W.tf(f)) for i in range(len(SIZES))]
        imgs = mv.render(gc, views, W.step, ls, frame_index=f, seed=W.seed, samples_per_iter=W.samples_per_iter)
        gst = mv.last_stats()
        ps = [O.make_params(W.step, ls, seed=W.seed, frame_index=f, samples_per_iter=W.samples_per_iter)
              for _ in SIZES]
        ref = oc.render_views([(VOLS[i], view_cam(i, f), W.tf(f)) for i in range(len(SIZES))], ps)
        for i, ((rimg, rst), img) in enumerate(zip(ref, imgs)):
            err = np.abs(img.cpu().numpy().astype(np.float64) - rimg).max()
            for k in ("rays", "samples", "hits", "fallbacks", "misses", "skipped", "requested", "selected", "evicted"):
                assert gst[i][k] == rst[k], (f, i, k, gst[i][k], rst[k])
            assert err <= TOL["f32"], (f, i, err)
        for kind, ref_state in ((cinr.DUMP_PAGE_TABLE, oc.page_table()), (cinr.DUMP_SLOT_OWNER, oc.owner()),
                                (cinr.DUMP_LAST_USED, oc.last_used()), (cinr.DUMP_RANK, oc.rank()),
                                (cinr.DUMP_REQ_COUNT, oc.req_count()), (cinr.DUMP_REQUEST_LIST, oc.request_list()),
                                (cinr.DUMP_EVICTION_LOG, oc.evict_log())):
            np.testing.assert_array_equal(gc.dump(kind), ref_state, err_msg=f"frame {f} dump {kind}")
        # misses of all views: the same multiset of (pixel, k, position)
        gpk, gpos = gc.dump(cinr.DUMP_MISS_LIST)
        opk, opos = oc.miss_list()
        g = np.concatenate([gpk, gpos.view(np.int32)], axis=1)
        o = np.concatenate([opk, opos.view(np.int32)], axis=1)
        np.testing.assert_array_equal(g[np.lexsort(g.T[::-1])], o[np.lexsort(o.T[::-1])])
        print(f"frame {f}: stats {gst[0]}", flush=True)


def test_online_launch_tuning_converges_and_changes_nothing():
    from paper_2504_18001_amd import cinr
    w = configs.scaled(configs.HD512, 160, 96, orbit_radius=300.0, lod_scale=1.0 / 200.0)
    dims = (128, 112, 96)
    imgs = {}
    for mode in ("tuned", "fixed"):
        t, wt = inr_params(w.arch, 0)
        s, o = value_range(w.arch, 0)
        vol = cinr.Volume(w.arch, t, wt, s, o, dims=dims)
        cache = cinr.Cache(vol, 16, 4, 400, 20, preload_period=2)
        r = cinr.Renderer()
        out = []
        # 48 trials, plus up to 96 frames cut short by true misses and the
        # frames under a pre-load LoD floor, which are not counted
        for f in range(160):
            kw = dict(pipe_depth=0, xcd_bands=0) if mode == "tuned" else dict(pipe_depth=2, xcd_bands=4)
            img = r.render(vol, w.camera(f, dims), w.tf(f), w.step, w.lod_scale, frame_index=f, seed=w.seed,
                           ert_threshold=w.ert_threshold, samples_per_iter=w.samples_per_iter, mode=cinr.CACHED,
                           dtype="f32", cache=cache, **kw)
            out.append(img.cpu().numpy())
        imgs[mode] = out
        if mode == "tuned":
            p, b, left, waves = cinr.tuned_launch(vol, 160, 96)
            print("tuned launch", p, b, waves, left)
            assert left == 0 and p in (1, 2) and b in (1, 4, 16) and waves in (3, 4)
    for a, b in zip(imgs["tuned"], imgs["fixed"]):
        np.testing.assert_array_equal(a, b)
