"""GPU parity of the pre-load (Section 4.3.4) and of the performance mode
(early ray termination on), through the C ABI.

Pre-load: the frames that force the coarsest LoD march every ray to the end
of the box, early termination suspended, so that the coarsest bricks behind
opaque material are requested too; the cache then holds a low-resolution copy
of the whole visible volume to fall back on, and later frames have no true
miss.

Performance mode: the GPU records, per pixel, the sample-grid index just past
the sample whose compositing ended the ray (`ert_record`); the oracle replays
those ends instead of testing its own FP64 opacity.  Both then take every
sample of the frame in the same places, so all cache state (page table,
owners, stamps, ranks, request counts, request lists, miss lists, eviction
log) is compared bit for bit, the images within the value tolerance, and the
oracle counts the replayed ends its own opacity does not justify
(A < threshold - slack at an end, A >= threshold + slack before it): none may
occur.  The slack is 1e-4 for the FP32 MLP and the image tolerance (8e-3)
for reduced precision, whose values, and so opacities, may differ by that
much.
"""
import numpy as np
import pytest
import torch

from paper_2504_18001_amd import configs, synth
from tests.helpers import inr_params, oracle_inr, value_range
from tests.test_gpu_parity import TOL, _compare_state, gpu_volume

pytestmark = pytest.mark.gpu

ERT = 0.999


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_18001_amd import cinr
    cinr.lib()


def _performance_sequence(w, frames, width, height, dims=None, pool=None, max_req=None, preload=0, macro=False,
                          adapt=0, tf_fn=None, dtype="f32", ert=ERT):
    """A cached sequence with early termination on: each GPU frame records its
    terminations and the oracle replays them.  Returns the number of rays
    ended early per frame and the two caches."""
    from oracle import oracle as O
    from paper_2504_18001_amd import cinr
    cs = w.cache
    pool = pool if pool is not None else cs.pool_bricks
    max_req = max_req if max_req is not None else cs.max_requests
    m = oracle_inr(w.arch, 0, dims=dims)
    mm = m.macrocells(w.macro_cell) if macro else None
    vol = gpu_volume(w.arch, 0, dims=dims, macrocells=mm, macro_cell=w.macro_cell if macro else 0)
    gc = cinr.Cache(vol, cs.brick, cs.n_lods, pool, max_req, ranking=cs.ranking, preload_period=preload,
                    miss_log_capacity=1 << 22, evict_log_capacity=1 << 16, keep_request_counts=True)
    oc = O.OracleCache(m, brick=cs.brick, n_lods=cs.n_lods, pool_bricks=pool, max_requests=max_req,
                       ranking=cs.ranking, preload_period=preload, log_misses=True)
    r = cinr.Renderer()
    ended = []
    for f in frames:
        cam = w.camera(f, dims)
        cam.width, cam.height = width, height
        tf = tf_fn(f) if tf_fn else w.tf(f)
        rec = torch.full((height, width), -7, dtype=torch.int32, device="cuda")
        img = r.render(vol, cam, tf, w.step, w.lod_scale, frame_index=f, seed=w.seed, ert_threshold=ert,
                       samples_per_iter=w.samples_per_iter, mode=cinr.CACHED, dtype=dtype, cache=gc,
                       adapt_max_exp=adapt, ert_record=rec).cpu().numpy().astype(np.float64)
        st = r.last_stats()
        rec = rec.cpu().numpy()
        assert rec.min() >= -1, "every pixel is written"
        p = O.make_params(w.step, w.lod_scale, seed=w.seed, frame_index=f, ert_threshold=ert,
                          samples_per_iter=w.samples_per_iter, mode=O.CACHED, macro_cell=w.macro_cell if macro else 0,
                          macro_minmax=mm, adapt_max_exp=adapt if adapt > 0 else -1, ert_replay=rec,
                          ert_slack=1e-4 if dtype == "f32" else TOL[dtype])
        ref, rst = oc.render(cam, tf, p)
        err = np.abs(img - ref).max()
        n_end = int((rec >= 0).sum())
        print(f"frame {f}: ended early {n_end}, err {err:.2e}, gpu {st}, oracle {rst}", flush=True)
        assert rst["ert_violations"] == 0, (f, rst["ert_violations"])
        for k in ("rays", "samples", "hits", "fallbacks", "misses", "skipped", "requested", "selected", "evicted"):
            assert st[k] == rst[k], (f, k, st[k], rst[k])
        _compare_state(gc, oc, f)
        assert err <= TOL[dtype], (f, err)
        if preload and f < preload:
            assert n_end == 0, "pre-load frames march without early termination"
        ended.append(n_end)
    return ended, gc, oc


def test_performance_mode_small_replay():
    # 64^3, 128x128 orthographic, B = 8, 2 LoDs, 96 slots with eviction; a
    # TF of rising opacity so that many rays end early
    w = configs.SMALL

    def tf(f):
        t = synth.tf_ramp()
        t[:, 3] = np.minimum(1.0, np.linspace(0.0, 3.0, 256)).astype(np.float32)
        return t

    ended, _, _ = _performance_sequence(w, range(10), 128, 128, tf_fn=tf)
    assert min(ended) > 1000


def test_performance_mode_512_arch_with_preload():
    # the 512^3 architecture on a 120x104x96 virtual volume, 4 LoDs, B = 16,
    # pre-load of 2 frames per LoD, macro-cells from the INR: the two pre-load
    # frames record no early end, the frames after them do
    w = configs.scaled(configs.HD512, 96, 64, orbit_radius=260.0, lod_scale=1.0 / 180.0)
    ended, gc, oc = _performance_sequence(w, range(8), 96, 64, dims=(120, 104, 96), pool=300, max_req=12, preload=2,
                                          macro=True)
    assert ended[0] == ended[1] == 0 and max(ended[2:]) > 500


def test_performance_mode_adaptive_rate_bf16():
    # the adaptive sampling rate (ends recorded at k + 2^e) with the BF16 MLP
    w = configs.scaled(configs.HD512, 80, 48, orbit_radius=260.0, lod_scale=1.0 / 180.0)

    def tf(f):
        t = synth.tf_ramp()
        t[:, 3] = np.linspace(0.0, 0.35, 256).astype(np.float32)
        return t

    ended, _, _ = _performance_sequence(w, range(5), 80, 48, dims=(120, 104, 96), pool=300, max_req=12, preload=1,
                                        macro=True, adapt=2, tf_fn=tf, dtype="bf16", ert=0.95)
    assert max(ended[1:]) > 200


def test_ert_record_argument_checks():
    from paper_2504_18001_amd import cinr
    w = configs.SMALL
    vol = gpu_volume(w.arch, 0)
    cam = w.camera(0)
    cam.width, cam.height = 16, 8
    r = cinr.Renderer()
    with pytest.raises(ValueError):
        r.render(vol, cam, w.tf(0), w.step, ert_threshold=ERT, mode=cinr.UNCACHED_DIRECT,
                 ert_record=torch.zeros((16, 8), dtype=torch.int32, device="cuda"))
    with pytest.raises(cinr.CinrError):  # a ray-marching output only
        r.render(vol, cam, w.tf(0), w.step, mode=cinr.UNCACHED_DIRECT, path={"density": 0.1},
                 ert_record=torch.zeros((8, 16), dtype=torch.int32, device="cuda"))


def test_uncached_record_matches_oracle_own_ends():
    # the uncached renderer's ends against the oracle's own FP64 test: they
    # agree except where the FP32 and FP64 opacities straddle the threshold
    from oracle import oracle as O
    from paper_2504_18001_amd import cinr
    w = configs.SMALL
    vol = gpu_volume(w.arch, 0)
    m = oracle_inr(w.arch, 0)
    cam = w.camera(1)
    cam.width, cam.height = 96, 96
    tf = synth.tf_ramp()
    tf[:, 3] = np.minimum(1.0, np.linspace(0.0, 2.0, 256)).astype(np.float32)
    rec = torch.full((96, 96), -7, dtype=torch.int32, device="cuda")
    r = cinr.Renderer()
    r.render(vol, cam, tf, w.step, w.lod_scale, ert_threshold=0.99, samples_per_iter=w.samples_per_iter,
             mode=cinr.UNCACHED_DIRECT, dtype="f32", ert_record=rec)
    g = rec.cpu().numpy()
    p = O.make_params(w.step, w.lod_scale, ert_threshold=0.99, samples_per_iter=w.samples_per_iter,
                      mode=O.UNCACHED_DIRECT)
    own = O.record_ert(p, 96, 96)
    O.render_uncached(m, cam, tf, p)
    agree = float((g == own).mean())
    print("ended early:", int((g >= 0).sum()), "agreement with the oracle's own ends:", agree)
    assert (g >= 0).sum() > 2000 and agree >= 0.999


# ---------------------------------------------------------------------------
# Full size: the bench configuration with the INR's own macro-cells
# ---------------------------------------------------------------------------

W = configs.HD512


@pytest.fixture(scope="module")
def own_scene():
    """The bench's volume: macro-cells of side 16 built from the INR on the
    GPU (the table both sides read), spot-checked against the oracle's lattice
    values on 12 cells."""
    from oracle import oracle as O
    from paper_2504_18001_amd import cinr
    t, wts = inr_params(W.arch, 0)
    s, o = value_range(W.arch, 0)
    base = cinr.Volume(W.arch, t, wts, s, o)
    mm = base.build_macrocells(W.macro_cell, "f32").cpu().numpy()
    vol = cinr.Volume(W.arch, t, wts, s, o, macrocells=mm, macro_cell=W.macro_cell)
    m = O.OracleInr(W.arch, t, wts, s, o)
    N, V = W.macro_cell, np.asarray(W.arch.dims)
    M = (V + N - 1) // N
    rng = np.random.default_rng(21)
    cells = [rng.integers(0, M) for _ in range(10)] + [M - 1, np.zeros(3, int)]
    for c in cells:
        ax = [np.arange(c[a] * N, min((c[a] + 1) * N, V[a] - 1) + 1) for a in range(3)]
        zz, yy, xx = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1).astype(np.float64)
        v = m.value(pts)
        got = mm[c[2], c[1], c[0]]
        assert abs(got[0] - v.min()) <= 1e-4 and abs(got[1] - v.max()) <= 1e-4, (c, got, v.min(), v.max())
    return vol, m, mm


def test_fullsize_preload_leaves_the_coarsest_lod_complete(own_scene):
    # the bench's command in miniature: frames 0-11 of the orbit with early
    # termination on.  The 4 pre-load frames record no early end and select
    # every LoD-3 brick (125 <= 4 x 40); from frame 4 on every LoD-3 brick
    # is mapped, so no sample can be a true miss.
    from paper_2504_18001_amd import cinr
    vol, m, mm = own_scene
    cs = W.cache
    cache = cinr.Cache(vol, cs.brick, cs.n_lods, cs.pool_bricks, cs.max_requests, preload_period=cs.preload_period)
    off = vol.geometry(cs.brick, cs.n_lods)[1]
    r = cinr.Renderer()
    rec = torch.empty((W.height, W.width), dtype=torch.int32, device="cuda")
    misses = []
    for f in range(12):
        r.render(vol, W.camera(f), W.tf(f), W.step, W.lod_scale, frame_index=f, seed=W.seed, ert_threshold=ERT,
                 samples_per_iter=W.samples_per_iter, mode=cinr.CACHED, dtype="bf16x3", cache=cache, ert_record=rec)
        st = r.last_stats()
        misses.append(st["misses"])
        n_end = int((rec >= 0).sum().item())
        print(f"frame {f}: {st}, ended early {n_end}", flush=True)
        if f < cs.preload_period:
            assert n_end == 0
        else:
            assert n_end > 10000
        if f == cs.preload_period:
            pt = cache.dump(cinr.DUMP_PAGE_TABLE)
            assert (pt[int(off[3]):int(off[4])] >= 0).all(), "every coarsest brick resident after the pre-load"
    assert misses[0] > 0 and misses[cs.preload_period:] == [0] * (12 - cs.preload_period), misses


def test_fullsize_performance_mode_replay_bit_exact(own_scene):
    # a prefilled residency at frame 12 of the orbit, the bench's launch
    # (split-BF16 decoding is not involved: the prefill decodes in FP32),
    # early termination at 0.999 recorded on the GPU and replayed by a full
    # oracle frame: request counts, request list, page table and stamps
    # bit-exact; sampled pixels within the FP32 bound
    from oracle import oracle as O
    from paper_2504_18001_amd import cinr
    vol, m, mm = own_scene
    cs = W.cache
    off = vol.geometry(cs.brick, cs.n_lods)[1]
    rng = np.random.default_rng(5)
    keys = [np.arange(off[3], off[4])]
    for L, frac in ((2, 0.3), (1, 0.03), (0, 0.003)):
        n = off[L + 1] - off[L]
        keys.append(off[L] + rng.choice(n, size=int(frac * n), replace=False))
    keys = np.sort(np.concatenate(keys)).astype(np.int32)
    cache = cinr.Cache(vol, cs.brick, cs.n_lods, cs.pool_bricks, cs.max_requests, preload_period=cs.preload_period,
                       keep_request_counts=True, evict_log_capacity=64)
    cache.prefill(torch.from_numpy(keys).cuda(), stamp=0, dtype="f32")
    oc = O.OracleCache(m, brick=cs.brick, n_lods=cs.n_lods, pool_bricks=cs.pool_bricks,
                       max_requests=cs.max_requests, preload_period=cs.preload_period)
    oc.prefill(keys, 0)
    f = 12
    cam, tf = W.camera(f), W.tf(f)
    rec = torch.empty((W.height, W.width), dtype=torch.int32, device="cuda")
    r = cinr.Renderer()
    img = r.render(vol, cam, tf, W.step, W.lod_scale, frame_index=f, seed=W.seed, ert_threshold=ERT,
                   samples_per_iter=W.samples_per_iter, mode=cinr.CACHED, dtype="f32", cache=cache, ert_record=rec)
    st = r.last_stats()
    g = rec.cpu().numpy()
    p = O.make_params(W.step, W.lod_scale, seed=W.seed, frame_index=f, ert_threshold=ERT,
                      samples_per_iter=W.samples_per_iter, mode=O.CACHED, macro_cell=W.macro_cell, macro_minmax=mm,
                      ert_replay=g)
    px = np.random.default_rng(6).choice(W.width * W.height, size=3000, replace=False).astype(np.int32)
    ref = O.render_pixels(m, cam, tf, p, px, cache=oc)
    got = img.reshape(-1, 4)[torch.from_numpy(px).long().cuda()].cpu().numpy().astype(np.float64)
    err = np.abs(got - ref).max()
    _, ost = oc.render(cam, tf, p)
    print(f"ended early {(g >= 0).sum()}, skipped {st['skipped']}, pixels max abs {err:.2e}; gpu {st}; oracle {ost}")
    assert ost["ert_violations"] == 0
    # the bench's TFs give every cell a positive opacity somewhere in its
    # range, so its frames skip no sample; the skip counts are compared below
    # all the same (the test with a windowed TF follows)
    assert (g >= 0).sum() > 10000
    for k in ("rays", "samples", "hits", "fallbacks", "misses", "skipped", "requested", "selected"):
        assert st[k] == ost[k], (k, st[k], ost[k])
    np.testing.assert_array_equal(cache.dump(cinr.DUMP_REQ_COUNT), oc.req_count())
    np.testing.assert_array_equal(cache.dump(cinr.DUMP_REQUEST_LIST), oc.request_list())
    np.testing.assert_array_equal(cache.dump(cinr.DUMP_PAGE_TABLE), oc.page_table())
    np.testing.assert_array_equal(cache.dump(cinr.DUMP_LAST_USED), oc.last_used())
    assert err <= 2e-3
    # the next frame with a TF transparent below row 200: cells whose value
    # range stays under it are skipped, and the skip decisions of the INR's
    # own macro-cells are compared with the oracle's, with every request and
    # stamp they change
    f = 13
    cam, tf = W.camera(f), synth.tf_window(200, 255)
    img = r.render(vol, cam, tf, W.step, W.lod_scale, frame_index=f, seed=W.seed, ert_threshold=ERT,
                   samples_per_iter=W.samples_per_iter, mode=cinr.CACHED, dtype="f32", cache=cache, ert_record=rec)
    st = r.last_stats()
    g = rec.cpu().numpy()
    p = O.make_params(W.step, W.lod_scale, seed=W.seed, frame_index=f, ert_threshold=ERT,
                      samples_per_iter=W.samples_per_iter, mode=O.CACHED, macro_cell=W.macro_cell, macro_minmax=mm,
                      ert_replay=g)
    _, ost = oc.render(cam, tf, p)
    print(f"windowed TF: skipped {st['skipped']}; gpu {st}; oracle {ost}")
    assert ost["ert_violations"] == 0
    for k in ("rays", "samples", "hits", "fallbacks", "misses", "skipped", "requested", "selected"):
        assert st[k] == ost[k], (k, st[k], ost[k])
    np.testing.assert_array_equal(cache.dump(cinr.DUMP_REQ_COUNT), oc.req_count())
    np.testing.assert_array_equal(cache.dump(cinr.DUMP_PAGE_TABLE), oc.page_table())
    np.testing.assert_array_equal(cache.dump(cinr.DUMP_LAST_USED), oc.last_used())
