"""Oracle pins: the pre-load of Section 4.3.4 and the replay of early ray
termination.

Pre-load: the first `preload_period` frames force every sample to the
coarsest LoD and march every ray through the whole volume (early ray
termination suspended), so that the cache holds a low-resolution copy of
nearly the entire volume to fall back on:
- with an opaque TF and a camera that sees the whole box, every coarsest
  brick is resident once the pre-load has selected them (with early
  termination during the pre-load, the bricks behind the first opaque layer
  would never be requested);
- a pre-load frame with early termination requested renders and decides
  exactly as the same frame with early termination off;
- after the pre-load, early termination is active again;
- the 1080p orbit (at 1/64 of its pixels) has no true miss once the pre-load
  is over.

Replay: the renderer under test records where each ray ended early; the
oracle ending its rays exactly there reproduces its own frame when the record
is its own, and counts the ends its own opacity contradicts.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2504_18001_amd import configs, synth
from tests.helpers import oracle_inr


def _opaque_tf():
    tf = synth.tf_ramp()
    tf[:, 3] = 0.9  # every sample is nearly opaque: rays end within a few samples
    return tf


def _small_cache(m, period, max_requests=32, pool=400):
    return O.OracleCache(m, brick=8, n_lods=2, pool_bricks=pool, max_requests=max_requests, preload_period=period)


def _frame_params(f, ert):
    w = configs.SMALL
    return O.make_params(0.5, w.lod_scale, seed=5, frame_index=f, ert_threshold=ert, samples_per_iter=8)


def _camera(f, n=64):
    cam = configs.SMALL.camera(f)
    cam.width = cam.height = n
    return cam


def test_preload_frame_schedule():
    assert [O.lib().orc_preload_frame(f, 4) for f in range(8)] == [1] * 4 + [0] * 4
    assert O.lib().orc_preload_frame(0, 0) == 0 and O.lib().orc_preload_frame(3, 0) == 0


def test_preload_makes_every_coarsest_brick_resident():
    # 64^3, B = 8, 2 LoDs: LoD 1 has 5^3 = 125 bricks; 4 pre-load frames of 32
    # requests select 128 >= 125.  The orthographic view of side 64 sqrt 3
    # covers the whole box from every orbit angle.
    m = oracle_inr(configs.ARCH_SMALL, 0)
    _, _, off = O.lod_geometry(configs.ARCH_SMALL.dims, 8, 2)
    c = _small_cache(m, period=4)
    tf = _opaque_tf()
    for f in range(4):
        c.render(_camera(f), tf, _frame_params(f, 0.999))
    coarse = c.page_table()[int(off[1]):int(off[2])]
    assert (coarse >= 0).all(), f"{int((coarse < 0).sum())} coarsest bricks not resident after the pre-load"
    # samples forced to the coarsest LoD by distance instead (lod_scale 100)
    # with early termination: only the bricks of the front layers are requested
    c0 = _small_cache(m, period=0)
    for f in range(4):
        p = _frame_params(f, 0.999)
        p.lod_scale = 100.0
        c0.render(_camera(f), tf, p)
    pt0 = c0.page_table()
    assert (pt0[:int(off[1])] < 0).all() and (pt0[int(off[1]):] >= 0).sum() < 100


def test_preload_frames_decide_as_without_early_termination():
    m = oracle_inr(configs.ARCH_SMALL, 1)
    tf = _opaque_tf()
    a, b = _small_cache(m, period=3), _small_cache(m, period=3)
    for f in range(5):
        ia, sa = a.render(_camera(f, 40), tf, _frame_params(f, 0.999))
        ib, sb = b.render(_camera(f, 40), tf, _frame_params(f, 2.0))
        same = np.array_equal(ia, ib) and sa == sb and np.array_equal(a.page_table(), b.page_table()) and \
            np.array_equal(a.last_used(), b.last_used()) and np.array_equal(a.rank(), b.rank())
        if f < 3:
            assert same, f"pre-load frame {f} differs from the frame without early termination"
        else:
            # early termination is active again after the pre-load
            assert sa["samples"] < sb["samples"]


def test_orbit_has_no_true_miss_after_the_preload():
    # the 1080p workload at 240 x 135 (1/64 of the pixels), no macro-cells:
    # the coarsest LoD (125 bricks of LoD 3) is complete after the 4 pre-load
    # frames, so every later sample is served by a brick (hit or fallback)
    w = configs.HD512
    m = oracle_inr(w.arch, w.inr_seed)
    cs = w.cache
    c = O.OracleCache(m, brick=cs.brick, n_lods=cs.n_lods, pool_bricks=cs.pool_bricks, max_requests=cs.max_requests,
                      ranking=cs.ranking, preload_period=cs.preload_period)
    _, _, off = O.lod_geometry(w.arch.dims, cs.brick, cs.n_lods)
    misses = []
    for f in range(14):
        cam = w.camera(f)
        cam.width, cam.height = 240, 135
        p = O.make_params(w.step, w.lod_scale, seed=w.seed, frame_index=f, ert_threshold=w.ert_threshold,
                          samples_per_iter=w.samples_per_iter)
        _, st = c.render(cam, w.tf(f), p)
        misses.append(st["misses"])
        if f == 4:
            assert (c.page_table()[int(off[3]):] >= 0).all()
    assert misses[0] > 0 and misses[4:] == [0] * 10, misses


# ---------------------------------------------------------------------------
# Early-termination replay (performance mode)
# ---------------------------------------------------------------------------


def _replay_scene(seed=0):
    m = oracle_inr(configs.ARCH_SMALL, seed)
    tf = synth.tf_ramp()
    tf[:, 3] = np.linspace(0.0, 0.6, 256, dtype=np.float32)
    return m, tf


@pytest.mark.parametrize("prefill", [False, True])
def test_replay_of_own_terminations_reproduces_the_frame(prefill):
    m, tf = _replay_scene(2)
    cam = _camera(1, 48)
    caches = [_small_cache(m, period=0, max_requests=16, pool=96) for _ in range(2)]
    if prefill:
        for c in caches:
            c.prefill(np.arange(0, 854, 5).astype(np.int32)[:96], 0)
    p = _frame_params(1, 0.95)
    rec = O.record_ert(p, 48, 48)
    img_a, st_a = caches[0].render(cam, tf, p)
    assert (rec >= 0).sum() > 100 and st_a["ert_violations"] == 0
    q = _frame_params(1, 0.95)
    q2 = O.make_params(q.step, q.lod_scale, seed=5, frame_index=1, ert_threshold=0.95, samples_per_iter=8,
                       ert_replay=rec)
    img_b, st_b = caches[1].render(cam, tf, q2)
    assert st_a == st_b and st_b["ert_violations"] == 0
    np.testing.assert_array_equal(img_a, img_b)
    for get in ("page_table", "last_used", "rank", "req_count", "request_list"):
        np.testing.assert_array_equal(getattr(caches[0], get)(), getattr(caches[1], get)())


def test_replay_counts_unjustified_terminations():
    m, tf = _replay_scene(3)
    cam = _camera(2, 40)
    p = O.make_params(0.5, 1 / 96, ert_threshold=0.95, samples_per_iter=8, mode=O.UNCACHED_DIRECT)
    rec = O.record_ert(p, 40, 40)
    ref, st = O.render_uncached(m, cam, tf, p)
    ended = rec >= 0
    assert ended.sum() > 50 and st["ert_violations"] == 0
    # no replayed end: every ray the oracle would end counts once, and the
    # image is the one without early termination
    none = np.full_like(rec, -1)
    img, st0 = O.render_uncached(m, cam, tf, O.make_params(0.5, 1 / 96, ert_threshold=0.95, samples_per_iter=8,
                                                            mode=O.UNCACHED_DIRECT, ert_replay=none))
    full, _ = O.render_uncached(m, cam, tf, O.make_params(0.5, 1 / 96, ert_threshold=2.0, samples_per_iter=8,
                                                           mode=O.UNCACHED_DIRECT))
    np.testing.assert_array_equal(img, full)
    assert st0["ert_violations"] >= ended.sum()
    # ends moved one sample early are unjustified for rays whose opacity
    # crosses the threshold in a real step
    early = rec.copy()
    early[ended] -= 1
    _, st1 = O.render_uncached(m, cam, tf, O.make_params(0.5, 1 / 96, ert_threshold=0.95, samples_per_iter=8,
                                                          mode=O.UNCACHED_DIRECT, ert_replay=early))
    assert st1["ert_violations"] > 0.5 * ended.sum()
