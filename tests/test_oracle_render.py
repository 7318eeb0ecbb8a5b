"""Oracle pins: ray setup, compositing, stochastic LoD, the sampler with
fallback, and the invariants of the cached renderer.

- hand-computed ray/box results (axis-aligned, grazing, missing rays);
- closed-form compositing of a constant field; alpha = 0 is the identity;
- I1: an empty cache without pre-load renders exactly the uncached INR image;
- I2: a fully resident single-LoD cache renders exactly the uncached lattice
  (trilinear of LoD-0 values) image;
- brute force on tiny volumes: an independent per-sample Python march with
  residency by set membership reproduces image, request counts and stamps;
- stochastic LoD: values in {floor D, floor D + 1} with mean D, continuous
  across integers (Section 5.3);
- macro-cell skipping is exact in lattice mode (Section 5.2).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2504_18001_amd import configs, synth
from tests.helpers import constant_inr, coordinate_inr, oracle_inr


def _ortho_z(dims, W=4, H=4, extent=None, eye_z=100.0):
    c = [(d - 1) / 2.0 for d in dims]
    e = extent if extent is not None else float(dims[0])
    cam = synth.Camera(projection=synth.ORTHOGRAPHIC, eye=np.array([c[0], c[1], eye_z], np.float32),
                       forward=np.array([0, 0, -1], np.float32), right=np.array([1, 0, 0], np.float32),
                       up=np.array([0, 1, 0], np.float32), width=W, height=H, ortho_w=e, ortho_h=e)
    return cam


# ---------------------------------------------------------------------------
# Ray setup
# ---------------------------------------------------------------------------


def test_axis_aligned_ray_hand_result():
    # Orthographic camera looking down -z from z = 100 onto a 16^3 box: the
    # box spans t in [100 - 15, 100].
    cam = _ortho_z((16, 16, 16), W=4, H=4, extent=8.0)
    ok, o, d, ts, te = O.ray_setup(cam, (16, 16, 16), 1, 2)
    assert ok
    # pixel (1,2): x = 7.5 + ((1.5/4) - 0.5) * 8 = 6.5 ; y = 7.5 + (0.5 - 2.5/4) * 8 = 6.5
    assert o.tolist() == [6.5, 6.5, 100.0]
    assert d.tolist() == [0.0, 0.0, -1.0]
    assert (ts, te) == (85.0, 100.0)


def test_rays_missing_and_grazing_the_box():
    cam = _ortho_z((16, 16, 16), W=4, H=4, extent=64.0)
    ok, *_ = O.ray_setup(cam, (16, 16, 16), 0, 0)  # x = 7.5 - 24 < 0
    assert not ok
    # a ray exactly on the x = 0 face is inside (closed box)
    cam2 = _ortho_z((16, 16, 16), W=1, H=1, extent=1.0)
    cam2.eye = np.array([0.0, 3.0, 50.0], np.float32)
    ok, o, d, ts, te = O.ray_setup(cam2, (16, 16, 16), 0, 0)
    assert ok and o[0] == 0.0 and (ts, te) == (35.0, 50.0)
    cam2.eye = np.array([-1e-6, 3.0, 50.0], np.float32)
    ok, *_ = O.ray_setup(cam2, (16, 16, 16), 0, 0)
    assert not ok


def test_perspective_ray_through_box_corner():
    # eye at (-1,-1,-1) looking at the origin corner: the centre ray enters at
    # the corner (t = sqrt 3) and leaves at the far corner (t = 16 sqrt 3).
    cam = synth.look_at(synth.PERSPECTIVE, (-1.0, -1.0, -1.0), (0.0, 0.0, 0.0), 1, 1, fov_y_deg=10.0)
    ok, o, d, ts, te = O.ray_setup(cam, (16, 16, 16), 0, 0)
    assert ok
    assert ts == pytest.approx(math.sqrt(3.0), rel=1e-6)
    assert te == pytest.approx(16.0 * math.sqrt(3.0), rel=1e-6)


def test_eye_inside_box_starts_at_zero():
    cam = synth.look_at(synth.PERSPECTIVE, (8.0, 8.0, 8.0), (8.0, 8.0, 0.0), 2, 2)
    ok, o, d, ts, te = O.ray_setup(cam, (16, 16, 16), 0, 0)
    assert ok and ts == 0.0 and te > 0.0


# ---------------------------------------------------------------------------
# Compositing
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("mode", [O.UNCACHED_DIRECT, O.CACHED])
def test_constant_field_closed_form(mode):
    # v = 0.5 everywhere; a constant TF of 0.5 gives rgba = 0.5; a' = 1 - 0.5^0.5 per
    # half-voxel step; the axis-aligned rays see (15 / 0.5) + 1 = 31 samples:
    # A = 1 - (1 - a')^31, C = 0.5 A.
    dims = (16, 16, 16)
    m = constant_inr(dims, 0.5)
    cam = _ortho_z(dims, W=4, H=4, extent=8.0)
    p = O.make_params(0.5, 0.1, ert_threshold=2.0, samples_per_iter=4, mode=mode)
    tf = np.full((256, 4), 0.5, np.float32)
    if mode == O.CACHED:
        c = O.OracleCache(m, brick=4, n_lods=2, pool_bricks=0, max_requests=0)
        img, st = c.render(cam, tf, p)
    else:
        img, st = O.render_uncached(m, cam, tf, p)
    a1 = 1.0 - 0.5 ** 0.5
    A = 1.0 - (1.0 - a1) ** 31
    np.testing.assert_allclose(img[..., 3], A, rtol=0, atol=1e-14)
    np.testing.assert_allclose(img[..., :3], 0.5 * A, rtol=0, atol=1e-14)
    assert st["samples"] == 16 * 31 and st["misses"] == 16 * 31


def test_zero_opacity_is_identity():
    m = oracle_inr(configs.ARCH_SMALL, 0)
    tf = synth.tf_ramp()
    tf[:, 3] = 0.0
    cam = configs.SMALL.camera(0)
    cam.width = cam.height = 16
    img, _ = O.render_uncached(m, cam, tf, O.make_params(0.5, 1 / 96, mode=O.UNCACHED_DIRECT))
    assert np.all(img == 0.0)


def test_early_termination_stops_at_threshold():
    dims = (16, 16, 16)
    m = constant_inr(dims, 0.5)
    cam = _ortho_z(dims, W=2, H=2, extent=4.0)
    p = O.make_params(0.5, 0.1, ert_threshold=0.99, samples_per_iter=4, mode=O.UNCACHED_DIRECT)
    img, st = O.render_uncached(m, cam, np.full((256, 4), 0.8, np.float32), p)
    a1 = 1.0 - (1.0 - 0.8) ** 0.5
    n = math.ceil(math.log(0.01) / math.log(1 - a1))  # first n with A_n >= 0.99
    np.testing.assert_allclose(img[..., 3], 1 - (1 - a1) ** n, atol=1e-14)
    # the first sample is a true miss, so a wavefront step of 4 samples is gathered
    assert st["samples"] == 4 * 4 * math.ceil(n / 4)


# ---------------------------------------------------------------------------
# Invariants I1 and I2
# ---------------------------------------------------------------------------


def test_I1_empty_cache_equals_uncached_inr():
    m = oracle_inr(configs.ARCH_SMALL, 0)
    w = configs.SMALL
    cam = w.camera(1)
    cam.width = cam.height = 24
    cam.ortho_w = cam.ortho_h = np.float32(64 * math.sqrt(3))
    p = O.make_params(0.5, w.lod_scale, seed=7, frame_index=0, samples_per_iter=8, mode=O.CACHED)
    c = O.OracleCache(m, brick=8, n_lods=2, pool_bricks=96, max_requests=16)
    img_c, st = c.render(cam, synth.tf_ramp(), p)
    p.mode = O.UNCACHED_DIRECT
    img_u, st_u = O.render_uncached(m, cam, synth.tf_ramp(), p)
    np.testing.assert_array_equal(img_c, img_u)
    assert st["misses"] == st["samples"] > 0 and st["hits"] == st["fallbacks"] == 0


def test_I2_full_single_lod_cache_equals_lattice_image():
    dims = (24, 20, 18)
    m = oracle_inr(configs.ARCH_SMALL, 3, dims=dims)
    cam = synth.orbit_camera(synth.PERSPECTIVE, dims, 60.0, 30.0, 15.0, 20, 16, fov_y_deg=40.0)
    _, _, off = O.lod_geometry(dims, 5, 1)
    n = int(off[-1])
    c = O.OracleCache(m, brick=5, n_lods=1, pool_bricks=n, max_requests=n)
    p = O.make_params(0.5, 0.01, seed=1, frame_index=0, samples_per_iter=4, mode=O.CACHED)
    c.render(cam, synth.tf_ramp(), p)
    p.frame_index = 1
    img, st = c.render(cam, synth.tf_ramp(), p)
    assert st["hits"] == st["samples"] and st["misses"] == 0
    p.mode = O.UNCACHED_LATTICE
    ref, _ = O.render_uncached(m, cam, synth.tf_ramp(), p)
    np.testing.assert_array_equal(img, ref)


# ---------------------------------------------------------------------------
# Brute force on tiny volumes
# ---------------------------------------------------------------------------


def _bf_decide(m, V, K, nb, off, B, n_lods, resident, o, d, t, eye, lod_scale, fseed, lod_floor):
    """One sample of the independent march: (value, status, requested key,
    serving slot).  Residency by set membership; a served sample is the
    trilinear interpolation of the INR's LoD-L* lattice values; a true miss
    is the INR at the sample."""
    f32 = np.float32
    p = np.array([min(max(f32(o[a] + f32(t * d[a])), f32(0)), f32(V[a] - 1)) for a in range(3)], f32)
    L = O.select_lod(p, eye, lod_scale, fseed, lod_floor, n_lods)
    for Lp in range(L, n_lods):
        q = p * f32(2.0 ** -Lp)
        jj = np.minimum(q.astype(np.int64), K[Lp] - 2)
        b = jj // (B - 1)
        key = int(off[Lp] + (b[2] * nb[Lp][1] + b[1]) * nb[Lp][0] + b[0])
        if Lp == L:
            rkey = key
        if key in resident:
            fr = (q - jj.astype(f32)).astype(np.float64)
            corners = []
            for n in range(8):
                dlt = np.array([n & 1, (n >> 1) & 1, (n >> 2) & 1])
                x = np.minimum((jj + dlt) << Lp, V - 1).astype(np.float64)
                corners.append(m.value(x[None])[0])
            c = np.array(corners).reshape(2, 2, 2)  # [z][y][x]
            cx = c[..., 0] * (1 - fr[0]) + c[..., 1] * fr[0]
            cy = cx[:, 0] * (1 - fr[1]) + cx[:, 1] * fr[1]
            return cy[0] * (1 - fr[2]) + cy[1] * fr[2], ("hit" if Lp == L else "fb"), rkey, resident[key]
    return m.value(p.astype(np.float64)[None])[0], "miss", rkey, None


def _bf_composite(C, A, val, tf, step):
    x = val * 255.0
    i0 = min(int(math.floor(x)), 254)
    tt = x - i0
    rgba = tf[i0].astype(np.float64) * (1 - tt) + tf[i0 + 1].astype(np.float64) * tt
    a1 = 1.0 - (1.0 - rgba[3]) ** float(step)
    wgt = (1.0 - A) * a1
    return C + wgt * rgba[:3], A + wgt


def _brute_force_frame(m, dims, B, n_lods, resident, cam, tf, step, lod_scale, seed, frame, lod_floor,
                       ert=2.0, S=1):
    """Independent march of a frame.  Without early termination (ert > 1)
    every sample is decided and composited in order.  With it, the wavefront
    schedule: samples one at a time until the first true miss, then a step of
    S samples from the miss on (all decided: requests and stamps) composited
    in order; a ray ends at the first composited sample with A >= ert."""
    f32 = np.float32
    V = np.asarray(dims)
    K = [((V - 1) + (1 << L) - 1) // (1 << L) + 1 for L in range(n_lods)]
    nb = [(k - 1 + (B - 2)) // (B - 1) for k in K]
    off = np.concatenate([[0], np.cumsum([int(np.prod(x)) for x in nb])])
    fseed = O.lib().orc_frame_seed(seed, frame)
    img = np.zeros((cam.height, cam.width, 4))
    req = {}
    stamps = {}
    counts = dict(hit=0, fb=0, miss=0)

    def decide(o, d, t):
        val, stt, rkey, slot = _bf_decide(m, V, K, nb, off, B, n_lods, resident, o, d, t, cam.eye, lod_scale,
                                          fseed, lod_floor)
        counts[stt] += 1
        if slot is not None:
            stamps[slot] = frame
        if stt != "hit":
            req[rkey] = req.get(rkey, 0) + 1
        return val, stt

    for j in range(cam.height):
        for i in range(cam.width):
            ok, o, d, ts, te = O.ray_setup(cam, dims, i, j)
            if not ok:
                continue
            ts_list = []
            while True:
                t = f32(f32(ts) + f32(f32(len(ts_list)) * f32(step)))
                if t > f32(te):
                    break
                ts_list.append(t)
            nk = len(ts_list)
            C, A = np.zeros(3), 0.0
            k, done = 0, False
            while not done and k < nk:
                stt = None
                while k < nk:
                    val, stt = decide(o, d, ts_list[k])
                    if stt == "miss" and ert <= 1.0:
                        break
                    C, A = _bf_composite(C, A, val, tf, step)
                    k += 1
                    if A >= ert:
                        done = True
                        break
                if done or k >= nk:
                    break
                batch = [val] + [decide(o, d, ts_list[q])[0] for q in range(k + 1, min(k + S, nk))]
                for v in batch:
                    C, A = _bf_composite(C, A, v, tf, step)
                    if A >= ert:
                        done = True
                        break
                k += len(batch)
            img[j, i, :3] = C
            img[j, i, 3] = A
    return img, req, stamps, counts


@pytest.mark.parametrize("seed,frac", [(0, 0.3), (1, 0.7), (2, 0.0)])
def test_brute_force_tiny_volume(seed, frac):
    dims = (9, 10, 11)
    B, n_lods = 3, 3
    m = oracle_inr(configs.ARCH_SMALL, seed, dims=dims)
    _, nb, off = O.lod_geometry(dims, B, n_lods)
    n_keys = int(off[-1])
    rng = np.random.default_rng(seed)
    keys = np.sort(rng.choice(n_keys, size=int(n_keys * frac), replace=False)).astype(np.int32)
    cache = O.OracleCache(m, brick=B, n_lods=n_lods, pool_bricks=n_keys, max_requests=0)
    if keys.size:
        cache.prefill(keys, stamp=0)
    pt = cache.page_table()
    resident = {int(k): int(pt[k]) for k in keys}
    cam = synth.orbit_camera(synth.PERSPECTIVE, dims, 18.0, 20.0 + 40 * seed, 25.0, 7, 6, fov_y_deg=50.0)
    tf = synth.tf_random(seed)
    lod_scale = 0.12
    p = O.make_params(0.5, lod_scale, seed=11, frame_index=3, samples_per_iter=5, mode=O.CACHED)
    img, st = cache.render(cam, tf, p)
    ref, req, stamps, counts = _brute_force_frame(m, dims, B, n_lods, resident, cam, tf, 0.5, lod_scale, 11, 3, 0)
    np.testing.assert_allclose(img, ref, rtol=0, atol=1e-12)
    rc = cache.req_count()
    expect = np.zeros(n_keys, np.uint32)
    for k, v in req.items():
        expect[k] = v
    np.testing.assert_array_equal(rc, expect)
    lu = cache.last_used()
    for slot, f in stamps.items():
        assert lu[slot] == f
    assert (st["hits"], st["fallbacks"], st["misses"]) == (counts["hit"], counts["fb"], counts["miss"])


@pytest.mark.parametrize("seed,frac,S", [(3, 0.4, 4), (4, 0.8, 3), (5, 0.1, 6)])
def test_brute_force_schedule_with_early_termination(seed, frac, S):
    # the wavefront schedule with early termination on a non-constant field:
    # the samples decided past an early termination inside a wavefront step
    # still request and stamp, the others are never decided
    dims = (9, 10, 11)
    B, n_lods = 3, 3
    m = oracle_inr(configs.ARCH_SMALL, seed, dims=dims)
    _, nb, off = O.lod_geometry(dims, B, n_lods)
    n_keys = int(off[-1])
    rng = np.random.default_rng(seed)
    keys = np.sort(rng.choice(n_keys, size=int(n_keys * frac), replace=False)).astype(np.int32)
    cache = O.OracleCache(m, brick=B, n_lods=n_lods, pool_bricks=n_keys, max_requests=0)
    if keys.size:
        cache.prefill(keys, stamp=0)
    pt = cache.page_table()
    resident = {int(k): int(pt[k]) for k in keys}
    cam = synth.orbit_camera(synth.PERSPECTIVE, dims, 18.0, 10.0 + 50 * seed, 15.0, 7, 6, fov_y_deg=50.0)
    tf = synth.tf_random(seed)
    tf[:, 3] = np.clip(tf[:, 3] * 1.5, 0, 1)
    lod_scale, thr = 0.12, 0.9
    p = O.make_params(0.5, lod_scale, seed=11, frame_index=3, ert_threshold=thr, samples_per_iter=S, mode=O.CACHED)
    img, st = cache.render(cam, tf, p)
    ref, req, stamps, counts = _brute_force_frame(m, dims, B, n_lods, resident, cam, tf, 0.5, lod_scale, 11, 3, 0,
                                                  ert=thr, S=S)
    full, *_ = _brute_force_frame(m, dims, B, n_lods, resident, cam, tf, 0.5, lod_scale, 11, 3, 0)
    assert (ref[..., 3] >= thr).sum() > 5 and not np.array_equal(ref, full)  # some rays end early
    np.testing.assert_allclose(img, ref, rtol=0, atol=1e-12)
    rc = cache.req_count()
    expect = np.zeros(n_keys, np.uint32)
    for k, v in req.items():
        expect[k] = v
    np.testing.assert_array_equal(rc, expect)
    lu = cache.last_used()
    for slot, f in stamps.items():
        assert lu[slot] == f
    assert (st["hits"], st["fallbacks"], st["misses"]) == (counts["hit"], counts["fb"], counts["miss"])


# ---------------------------------------------------------------------------
# Stochastic LoD (Algorithm 2, Section 5.3)
# ---------------------------------------------------------------------------


def _lods(xs, seed=0x1234567, floor=0, n_lods=6):
    eye = np.zeros(3, np.float32)
    return np.array([O.select_lod(np.array([x, 0, 0], np.float32), eye, 1.0, seed, floor, n_lods) for x in xs])


def test_stochastic_lod_values_and_mean():
    rng = np.random.default_rng(0)
    xs = rng.uniform(1.2, 1.3, size=20000).astype(np.float32)
    L = _lods(xs)
    assert set(np.unique(L)) <= {1, 2}
    sigma = 0.5 / math.sqrt(xs.size)
    assert abs(L.mean() - xs.astype(np.float64).mean()) < 3 * sigma


def test_stochastic_lod_is_continuous_across_integers():
    # E[L] = D: just below 1 the mean is about 0.975, just above about 1.025.
    # (Moving up when the variate exceeds the fraction would jump from
    # about 0.025 to about 1.975 here.)
    rng = np.random.default_rng(1)
    lo = _lods(rng.uniform(0.95, 1.0, size=20000).astype(np.float32)).mean()
    hi = _lods(rng.uniform(1.0, 1.05, size=20000).astype(np.float32)).mean()
    assert abs(lo - 0.975) < 0.012 and abs(hi - 1.025) < 0.012
    assert hi - lo < 0.1


def test_lod_clamps_and_preload_floor():
    assert _lods([40.7], n_lods=4)[0] == 3
    assert _lods([0.0], floor=2, n_lods=4)[0] == 2
    assert [O.lib().orc_lod_floor(f, 4, 4) for f in range(14)] == [3] * 4 + [2] * 4 + [1] * 4 + [0] * 2
    assert O.lib().orc_lod_floor(5, 0, 4) == 0


def test_frame_seed_changes_choices_between_frames():
    rng = np.random.default_rng(2)
    xs = rng.uniform(2.0, 3.0, size=2000).astype(np.float32)
    a = _lods(xs, seed=O.lib().orc_frame_seed(1, 0))
    b = _lods(xs, seed=O.lib().orc_frame_seed(1, 1))
    assert 0.2 < np.mean(a != b) < 0.8


# ---------------------------------------------------------------------------
# Macro-cell skipping (Section 5.2)
# ---------------------------------------------------------------------------


def test_macrocell_skip_is_exact_in_lattice_mode():
    # a smooth field (value = normalised x) so that whole cells are transparent
    m = coordinate_inr((64, 64, 64), 0)
    mm = m.macrocells(16)
    tf = synth.tf_window(140, 255)
    cam = configs.SMALL.camera(2)
    cam.width = cam.height = 20
    p0 = O.make_params(0.5, 1 / 96, mode=O.UNCACHED_LATTICE)
    p1 = O.make_params(0.5, 1 / 96, mode=O.UNCACHED_LATTICE, macro_cell=16, macro_minmax=mm)
    a, sa = O.render_uncached(m, cam, tf, p0)
    b, sb = O.render_uncached(m, cam, tf, p1)
    assert sb["skipped"] > 0
    np.testing.assert_array_equal(a, b)


def test_pixel_renderer_matches_full_frames():
    m = oracle_inr(configs.ARCH_SMALL, 0)
    w = configs.SMALL
    cam = w.camera(1)
    cam.width = cam.height = 40
    px = np.arange(0, 1600, 7)
    p = O.make_params(0.5, w.lod_scale, seed=3, frame_index=2, samples_per_iter=8, mode=O.UNCACHED_DIRECT)
    full, _ = O.render_uncached(m, cam, w.tf(0), p)
    np.testing.assert_array_equal(full.reshape(-1, 4)[px], O.render_pixels(m, cam, w.tf(0), p, px))
    c = O.OracleCache(m, brick=8, n_lods=2, pool_bricks=400, max_requests=16)
    c.prefill(np.arange(0, 854, 3), 0)
    p.mode = O.CACHED
    part = O.render_pixels(m, cam, w.tf(0), p, px, cache=c)
    before = c.page_table().copy()
    full, _ = c.render(cam, w.tf(0), p)
    np.testing.assert_array_equal(full.reshape(-1, 4)[px], part)
    assert np.array_equal(before[before >= 0], c.page_table()[before >= 0])
