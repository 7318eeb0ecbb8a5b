"""Oracle pins of path tracing with Woodcock delta tracking through the same
sampler (Section 5.1).

The medium has extinction pt_density * TF opacity, TF colour as albedo, an
isotropic phase function, one directional light (next-event estimate by a
delta-tracked shadow ray) and an environment term for scattered rays that
leave the box.

- primitives: the free-flight length is the correctly rounded binary32 value
  of -ln(xi) (checked against 50-digit decimal logarithms) and Exp(1)
  distributed; uniforms on hand values; Marsaglia directions are unit vectors,
  uniform on the sphere, and take 4/pi draws on average; segment exits and the
  binary32 TF opacity on hand cases;
- closed forms of a homogeneous slab seen by an orthographic camera: the
  collision probability 1 - exp(-sigma L), single scattering with the light
  behind the camera, rho (1 - exp(-2 sigma L)) / 2, and with the light across
  the view, rho (1 - exp(-sigma L)) exp(-sigma s(x)); opacity 1 (every
  tentative collision real) and 0 (none);
- a white furnace: albedo 1, environment 1, no light: every colliding path
  returns exactly 1, so colour equals opacity pixel by pixel;
- invariants: the image does not depend on how many tentative collisions are
  gathered after a true miss (only the lookup counts do); an empty cache gives
  the uncached image (I1); a fully resident LoD-0 cache gives the lattice
  image (I2); the event budget drops cut paths without bias.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from paper_2504_18001_amd import configs, synth
from tests.helpers import constant_inr, oracle_inr
from tests.test_oracle_render import _ortho_z


# ---------------------------------------------------------------------------
# Primitives
# ---------------------------------------------------------------------------


def _round_f32(x: Decimal) -> np.float32:
    """x rounded to the nearest binary32 value (ties to even), exactly."""
    f = np.float32(float(x))
    best = None
    for c in (np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))):
        err = abs(Decimal(float(c)) - x)
        if best is None or err < best[0] or (err == best[0] and (c.view(np.uint32) & 1) == 0):
            best = (err, c)
    return best[1]


def test_free_flight_is_correctly_rounded_minus_log():
    getcontext().prec = 50
    rng = np.random.default_rng(21)
    words = np.concatenate([rng.integers(0, 2 ** 32, 3000, dtype=np.uint64),
                            [0, 255, 256, 0xFFFFFFFF, 0xFFFFFF00, 0x80000000]]).astype(np.uint64)
    for r in words:
        m = int(r) >> 8
        xi = Decimal(m + 1) / Decimal(2 ** 24)
        want = _round_f32(-xi.ln()) if m + 1 < 2 ** 24 else np.float32(0.0)
        got = np.float32(O.pt_free_flight(int(r)))
        assert got == want, (int(r), got, want)
    # the largest step: xi = 2^-24, -ln xi = 24 ln 2
    assert np.float32(O.pt_free_flight(0)) == _round_f32(24 * Decimal(2).ln())


def test_free_flight_is_exponential():
    words = np.random.default_rng(22).integers(0, 2 ** 32, 20000, dtype=np.uint64)
    E = np.array([O.pt_free_flight(int(r)) for r in words])
    assert stats.kstest(E, "expon").pvalue > 1e-3
    assert abs(E.mean() - 1.0) < 4 / math.sqrt(E.size)


def test_uniform_hand_values():
    assert O.pt_uniform(0) == 0.0
    assert O.pt_uniform(255) == 0.0
    assert O.pt_uniform(256) == 2.0 ** -24
    assert O.pt_uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert O.pt_uniform(0x80000000) == 0.5


def test_marsaglia_directions_are_uniform_unit_vectors():
    key = (9, 3)
    n = 0
    dirs = []
    for pix in range(4000):
        d, n1 = O.pt_direction(pix, 17, key)
        dirs.append(d)
        n += n1 - 17
    D = np.asarray(dirs, np.float64)
    norms = np.linalg.norm(D, axis=1)
    assert np.abs(norms - 1.0).max() < 4e-7
    # uniform on the sphere: each coordinate uniform on [-1, 1], azimuth uniform
    assert stats.kstest(D[:, 2], "uniform", args=(-1, 2)).pvalue > 1e-3
    assert stats.kstest(D[:, 0], "uniform", args=(-1, 2)).pvalue > 1e-3
    phi = np.arctan2(D[:, 1], D[:, 0])
    assert stats.kstest(phi, "uniform", args=(-math.pi, 2 * math.pi)).pvalue > 1e-3
    assert np.abs(D.mean(0)).max() < 4 / math.sqrt(3 * len(D))
    # acceptance of the square's points inside the unit disc: pi / 4
    assert abs(n / len(D) - 4 / math.pi) < 0.05


def test_segment_exit_hand_cases():
    vm1 = (10.0, 10.0, 10.0)
    assert O.pt_segment_exit((1, 2, 3), (1, 0, 0), vm1) == 9.0
    assert O.pt_segment_exit((1, 2, 3), (-1, 0, 0), vm1) == 1.0
    assert O.pt_segment_exit((1, 2, 3), (0.6, 0.8, 0), vm1) == np.float32(8.0) / np.float32(0.8)
    assert O.pt_segment_exit((1, 2, 3), (0, 0, -1), vm1) == 3.0
    assert O.pt_segment_exit((10, 2, 3), (1, 0, 0), vm1) == 0.0  # on the wall, leaving
    assert O.pt_segment_exit((0, 0, 0), (0.6, 0.0, 0.8), (30.0, 5.0, 20.0)) == np.float32(20.0) / np.float32(0.8)


def test_tf_alpha32():
    tf = np.zeros((256, 4), np.float32)
    tf[:, 3] = np.linspace(0, 1, 256, dtype=np.float32)
    tf[200:, 3] = 1.5  # clamped
    assert O.tf_alpha32(tf, 0.0) == 0.0
    assert O.tf_alpha32(tf, 1.0) == 1.0
    rng = np.random.default_rng(23)
    for v in rng.uniform(0, 0.75, 200).astype(np.float32):
        x = float(v) * 255
        i0 = min(int(x), 254)
        ref = tf[i0, 3] * (1 - (x - i0)) + tf[i0 + 1, 3] * (x - i0)
        assert abs(O.tf_alpha32(tf, v) - ref) < 1e-6
    assert O.tf_alpha32(tf, 0.9) == 1.0


# ---------------------------------------------------------------------------
# Closed forms on a homogeneous slab
# ---------------------------------------------------------------------------

DIMS = (32, 32, 32)


def _slab(alpha, rgb=(0.8, 0.5, 0.2)):
    tf = np.zeros((256, 4), np.float32)
    tf[:, 0], tf[:, 1], tf[:, 2] = rgb
    tf[:, 3] = alpha
    return tf


def _render_slab(tf, path, W=32, extent=16.0, S=4, mode=O.UNCACHED_DIRECT):
    m = constant_inr(DIMS, 0.5)
    cam = _ortho_z(DIMS, W=W, H=W, extent=extent)
    p = O.make_params(0.5, 0.1, mode=mode, samples_per_iter=S, path=path)
    img, st = O.render_uncached(m, cam, tf, p)
    return img, st, cam


def _close(x, want, n, k=5.0):
    se = math.sqrt(max(want * (1 - want), 1e-12) / n)
    assert abs(x - want) < k * se + 1e-12, (x, want, se)


def test_single_scattering_light_behind_the_camera():
    sig, alpha, spp = 0.05, 0.6, 256
    path = dict(density=sig, light_dir=(0, 0, 1), light=(1, 1, 1), max_bounces=1, spp=spp, seed=7)
    img, st, _ = _render_slab(_slab(alpha), path)
    s, L = sig * alpha, 31.0
    n = img.shape[0] * img.shape[1] * spp
    _close(img[..., 3].mean(), 1 - math.exp(-s * L), n)
    # the shadow ray from depth t back to the face the camera sees is t long
    want = (1 - math.exp(-2 * s * L)) / 2
    r, g = float(np.float32(0.8)), float(np.float32(0.5))
    _close(img[..., 0].mean() / r, want, n)
    np.testing.assert_allclose(img[..., 1] / g, img[..., 0] / r, rtol=1e-12)
    assert st["rays"] == img.shape[0] * img.shape[1] and st["misses"] == st["samples"]


def test_single_scattering_light_across_the_view():
    # light toward +x: the shadow ray leaves through the wall x = 31, s(x) = 31 - x
    sig, alpha, spp = 0.04, 1.0, 128
    W = 32
    path = dict(density=sig, light_dir=(1, 0, 0), light=(2, 2, 2), max_bounces=1, spp=spp, seed=8)
    img, _, cam = _render_slab(_slab(alpha, (1, 1, 1)), path, W=W, extent=31.0)
    L = 31.0
    xs = (np.arange(W) + 0.5) / W * 31.0 - 15.5 + 15.5  # pixel centres across [0, 31]
    for col in range(0, W, 4):
        want = (1 - math.exp(-sig * L)) * math.exp(-sig * (31.0 - xs[col]))
        got = img[:, col, 0].mean() / 2.0
        _close(got, want, W * spp)


def test_opacity_one_and_zero():
    sig = 0.07
    path = dict(density=sig, light_dir=(0, 0, 1), max_bounces=1, spp=128, seed=3)
    img, st, _ = _render_slab(_slab(1.0), path)
    _close(img[..., 3].mean(), 1 - math.exp(-sig * 31.0), img.shape[0] * img.shape[1] * 128)
    img0, st0, _ = _render_slab(_slab(0.0), path)
    assert np.all(img0 == 0.0)
    # every tentative collision is looked up and rejected: sigma L per path on average
    per_path = st0["samples"] / (img0.shape[0] * img0.shape[1] * 128)
    assert abs(per_path - sig * 31.0) < 0.05


def test_white_furnace():
    # albedo 1, environment 1, no light: a colliding path scatters until it
    # leaves the box and returns exactly 1; a path that never collides returns 0
    path = dict(density=0.05, light_dir=(0, 0, 1), light=(0, 0, 0), ambient=(1, 1, 1), max_bounces=500, spp=64,
                seed=4)
    img, _, _ = _render_slab(_slab(0.7, (1, 1, 1)), path, W=16)
    np.testing.assert_array_equal(img[..., 0], img[..., 3])
    np.testing.assert_array_equal(img[..., 2], img[..., 3])
    assert img[..., 3].max() > 0
    # one collision at most: nothing escapes after scattering, so no environment
    path["max_bounces"] = 1
    img1, _, _ = _render_slab(_slab(0.7, (1, 1, 1)), path, W=16)
    assert np.all(img1[..., :3] == 0.0) and img1[..., 3].max() > 0


def test_event_budget_drops_cut_paths_without_bias():
    # 4096 paths per pixel need about 16k events, twice the budget
    sig, alpha = 0.05, 0.6
    path = dict(density=sig, light_dir=(0, 0, 1), max_bounces=1, spp=4096, seed=7)
    img, st, _ = _render_slab(_slab(alpha), path, W=4, extent=8.0)
    assert st["samples"] < 16 * O.PT_MAX_EVENTS  # the budget ended every pixel early
    # a path takes about 4 events here, so each pixel completes about 2000;
    # 1500 per pixel sizes the standard error conservatively
    _close(img[..., 3].mean(), 1 - math.exp(-sig * alpha * 31.0), 16 * 1500)


# ---------------------------------------------------------------------------
# Invariants
# ---------------------------------------------------------------------------

PATH = dict(density=0.08, light_dir=(0.48, 0.6, 0.64), light=(3, 3, 3), ambient=(0.2, 0.3, 0.4), max_bounces=4,
            spp=2, seed=11)


def _scene():
    w = configs.SMALL
    m = oracle_inr(w.arch, 0)
    cam = w.camera(2)
    cam.width, cam.height = 24, 20
    return w, m, cam


def test_image_does_not_depend_on_the_gather_size():
    w, m, cam = _scene()
    out = {}
    for S in (1, 3, 8, 16):
        p = O.make_params(w.step, w.lod_scale, seed=w.seed, frame_index=2, samples_per_iter=S, mode=O.CACHED, path=PATH)
        c = O.OracleCache(m, brick=8, n_lods=2, pool_bricks=60, max_requests=16)
        c.prefill(np.arange(0, c.n_keys, 7, dtype=np.int32)[:60])
        out[S] = c.render(cam, w.tf(2), p)
    for S in (3, 8, 16):
        np.testing.assert_array_equal(out[S][0], out[1][0])
    assert out[1][1]["samples"] < out[3][1]["samples"] < out[8][1]["samples"] == out[16][1]["samples"]
    assert out[8][1]["misses"] > 0 and out[8][1]["hits"] > 0


def test_I1_empty_cache_equals_uncached_paths():
    w, m, cam = _scene()
    p = O.make_params(w.step, w.lod_scale, seed=w.seed, frame_index=0, samples_per_iter=4, mode=O.CACHED, path=PATH)
    c = O.OracleCache(m, brick=8, n_lods=2, pool_bricks=96, max_requests=16)
    img_c, st = c.render(cam, w.tf(0), p)
    p.mode = O.UNCACHED_DIRECT
    img_u, st_u = O.render_uncached(m, cam, w.tf(0), p)
    np.testing.assert_array_equal(img_c, img_u)
    assert st["misses"] == st["samples"] == st_u["samples"] > 0
    assert img_u[..., 3].max() > 0 and img_u[..., 0].max() > 0


def test_I2_full_lod0_cache_equals_lattice_paths():
    dims = (24, 20, 18)
    m = oracle_inr(configs.ARCH_SMALL, 3, dims=dims)
    cam = synth.orbit_camera(synth.PERSPECTIVE, dims, 60.0, 30.0, 15.0, 20, 16, fov_y_deg=40.0)
    _, _, off = O.lod_geometry(dims, 5, 1)
    n = int(off[-1])
    c = O.OracleCache(m, brick=5, n_lods=1, pool_bricks=n, max_requests=n)
    c.prefill(np.arange(n, dtype=np.int32))
    p = O.make_params(0.5, 0.01, seed=1, frame_index=1, samples_per_iter=4, mode=O.CACHED, path=PATH)
    img, st = c.render(cam, synth.tf_ramp(), p)
    assert st["hits"] == st["samples"] > 0 and st["misses"] == 0
    p.mode = O.UNCACHED_LATTICE
    ref, _ = O.render_uncached(m, cam, synth.tf_ramp(), p)
    np.testing.assert_array_equal(img, ref)


def test_seed_and_frame_change_the_paths_only():
    w, m, cam = _scene()
    base = O.make_params(w.step, w.lod_scale, seed=w.seed, frame_index=0, samples_per_iter=4,
                         mode=O.UNCACHED_DIRECT, path=PATH)
    a, _ = O.render_uncached(m, cam, w.tf(0), base)
    b, _ = O.render_uncached(m, cam, w.tf(0), base)
    np.testing.assert_array_equal(a, b)
    other = O.make_params(w.step, w.lod_scale, seed=w.seed, frame_index=0, samples_per_iter=4,
                          mode=O.UNCACHED_DIRECT, path=dict(PATH, seed=12))
    c, _ = O.render_uncached(m, cam, w.tf(0), other)
    assert np.any(a != c)
    base.frame_index = 1
    d, _ = O.render_uncached(m, cam, w.tf(0), base)
    assert np.any(a != d)


def test_invalid_path_parameters_are_rejected():
    w, m, cam = _scene()
    for bad in (dict(PATH, density=0.0), dict(PATH, spp=0), dict(PATH, max_bounces=0)):
        p = O.make_params(w.step, w.lod_scale, mode=O.UNCACHED_DIRECT, path=bad)
        with pytest.raises(AssertionError):
            O.render_uncached(m, cam, w.tf(0), p)
    p = O.make_params(w.step, w.lod_scale, mode=O.UNCACHED_DIRECT, path=PATH, adapt_max_exp=1)
    with pytest.raises(AssertionError):
        O.render_uncached(m, cam, w.tf(0), p)
