"""Oracle pins of the reduced-precision brick pool (binary16 brick values, a
direction Section 7 leaves open): decoded brick values are rounded to the
nearest binary16 value, ties to even, when inserted; sampling interpolates
the rounded values.

- the rounding against hand values fixed by the binary16 format (ties to
  even, the largest finite value and the overflow threshold, subnormals);
- the rounding against numpy's float64 -> float16 conversion, an independent
  implementation, on values spread over the whole binary16 range;
- the rounded value is representable and within half a quantum of x;
- a prefilled pool and a pool filled by rendering are exactly the binary16
  rounding of the full-precision pool, slot for slot;
- a constant field renders, through the rounded pool, exactly as the same
  field with its value rounded beforehand.
"""
import numpy as np

from oracle import oracle as O
from paper_2504_18001_amd import configs, synth
from tests.helpers import constant_inr, oracle_inr


def test_round_half_hand_values():
    cases = [
        (1.0, 1.0),
        (1.0 + 2.0 ** -11, 1.0),                    # tie between 1 and 1 + 2^-10: even is 1
        (1.0 + 3 * 2.0 ** -11, 1.0 + 2.0 ** -9),    # tie between 1 + 2^-10 (odd) and 1 + 2^-9 (even)
        (1.0 + 2.0 ** -11 + 2.0 ** -30, 1.0 + 2.0 ** -10),  # just above the tie
        (0.1, 1638.0 / 16384.0),                    # 0.1 = 1.6 * 2^-4, quantum 2^-14: 1638.4 -> 1638
        (65504.0, 65504.0),                         # largest finite value
        (65519.99, 65504.0),                        # below the overflow threshold 65520
        (65520.0, np.inf),                          # tie with 2^16 rounds to even = overflow
        (-65520.0, -np.inf),
        (2.0 ** -14, 2.0 ** -14),                   # smallest normal
        (2.0 ** -24, 2.0 ** -24),                   # smallest subnormal
        (2.0 ** -25, 0.0),                          # tie with 0: even is 0
        (3 * 2.0 ** -25, 2.0 ** -23),               # tie between 1 (odd) and 2 (even) quanta
        (1.4 * 2.0 ** -24, 2.0 ** -24),
        (-0.3, -(1229.0 / 4096.0)),                 # 0.3 = 1.2 * 2^-2, quantum 2^-12: 1228.8 -> 1229
        (0.0, 0.0),
    ]
    for x, want in cases:
        assert O.round_half(x) == want, (x, O.round_half(x), want)


def test_round_half_matches_numpy_float16():
    rng = np.random.default_rng(11)
    mags = 10.0 ** rng.uniform(-9, 5.2, 30000)
    xs = np.concatenate([mags * rng.choice([-1.0, 1.0], mags.size), rng.uniform(-1, 1, 10000)])
    with np.errstate(over="ignore"):
        ref = xs.astype(np.float16).astype(np.float64)
    got = np.array([O.round_half(x) for x in xs])
    np.testing.assert_array_equal(got, ref)


def test_round_half_is_representable_and_nearest():
    rng = np.random.default_rng(12)
    xs = np.sort(rng.uniform(-4.0, 4.0, 20000))
    r = np.array([O.round_half(x) for x in xs])
    # representable: the binary16 cast keeps it
    np.testing.assert_array_equal(r.astype(np.float16).astype(np.float64), r)
    # within half the quantum of x's binade (2^(floor(log2|x|) - 10), at least 2^-24)
    q = np.maximum(2.0 ** (np.floor(np.log2(np.abs(xs))) - 10), 2.0 ** -24)
    assert np.all(np.abs(r - xs) <= q / 2)
    # monotone
    assert np.all(np.diff(r) >= 0)


def _caches(m, pool, max_req=16, B=8, n_lods=2):
    c64 = O.OracleCache(m, brick=B, n_lods=n_lods, pool_bricks=pool, max_requests=max_req)
    c16 = O.OracleCache(m, brick=B, n_lods=n_lods, pool_bricks=pool, max_requests=max_req, pool_f16=True)
    return c64, c16


def _rounded(a):
    return a.astype(np.float16).astype(np.float64)


def test_prefilled_pool_is_the_rounded_pool():
    m = oracle_inr(configs.ARCH_SMALL, 0)
    c64, c16 = _caches(m, pool=40)
    keys = np.arange(3, 3 + 40 * 3, 3, dtype=np.int32)
    keys = keys[keys < c64.n_keys][:40]
    c64.prefill(keys)
    c16.prefill(keys)
    np.testing.assert_array_equal(c16.owner(), c64.owner())
    p64, p16 = c64.pool(), c16.pool()
    np.testing.assert_array_equal(p16, _rounded(p64))
    assert np.any(p16 != p64)  # the INR's values are not all binary16 numbers


def test_rendered_pool_is_the_rounded_pool():
    # early termination off: the caching decisions do not depend on values,
    # so both caches insert and evict the same bricks
    w = configs.SMALL
    m = oracle_inr(w.arch, 0)
    c64, c16 = _caches(m, pool=60)
    worst, evicted = 0.0, 0
    for f in range(8):
        cam = w.camera(f)
        cam.width, cam.height = 40, 32
        p = O.make_params(w.step, w.lod_scale, seed=w.seed, frame_index=f, samples_per_iter=w.samples_per_iter,
                          mode=O.CACHED, ert_threshold=2.0)
        img64, st64 = c64.render(cam, w.tf(f), p)
        img16, st16 = c16.render(cam, w.tf(f), p)
        assert st16 == st64, f
        np.testing.assert_array_equal(c16.owner(), c64.owner())
        np.testing.assert_array_equal(c16.page_table(), c64.page_table())
        np.testing.assert_array_equal(c16.pool(), _rounded(c64.pool()))
        worst = max(worst, float(np.abs(img16 - img64).max()))
        evicted += st64["evicted"]
    assert evicted > 0  # the pool filled and slots were reused
    # the pool's rounding (relative 2^-11) reaches the image, and only a little
    assert 0.0 < worst < 2e-3, worst


def test_constant_field_renders_the_rounded_value():
    dims = (24, 24, 24)
    v = float(np.float32(0.3))
    vr = O.round_half(v)
    assert vr != v
    tf = synth.tf_ramp()
    cam = configs.SMALL.camera(1, dims)
    cam.width, cam.height = 24, 20
    p = O.make_params(0.5, 0.05, ert_threshold=2.0, samples_per_iter=4, mode=O.CACHED)
    imgs = {}
    for name, value, f16 in (("f16", v, True), ("rounded", vr, False), ("exact", v, False)):
        m = constant_inr(dims, value)
        c = O.OracleCache(m, brick=4, n_lods=2, pool_bricks=4096, max_requests=0, pool_f16=f16)
        c.prefill(np.arange(c.n_keys, dtype=np.int32))
        imgs[name], st = c.render(cam, tf, p)
        assert st["misses"] == 0 and st["samples"] > 0
    np.testing.assert_array_equal(imgs["f16"], imgs["rounded"])
    assert np.abs(imgs["f16"] - imgs["exact"]).max() > 0
