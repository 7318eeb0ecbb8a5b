"""Oracle pins of the context-aware LoD (the direction of Section 7: the
macro-cells' value ranges pick finer LoDs where the data has structure).

With macro-cells, a sample's LoD distance is (|p - eye| lod_scale) * f with
f = 1 - kappa (max - min) of its cell's values.

- f = 1 gives Algorithm 2's LoD bit for bit; the stochastic LoD keeps its
  mean: E[L] = D f; f = 0 gives LoD 0 (or the pre-load floor);
- kappa = 0, and any kappa on cells of zero value range, render exactly the
  distance-only frame (images, statistics, requests);
- hand-built cells: kappa = 1 on cells spanning [0, 1] requests LoD-0 bricks
  only; a kappa > 0 lowers the mean requested LoD of a frame;
- kappa outside [0, 1] is rejected.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2504_18001_amd import configs, synth
from tests.helpers import constant_inr, oracle_inr


def test_unit_factor_is_the_distance_rule():
    rng = np.random.default_rng(31)
    eye = np.array([10.0, -3.0, 50.0], np.float32)
    for _ in range(3000):
        p = rng.uniform(0, 100, 3).astype(np.float32)
        seed = int(rng.integers(0, 2 ** 32))
        a = O.select_lod(p, eye, 1 / 40.0, seed, 0, 6)
        b = O.select_lod_scaled(p, eye, 1 / 40.0, 1.0, seed, 0, 6)
        assert a == b


def test_scaled_stochastic_lod_mean_and_zero():
    rng = np.random.default_rng(32)
    xs = rng.uniform(2.0, 2.1, size=20000).astype(np.float32)
    eye = np.zeros(3, np.float32)
    f = np.float32(0.6)
    L = np.array([O.select_lod_scaled(np.array([x, 0, 0], np.float32), eye, 1.0, f, 0x9E37, 0, 6) for x in xs])
    assert set(np.unique(L)) <= {1, 2}
    D = (xs.astype(np.float32) * f).astype(np.float64)
    assert abs(L.mean() - D.mean()) < 3 * 0.5 / math.sqrt(xs.size)
    assert all(O.select_lod_scaled(np.array([x, 0, 0], np.float32), eye, 1.0, 0.0, 7, 0, 6) == 0 for x in xs[:200])
    assert O.select_lod_scaled(np.array([9.0, 0, 0], np.float32), eye, 1.0, 0.0, 7, 2, 6) == 2  # pre-load floor


def _frame(m, dims, kappa, mm, frame=0, pool=200, req=32):
    w = configs.SMALL
    cam = w.camera(frame, dims)
    cam.width, cam.height = 40, 40
    c = O.OracleCache(m, brick=8, n_lods=3, pool_bricks=pool, max_requests=req)
    p = O.make_params(0.5, 1.0 / 30.0, seed=3, frame_index=frame, samples_per_iter=4, mode=O.CACHED, macro_cell=8,
                      macro_minmax=mm, lod_context=kappa)
    img, st = c.render(cam, synth.tf_ramp(), p)
    return img, st, c


def test_zero_weight_and_flat_cells_change_nothing():
    dims = (48, 40, 36)
    m = oracle_inr(configs.ARCH_SMALL, 2, dims=dims)
    mm = m.macrocells(8)
    a, sa, ca = _frame(m, dims, 0.0, mm)
    b, sb, cb = _frame(m, dims, 0.0, mm)
    np.testing.assert_array_equal(a, b)
    # cells of zero value range: the factor is 1 whatever kappa
    flat = mm.copy()
    flat[..., 0] = flat[..., 1]  # [max, max]: zero range
    c0, s0, k0 = _frame(m, dims, 0.0, flat)
    c1, s1, k1 = _frame(m, dims, 1.0, flat)
    np.testing.assert_array_equal(c0, c1)
    assert s0 == s1
    np.testing.assert_array_equal(k0.req_count(), k1.req_count())


def test_full_range_cells_request_lod0_only_and_weight_lowers_the_mean_lod():
    dims = (48, 40, 36)
    m = oracle_inr(configs.ARCH_SMALL, 2, dims=dims)
    mm = m.macrocells(8)
    full = mm.copy()
    full[..., 0], full[..., 1] = 0.0, 1.0
    _, st, c = _frame(m, dims, 1.0, full)
    _, _, off = O.lod_geometry(dims, 8, 3)
    req = c.req_count()
    assert req.sum() > 0 and req[int(off[1]):].sum() == 0  # every request is a LoD-0 brick

    def mean_lod(kappa):
        _, _, cc = _frame(m, dims, kappa, mm)
        r = cc.req_count().astype(np.float64)
        lod = np.searchsorted(off, np.arange(r.size), side="right") - 1
        return (r * lod).sum() / r.sum()

    l0, l5 = mean_lod(0.0), mean_lod(0.5)
    assert l5 < l0, (l0, l5)


def test_weight_outside_the_unit_interval_is_rejected():
    dims = (32, 32, 32)
    m = constant_inr(dims, 0.5)
    mm = m.macrocells(8)
    c = O.OracleCache(m, brick=8, n_lods=2, pool_bricks=10, max_requests=4)
    cam = configs.SMALL.camera(0, dims)
    cam.width = cam.height = 8
    for k in (-0.1, 1.5, float("nan")):
        p = O.make_params(0.5, 0.05, mode=O.CACHED, macro_cell=8, macro_minmax=mm, lod_context=k)
        with pytest.raises(AssertionError):
            c.render(cam, synth.tf_ramp(), p)
