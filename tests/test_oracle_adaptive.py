"""Oracle pins of the adaptive sampling rate (Section 5.2): a macro-cell's
maximum opacity sets the step across it, on the ray's fixed sample grid.

- the step exponent min(E, floor(-log2 mu)) against its defining inequality
  2^-(e+1) < mu <= 2^-e, on hand values and on random binary32 opacities;
- per-cell codes on hand-built cells and TFs (transparent cells, clamping);
- E = 0 is the fixed-step sampler, bit for bit (images, statistics, cache);
- a constant opacity of 0.3 in every cell (exponent 1) samples every second
  grid point: bit-identical to the fixed sampler with twice the step, in the
  uncached, lattice and cached modes;
- a transparent volume takes ceil(n / 2^E) steps along a ray of n grid
  samples, all of them skipped.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2504_18001_amd import configs, synth
from tests.helpers import oracle_inr


def test_step_exponent_hand_values():
    cases = [(1.0, 3, 0), (0.9, 3, 0), (0.5, 3, 1), (0.49, 3, 1), (0.3, 3, 1), (0.25, 3, 2), (0.2, 3, 2),
             (0.125, 3, 3), (0.01, 3, 3), (0.01, 10, 6), (2.0 ** -20, 30, 20), (1.5, 3, 0), (0.75, 0, 0)]
    for mu, E, e in cases:
        assert O.step_exp(mu, E) == e, (mu, E)


def test_step_exponent_is_floor_of_minus_log2():
    rng = np.random.default_rng(3)
    mus = np.concatenate([rng.uniform(0, 1, 20000), 2.0 ** -rng.uniform(0, 40, 20000)]).astype(np.float32)
    mus = mus[mus > 0]
    for mu in mus[:8000]:
        e = O.step_exp(float(mu), 126)
        m = float(mu)  # exact in float64; multiplying by powers of two is exact
        assert m * 2.0 ** e <= 1.0 < m * 2.0 ** (e + 1), (m, e)
    # exact powers of two sit on the lower exponent
    for k in range(0, 30):
        assert O.step_exp(2.0 ** -k, 126) == k


def test_step_codes_of_hand_built_cells():
    tf = np.zeros((256, 4), np.float32)
    tf[100:200, 3] = 0.3
    tf[200:, 3] = 1.0
    # cells given by [min, max]: rows [floor(255 min), ceil(255 max)]
    mm = np.array([[0.10, 0.20],    # rows 25..51: transparent
                   [0.45, 0.50],    # rows 114..128: mu = 0.3 -> 1
                   [0.50, 0.90],    # rows 127..230: mu = 1 -> 0
                   [0.0, 0.3921],   # rows 0..100: touches row 100 (0.3) -> 1
                   [0.0, 0.39],     # rows 0..100 (99.45 rounds up): also 1
                   [0.0, 0.388]],   # rows 0..99: transparent
                  np.float32)
    codes = O.macrocell_step_codes(mm, tf, 3)
    assert codes.tolist() == [255, 1, 0, 1, 1, 255]
    tf[100:200, 3] = 0.05  # -> exponent 4, clamped to E
    assert O.macrocell_step_codes(mm, tf, 3).tolist() == [255, 3, 0, 3, 3, 255]
    assert O.macrocell_step_codes(mm, tf, 6).tolist() == [255, 4, 0, 4, 4, 255]
    # the flags of the fixed sampler are the non-transparent codes
    assert (O.macrocell_flags(mm, tf) == (O.macrocell_step_codes(mm, tf, 6) != 255)).all()


def _scene(W=24):
    m = oracle_inr(configs.ARCH_SMALL, 0)
    w = configs.SMALL
    cam = w.camera(1)
    cam.width = cam.height = W
    return m, w, cam


@pytest.mark.parametrize("mode", [O.UNCACHED_DIRECT, O.UNCACHED_LATTICE, O.CACHED])
def test_exponent_zero_is_the_fixed_sampler(mode):
    m, w, cam = _scene()
    mm = m.macrocells(16)
    tf = synth.tf_window(60, 255)
    out = []
    for E in (-1, 0):
        p = O.make_params(w.step, w.lod_scale, seed=w.seed, samples_per_iter=4, mode=mode, macro_cell=16,
                          macro_minmax=mm, adapt_max_exp=E)
        if mode == O.CACHED:
            c = O.OracleCache(m, brick=8, n_lods=2, pool_bricks=40, max_requests=12)
            for f in range(3):
                p.frame_index = f
                img, st = c.render(cam, tf, p)
            out.append((img, st, c.page_table()))
        else:
            img, st = O.render_uncached(m, cam, tf, p)
            out.append((img, st, None))
    (a, sa, pa), (b, sb, pb) = out
    np.testing.assert_array_equal(a, b)
    assert sa == sb
    if pa is not None:
        np.testing.assert_array_equal(pa, pb)


@pytest.mark.parametrize("mode", [O.UNCACHED_DIRECT, O.UNCACHED_LATTICE, O.CACHED])
def test_constant_opacity_samples_every_second_grid_point(mode):
    m, w, cam = _scene()
    mm = m.macrocells(16)
    tf = synth.tf_ramp().astype(np.float32)
    tf[:, 3] = 0.3  # every cell: mu = 0.3, exponent 1; colours still follow the value
    out = []
    for step, E in ((w.step, 3), (2.0 * w.step, -1)):
        p = O.make_params(step, w.lod_scale, seed=w.seed, samples_per_iter=4, mode=mode, macro_cell=16,
                          macro_minmax=mm, adapt_max_exp=E)
        if mode == O.CACHED:
            c = O.OracleCache(m, brick=8, n_lods=2, pool_bricks=40, max_requests=12)
            for f in range(3):
                p.frame_index = f
                img, st = c.render(cam, tf, p)
            out.append((img, st, c.page_table(), c.last_used()))
        else:
            img, st = O.render_uncached(m, cam, tf, p)
            out.append((img, st, None, None))
    (a, sa, pa, la), (b, sb, pb, lb) = out
    assert sa["samples"] > 0
    np.testing.assert_array_equal(a, b)
    assert sa == sb
    if pa is not None:
        np.testing.assert_array_equal(pa, pb)
        np.testing.assert_array_equal(la, lb)


@pytest.mark.parametrize("E", [1, 2, 3, 5])
def test_transparent_volume_steps(E):
    m, w, cam = _scene(W=1)
    mm = m.macrocells(16)
    tf = np.zeros((256, 4), np.float32)
    counts = {}
    for e in (0, E):
        p = O.make_params(w.step, w.lod_scale, mode=O.UNCACHED_DIRECT, macro_cell=16, macro_minmax=mm,
                          adapt_max_exp=e)
        img, st = O.render_uncached(m, cam, tf, p)
        assert float(np.abs(img).max()) == 0.0
        assert st["skipped"] == st["samples"] and st["misses"] == 0
        counts[e] = st["samples"]
    n = counts[0]
    assert n > 40  # the single ray crosses the volume
    assert counts[E] == math.ceil(n / 2 ** E)
