"""The adaptive sampling rate (Section 5.2) on the GPU against the oracle:
cached sequences (images, statistics, page table, stamps, ranks, request
lists, eviction and miss logs), the uncached INR renderer, and the constant
opacity case against the fixed sampler at twice the step (two different
kernels, bit for bit)."""
import numpy as np
import pytest
import torch

from paper_2504_18001_amd import configs, synth
from tests.helpers import oracle_inr
from tests.test_gpu_parity import TOL, _render_gpu, gpu_volume, run_cached_sequence

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("E", [1, 3])
def test_cached_sequence_adaptive(E):
    w = configs.SMALL
    worst = run_cached_sequence(w, range(8), 96, 96, macro=True, adapt=E, tf_fn=lambda f: synth.tf_window(60, 255))
    print("adaptive E", E, "worst", worst)


def test_cached_sequence_adaptive_512_arch():
    # the 512^3 architecture on a 120x104x96 volume, 16^3 bricks and macro-cells (the
    # sampler's 16^3 specialisation), 4 LoDs with pre-load
    w = configs.scaled(configs.HD512, 80, 45, orbit_radius=260.0, lod_scale=1.0 / 180.0)
    run_cached_sequence(w, range(6), 80, 45, dims=(120, 104, 96), pool=300, max_req=12, preload=2, macro=True,
                        adapt=2, tf_fn=lambda f: synth.tf_window(40, 255))


def test_uncached_adaptive_matches_oracle():
    from oracle import oracle as O
    from paper_2504_18001_amd import cinr
    w = configs.SMALL
    m = oracle_inr(w.arch, 0)
    mm = m.macrocells(16)
    vol = gpu_volume(w.arch, 0, macrocells=mm, macro_cell=16)
    tf = synth.tf_window(60, 255)
    for frame in (0, 2):
        cam = w.camera(frame)
        cam.width = cam.height = 64
        img, st = _render_gpu(vol, cam, tf, w, frame, cinr.UNCACHED_DIRECT, "f32", adapt=3)
        p = O.make_params(w.step, w.lod_scale, seed=w.seed, frame_index=frame, samples_per_iter=w.samples_per_iter,
                          mode=O.UNCACHED_DIRECT, macro_cell=16, macro_minmax=mm, adapt_max_exp=3)
        ref, rst = O.render_uncached(m, cam, tf, p)
        for k in ("rays", "samples", "hits", "fallbacks", "misses", "skipped"):
            assert st[k] == rst[k], (frame, k, st[k], rst[k])
        assert np.abs(img - ref).max() <= TOL["f32"]


@pytest.mark.parametrize("mode", ["uncached", "cached"])
def test_constant_opacity_equals_fixed_sampler_at_twice_the_step(mode):
    from paper_2504_18001_amd import cinr
    w = configs.SMALL
    m = oracle_inr(w.arch, 0)
    mm = m.macrocells(16)
    tf = synth.tf_ramp().astype(np.float32)
    tf[:, 3] = 0.3  # every macro-cell has exponent 1
    out = []
    for step, E in ((w.step, 3), (2.0 * w.step, 0)):
        vol = gpu_volume(w.arch, 0, macrocells=mm, macro_cell=16)
        cache = cinr.Cache(vol, 8, 2, 96, 16) if mode == "cached" else None
        r = cinr.Renderer()
        for f in range(4):
            cam = w.camera(f)
            cam.width = cam.height = 96
            img, st = _render_gpu(vol, cam, tf, w, f, cinr.CACHED if cache else cinr.UNCACHED_DIRECT, "f32",
                                  cache=cache, renderer=r, adapt=E, step=step)
        out.append((img, st, cache.dump(cinr.DUMP_PAGE_TABLE) if cache else None))
    (a, sa, pa), (b, sb, pb) = out
    assert sa["samples"] > 0
    np.testing.assert_array_equal(a, b)
    for k in ("rays", "samples", "hits", "fallbacks", "misses", "skipped", "requested", "selected"):
        assert sa[k] == sb[k], k
    if pa is not None:
        np.testing.assert_array_equal(pa, pb)
