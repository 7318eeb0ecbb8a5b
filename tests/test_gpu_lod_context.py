"""Context-aware LoD (macro-cell value ranges scale the LoD distance) on the
GPU against the oracle: cached sequences with the sampler's generic and 16^3
forms, the adaptive sampling rate, and the path tracer, with statistics and
all cache state bit-exact and images within tolerance."""
import numpy as np
import pytest
import torch

from paper_2504_18001_amd import configs, synth
from tests.test_gpu_parity import run_cached_sequence

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kappa", [0.5, 1.0])
def test_cached_sequence_lod_context(kappa):
    w = configs.scaled(configs.SMALL, 96, 96, lod_scale=1.0 / 40.0)
    run_cached_sequence(w, range(8), 96, 96, macro=True, lod_context=kappa, tf_fn=lambda f: synth.tf_window(40, 255))


def test_cached_sequence_lod_context_512_arch_adaptive():
    w = configs.scaled(configs.HD512, 80, 45, orbit_radius=260.0, lod_scale=1.0 / 120.0)
    run_cached_sequence(w, range(6), 80, 45, dims=(120, 104, 96), pool=300, max_req=12, preload=2, macro=True,
                        adapt=2, lod_context=0.7, tf_fn=lambda f: synth.tf_window(40, 255))


def test_cached_sequence_lod_context_512_arch():
    w = configs.scaled(configs.HD512, 80, 45, orbit_radius=260.0, lod_scale=1.0 / 120.0)
    run_cached_sequence(w, range(6), 80, 45, dims=(120, 104, 96), pool=300, max_req=12, preload=2, macro=True,
                        lod_context=0.8)


def test_grid_path_sequence_lod_context():
    from tests.test_gpu_path import PATH, _compare_misses, grid_volumes
    from tests.test_gpu_parity import TOL, _compare_state
    from oracle import oracle as O
    from paper_2504_18001_amd import cinr
    dims = (37, 29, 23)
    w = configs.scaled(configs.SMALL, 48, 40, orbit_radius=60.0, lod_scale=1.0 / 30.0, ortho_extent=60.0)
    m, vol, mm = grid_volumes(dims, 8)
    gc = cinr.Cache(vol, 8, 3, 60, 12, miss_log_capacity=1 << 20, evict_log_capacity=1 << 14,
                    keep_request_counts=True)
    oc = O.OracleCache(m, brick=8, n_lods=3, pool_bricks=60, max_requests=12, log_misses=True)
    r = cinr.Renderer()
    tf = synth.tf_window(40, 255)
    for f in range(5):
        cam = w.camera(f, dims)
        img = r.render(vol, cam, tf, w.step, w.lod_scale, frame_index=f, seed=w.seed, samples_per_iter=4,
                       mode=cinr.CACHED, cache=gc, path=PATH, lod_context=0.9)
        st = r.last_stats()
        p = O.make_params(w.step, w.lod_scale, seed=w.seed, frame_index=f, samples_per_iter=4, mode=O.CACHED,
                          macro_cell=8, macro_minmax=mm, path=PATH, lod_context=0.9)
        ref, rst = oc.render(cam, tf, p)
        for k in ("rays", "samples", "hits", "fallbacks", "misses", "skipped", "requested", "selected", "evicted"):
            assert st[k] == rst[k], (f, k, st[k], rst[k])
        _compare_state(gc, oc, f, check_misses=False)
        _compare_misses(gc, oc, f)
        assert np.abs(img.cpu().numpy().astype(np.float64) - ref).max() <= TOL["f32"]
