"""The explicit-grid volume source on the GPU against the oracle's grid
source: point values, brick decoding, macro-cells and a cached frame
sequence with bit-exact cache state."""
import numpy as np
import pytest
import torch

from paper_2504_18001_amd import configs, synth
from tests.test_gpu_parity import TOL, _compare_state, _render_gpu

pytestmark = pytest.mark.gpu

DIMS = (37, 29, 23)  # ragged against bricks and macro-cells


def volumes(dims=DIMS, macro=0):
    from oracle import oracle as O
    from paper_2504_18001_amd import cinr
    g = synth.blob_volume(dims, seed=5)
    m = O.OracleInr.from_grid(g)
    mm = m.macrocells(macro) if macro else None
    vol = cinr.GridVolume(torch.from_numpy(g).cuda(), macrocells=torch.from_numpy(mm) if macro else None,
                          macro_cell=macro)
    return g, m, vol, mm


def test_grid_points_match_oracle():
    g, m, vol, _ = volumes()
    rng = np.random.default_rng(3)
    V = np.array(DIMS, np.float64)
    x = (rng.uniform(-0.2, 1.2, size=(3001, 3)) * (V - 1)).astype(np.float32)
    got = vol.infer_points(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = m.value(x.astype(np.float64))
    err = np.abs(got - ref).max()
    print("grid points max abs", err)
    assert err < 1e-6


def test_grid_bricks_and_macrocells_are_exact():
    g, m, vol, _ = volumes()
    nb, _ = vol.geometry(8, 3)
    reqs = synth.random_requests([tuple(r) for r in nb], 40, seed=1)
    got = vol.decode_bricks(torch.from_numpy(reqs).cuda(), 8).cpu().numpy()
    np.testing.assert_array_equal(got.astype(np.float64), m.decode_bricks(reqs, 8, 3))
    np.testing.assert_array_equal(vol.build_macrocells(8).cpu().numpy(), m.macrocells(8))


def test_grid_cached_sequence_parity():
    from oracle import oracle as O
    from paper_2504_18001_amd import cinr
    w = configs.scaled(configs.SMALL, 64, 48, orbit_radius=60.0, lod_scale=1.0 / 60.0, ortho_extent=60.0)
    g, m, vol, mm = volumes(macro=16)
    B, nl, pool, req = 8, 2, 40, 10
    gc = cinr.Cache(vol, B, nl, pool, req, miss_log_capacity=1 << 20, evict_log_capacity=1 << 14,
                    keep_request_counts=True)
    oc = O.OracleCache(m, brick=B, n_lods=nl, pool_bricks=pool, max_requests=req, log_misses=True)
    r = cinr.Renderer()
    tf = synth.tf_window(40, 255)
    for f in range(8):
        cam = w.camera(f, DIMS)
        img, st = _render_gpu(vol, cam, tf, w, f, cinr.CACHED, "f32", cache=gc, renderer=r)
        p = O.make_params(w.step, w.lod_scale, seed=w.seed, frame_index=f, samples_per_iter=w.samples_per_iter,
                          mode=O.CACHED, macro_cell=16, macro_minmax=mm)
        ref, rst = oc.render(cam, tf, p)
        err = np.abs(img - ref).max()
        print(f"grid frame {f}: err {err:.2e} gpu {st}", flush=True)
        for k in ("rays", "samples", "hits", "fallbacks", "misses", "skipped", "requested", "selected", "evicted"):
            assert st[k] == rst[k], (f, k, st[k], rst[k])
        _compare_state(gc, oc, f)
        assert err <= TOL["f32"]
