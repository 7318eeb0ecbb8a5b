"""Stage timing of frames on the GPU (cinr_set_timing, cinr_collect_timing).

The timing events only take timestamps: frames rendered with timing on, for
every stage or for the march launches only, are bit-identical to frames
rendered without it, and the launch counts follow the frames' wavefront
iterations.
"""
import numpy as np
import pytest
import torch

from paper_2504_18001_amd import configs
from tests.helpers import inr_params, value_range

pytestmark = pytest.mark.gpu

FRAMES = range(8)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_18001_amd import cinr
    cinr.lib()


def _frames(timing):
    """A cached sequence on the small workload from a fresh cache (8 frames of
    96x64, the first ones with true misses, so that every stage runs)."""
    from paper_2504_18001_amd import cinr
    w = configs.SMALL
    t, wts = inr_params(w.arch, 0)
    s, o = value_range(w.arch, 0)
    vol = cinr.Volume(w.arch, t, wts, s, o)
    cs = w.cache
    c = cinr.Cache(vol, cs.brick, cs.n_lods, cs.pool_bricks, cs.max_requests, preload_period=cs.preload_period)
    r = cinr.Renderer()
    if timing is not None:
        vol.set_timing(True, march_only=timing == "march")
    imgs, iters = [], 0
    for f in FRAMES:
        cam = w.camera(f)
        cam.width, cam.height = 96, 64
        img = r.render(vol, cam, w.tf(f), w.step, w.lod_scale, frame_index=f, seed=w.seed, ert_threshold=0.99,
                       samples_per_iter=w.samples_per_iter, mode=cinr.CACHED, dtype="f32", cache=c)
        imgs.append(img.cpu().numpy().copy())
        iters += r.last_stats()["iterations"]
    torch.cuda.synchronize()
    tm = vol.collect_timing() if timing is not None else None
    if tm is not None:  # a collection clears what it returned
        assert all(v == (0.0, 0) for v in vol.collect_timing().values())
    vol.set_timing(False)
    return imgs, iters, tm


def test_timing_leaves_frames_unchanged_and_counts_launches():
    ref, iters, _ = _frames(None)
    assert iters > len(FRAMES)  # some frames take several iterations
    for mode in ("all", "march"):
        imgs, it2, tm = _frames(mode)
        assert it2 == iters
        for f, (a, b) in enumerate(zip(ref, imgs)):
            assert np.array_equal(a, b), (mode, f)
        ms, n = tm["march"]
        assert n == iters and ms > 0.0, (mode, tm)
        for stage, (ms_s, n_s) in tm.items():
            assert ms_s >= 0.0 and n_s >= 0, (mode, stage)
        if mode == "march":
            assert all(tm[s][1] == 0 for s in tm if s != "march"), tm
        else:
            assert tm["setup"][1] == len(FRAMES), tm
            # later iterations infer the true misses and composite them
            assert tm["infer"][1] == iters - len(FRAMES) and tm["shade"][1] == iters - len(FRAMES), tm
            assert tm["cm"][1] >= 1 and tm["decode"][1] >= 1, tm
