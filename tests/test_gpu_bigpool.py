"""Pools of 4 GiB and more with 16^3 bricks: each brick's base address is
formed in 64 bits (below 4 GiB the sampler and the path tracer use 32-bit
byte offsets).  The same frame sequence runs against two caches: one whose
pool is under 4 GiB, and one of 4.3 GiB whose lowest 262,144 slots (exactly
4 GiB of binary32 bricks) hold prefilled bricks the frames never sample, so
that every brick the frames load sits past byte offset 2^32.  Images, the
sampled bricks' page-table entries and the slots' stamps must agree bit for
bit, slot numbers shifted by 262,144.

The frames sample LoD 1 only: a LoD distance scale of 10 puts every sample
at distance > 1 and the 2-LoD cache clamps it to the coarsest LoD, so the
prefilled LoD-0 bricks are never looked up, requested or evicted.
"""
import numpy as np
import pytest
import torch

from paper_2504_18001_amd import configs, synth
from tests.helpers import inr_params, value_range

pytestmark = pytest.mark.gpu

DIMS = (1201, 1201, 1201)  # 80^3 LoD-0 bricks and 40^3 LoD-1 bricks of 16^3 samples
B, NL = 16, 2
LOW = 1 << 18              # slots below byte offset 2^32 (16 KiB per brick)
FREE = 4096                # free slots behind them (no eviction in the sequence)
PATH = dict(density=0.004, light_dir=(0.48, 0.6, 0.64), light=(2.5, 2.5, 2.5), ambient=(0.3, 0.35, 0.4),
            max_bounces=2, spp=1, seed=23)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_18001_amd import cinr
    cinr.lib()


@pytest.fixture(scope="module")
def volume():
    from paper_2504_18001_amd import cinr
    arch = configs.ARCH_SMALL
    t, w = inr_params(arch, 0)
    s, o = value_range(arch, 0)
    return cinr.Volume(arch, t, w, s, o, dims=DIMS)


def _camera(f, n=96):
    ext = DIMS[0] * 1.8
    return synth.orbit_camera(synth.ORTHOGRAPHIC, DIMS, 2200.0, 10.0 + 7.0 * f, 15.0, n, n, 45.0, ext, ext)


def _sequence(vol, path, frames=4):
    from paper_2504_18001_amd import cinr
    small = cinr.Cache(vol, B, NL, FREE, 64)
    big = cinr.Cache(vol, B, NL, LOW + FREE, 64)
    nb, off = vol.geometry(B, NL)
    assert off[1] >= LOW  # enough LoD-0 keys to fill the low slots
    big.prefill(torch.arange(LOW, dtype=torch.int32, device="cuda"), stamp=0, dtype="f32")
    torch.cuda.synchronize()
    owner = big.dump(cinr.DUMP_SLOT_OWNER)
    assert np.array_equal(owner[:LOW], np.arange(LOW)) and (owner[LOW:] == -1).all()
    ra, rb = cinr.Renderer(), cinr.Renderer()
    tf = synth.tf_ramp()
    kw = dict(lod_scale=10.0, seed=5, ert_threshold=0.999 if path is None else 2.0, samples_per_iter=8,
              mode=cinr.CACHED, dtype="f32", path=path, pipe_depth=1, xcd_bands=1)
    loaded = 0
    for f in range(frames):
        cam = _camera(f)
        print(f"[bigpool] frame {f} path {path is not None}", flush=True)
        ia = ra.render(vol, cam, tf, 1.0, frame_index=f, cache=small, **kw)
        ib = rb.render(vol, cam, tf, 1.0, frame_index=f, cache=big, **kw)
        torch.cuda.synchronize()
        sa, sb = ra.last_stats(), rb.last_stats()
        assert sa == sb, (f, sa, sb)
        assert torch.equal(ia, ib), f"frame {f}: max abs {(ia - ib).abs().max().item()}"
        pa, pb = small.dump(cinr.DUMP_PAGE_TABLE), big.dump(cinr.DUMP_PAGE_TABLE)
        lod1 = slice(int(off[1]), int(off[2]))
        assert np.array_equal(np.where(pa[lod1] >= 0, pa[lod1] + LOW, -1), pb[lod1])
        assert np.array_equal(pb[:LOW], np.arange(LOW))  # the prefilled bricks stay where they are
        ua, ub = small.dump(cinr.DUMP_LAST_USED), big.dump(cinr.DUMP_LAST_USED)
        assert np.array_equal(ua, ub[LOW:])
        assert (ub[:LOW] == 0).all()  # never stamped by a frame
        loaded = int((pa[lod1] >= 0).sum())
        if f > 0:
            assert sa["hits"] > 0  # frames after the first sample bricks past 4 GiB
    assert loaded > 0


def test_big_pool_ray_marching(volume):
    _sequence(volume, None)


def test_big_pool_path_tracing(volume):
    _sequence(volume, PATH)
