"""The learned part end to end at its full size: an INR (16 levels x 2, T =
2^20, 32-64-64-1) trained on the GPU for 2000 steps of 2^18 points (the last
200 at a tenth of the learning rate) on a 1024^3 turbulence-like field (512
Fourier modes, amplitude |k|^-5/3), judged
by PSNR over all 1024^3 lattice points against the explicit grid, and
rendered at 1080p against the explicit-grid source with the same cached
renderer.  The gain is measured against the untrained (random-init) INR and
against the equal-memory explicit baseline (256^3 box-downsampled grid,
trilinear upsampling, 64 MB like the INR's parameters).  The scope asks the
trained INR to beat both; on this band-limited field (modes up to |k| = 128,
exactly what a 256^3 grid resolves) it does not within 2000 steps, and that
comparison stays in the suite as a strict expected failure naming the
measured numbers."""
import json
import math

import numpy as np
import pytest
import torch

from paper_2504_18001_amd import configs, synth

pytestmark = pytest.mark.gpu

V = 1024
STEPS = 2000
ANNEAL_FROM = 1800


def psnr_lattice(vol, grid, chunk_z=16):
    n = grid.shape[0]
    ii = torch.arange(n, device="cuda", dtype=torch.float32)
    y, x = torch.meshgrid(ii, ii, indexing="ij")
    se = 0.0
    for z0 in range(0, n, chunk_z):
        zz = torch.arange(z0, z0 + chunk_z, device="cuda", dtype=torch.float32)
        pos = torch.stack([x[None].expand(chunk_z, n, n), y[None].expand(chunk_z, n, n),
                           zz[:, None, None].expand(chunk_z, n, n)], dim=-1).reshape(-1, 3).contiguous()
        v = vol.infer_points(pos, "f32").reshape(chunk_z, n, n)
        se += float(((v - grid[z0:z0 + chunk_z]) ** 2).double().sum())
    return 10.0 * math.log10(n ** 3 / se)


def psnr_downsampled(grid, factor=4):
    n = grid.shape[0]
    g = torch.nn.functional.avg_pool3d(grid[None, None], factor)
    m = n // factor
    se = 0.0
    slab = 64
    for z0 in range(0, n, slab):
        lo, hi = max(0, z0 // factor - 1), min(m, (z0 + slab) // factor + 1)
        up = torch.nn.functional.interpolate(g[:, :, lo:hi], size=((hi - lo) * factor, n, n), mode="trilinear",
                                             align_corners=False)[0, 0]
        up = up[z0 - lo * factor: z0 - lo * factor + slab]
        se += float(((up - grid[z0:z0 + slab]) ** 2).double().sum())
    return 10.0 * math.log10(n ** 3 / se)


def render_frames(vol, w, frames, dims):
    from paper_2504_18001_amd import cinr
    cs = w.cache
    cache = cinr.Cache(vol, cs.brick, cs.n_lods, cs.pool_bricks, 256, preload_period=cs.preload_period)
    r = cinr.Renderer()
    img = None
    for f in frames:
        img = r.render(vol, w.camera(f, dims), w.tf(f), w.step, w.lod_scale, frame_index=f, seed=w.seed,
                       ert_threshold=w.ert_threshold, samples_per_iter=w.samples_per_iter, mode=cinr.CACHED,
                       dtype="f32", cache=cache)
    torch.cuda.synchronize()
    return img


@pytest.fixture(scope="module")
def learned():
    from paper_2504_18001_amd import cinr
    arch = configs.ARCH_LEARN
    grid = synth.fourier_field(V, synth.fourier_modes(512, 128, seed=0), device="cuda")
    table, weights = synth.random_inr_params(arch, 0)
    vol = cinr.Volume(arch, table, weights, 1.0, 0.0)
    p_random = psnr_lattice(vol, grid)
    tr = cinr.Trainer(vol, batch=1 << 18, lr=1e-2, seed=0, dtype="bf16")
    loss = torch.empty(1, device="cuda")
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for s in range(STEPS):
        if s == ANNEAL_FROM:
            tr.set_lr(1e-3)  # the last tenth at a tenth of the rate
        tr.step(grid, s, loss)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / STEPS
    p_trained = psnr_lattice(vol, grid)
    p_grid256 = psnr_downsampled(grid)
    # 1080p renders of the trained INR and of the explicit grid, same cache decisions
    w = configs.scaled(configs.HD512, 1920, 1080, orbit_radius=2318.0, lod_scale=1.0 / 1600.0)
    gvol = cinr.GridVolume(grid)
    frames = range(0, 24)
    img_inr = render_frames(vol, w, frames, (V, V, V))
    img_grid = render_frames(gvol, w, frames, (V, V, V))
    mse = float(((img_inr - img_grid) ** 2).mean())
    p_render = 10.0 * math.log10(1.0 / max(mse, 1e-30))
    rep = {"psnr_random_init_db": round(p_random, 2), "psnr_trained_db": round(p_trained, 2),
           "psnr_grid256_equal_memory_db": round(p_grid256, 2), "render_1080p_psnr_vs_grid_db": round(p_render, 2),
           "train_ms_per_step": round(ms, 3), "final_batch_loss": loss.item()}
    print(json.dumps(rep))
    return rep


def test_trained_inr_gains_over_the_untrained_one_at_full_size(learned):
    assert learned["psnr_trained_db"] > learned["psnr_random_init_db"] + 30.0
    assert learned["psnr_trained_db"] > 45.0
    assert learned["render_1080p_psnr_vs_grid_db"] > 35.0


@pytest.mark.xfail(strict=True, reason="unmet: the trained INR reaches 52.2-52.5 dB over the 1024^3 lattice, the "
                                       "equal-memory 256^3 grid 61.0 dB")
def test_trained_inr_beats_the_equal_memory_grid(learned):
    assert learned["psnr_trained_db"] > learned["psnr_grid256_equal_memory_db"]
