#!/usr/bin/env python3
"""Frame rate of the cached INR renderer at 1080p (BF16 MLP) beside the
uncached FP32 INR renderer on the same GPU, and brick-decode throughput.

Workload (inr512_persp1080p): a 512^3 virtual volume defined by a seeded
random-init hash-grid INR (16 levels x 2 features, T = 2^19, growth 1.38,
MLP 32-64-64-1), rendered at 1920x1080 (perspective, 45 degree vertical FOV)
along a 60-frame orbit (6 degrees per frame, 20 degree elevation, ramp
transfer function for frames 0-29 of each loop, a seeded random one for
30-59); step 0.5 voxel, LoD distance scale 1/800, early ray termination at
0.999; cache of 16^3-sample bricks, 4 LoDs, 2 GiB FP32 pool (131072 slots),
up to 256 bricks requested and decoded per frame, pre-load of the coarsest
LoD (4 frames per LoD), macro-cells of side 16 built from the INR on the GPU.

A step is one whole frame of the hot path: ray generation, sampling through
the page tables, true-miss inference, compositing, the cache manager's
ranking and request selection, and brick decoding into the pool.  The cache
state evolves across steps exactly as in interactive use: the warm-up
frames fill it and the timed frames continue the same orbit.

Prints one JSON line.  Inputs are synthetic and seeded; the paper's datasets
are not used.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fps at 1080p (cached, BF16 MLP) vs uncached FP32 INR, PSNR≥45 dB; bricks/s"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes of the sampler: a served sample reads its page-table entry
# and 8 trilinear corners (36 B); a true miss probes the page tables (16 B
# budget for up to 4 LoDs); each marched ray reads and writes its colour
# (32 B), its sample index and its live-list entry (8 B)
BYTES_SERVED, BYTES_MISS, BYTES_RAY = 36, 16, 40
# HBM bytes per sampler launch measured with rocprofv3 (FETCH_SIZE and
# WRITE_SIZE scaled by a copy-kernel calibration); valid only while the
# sampler's sources are the ones that were profiled
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_march_inr512_1080p.json")


def measured_traffic():
    """HBM bytes per sampler launch from the committed profile, or None when
    the profiled sources have changed since (or no profile exists)."""
    import hashlib
    try:
        prof = json.load(open(TRAFFIC_PROFILE))
        h = hashlib.sha256()
        for rel in prof["sources"]:
            with open(os.path.join(ROOT, rel), "rb") as fh:
                h.update(fh.read())
    except (OSError, ValueError, KeyError):
        return None
    if h.hexdigest() != prof.get("sources_sha256"):
        return None
    return int(prof["traffic_bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_value_range(key):
    with open(os.path.join(ROOT, "tests", "golden", "value_ranges.json")) as f:
        vr = json.load(f)[key]
    return vr["value_scale"], vr["value_offset"]


def make_scene(w, dtype_decode="bf16"):
    import torch
    from paper_2504_18001_amd import cinr, synth
    table, weights = synth.random_inr_params(w.arch, w.inr_seed)
    s, o = load_value_range(f"inr512/{w.inr_seed}")
    base = cinr.Volume(w.arch, table, weights, s, o)
    mm = base.build_macrocells(w.macro_cell, "f32")
    vol = cinr.Volume(w.arch, base.table, base.weights, s, o, macrocells=mm, macro_cell=w.macro_cell)
    cams = [w.camera(f) for f in range(w.n_frames)]
    tfs = [torch.as_tensor(w.tf(f)).cuda() for f in range(w.n_frames)]
    return vol, cams, tfs


def new_cache(vol, w, pool_dtype="f32", pool_bricks=None, f16_lods=0, pool_bricks_f16=0, virtual_pt=False,
              max_requests=None):
    from paper_2504_18001_amd import cinr
    cs = w.cache
    return cinr.Cache(vol, cs.brick, cs.n_lods, pool_bricks or cs.pool_bricks, max_requests or cs.max_requests,
                      rank_window=cs.rank_window, ranking=cs.ranking, preload_period=cs.preload_period,
                      pool_dtype=pool_dtype, f16_lods=f16_lods, pool_bricks_f16=pool_bricks_f16,
                      virtual_page_table=virtual_pt)


def run_frames(r, vol, cams, tfs, w, frames, mode, dtype, cache, stats=None, out=None):
    from paper_2504_18001_amd import cinr
    img = None
    for i, f in enumerate(frames):
        img = r.render(vol, cams[f % w.n_frames], tfs[f % w.n_frames], w.step, w.lod_scale, frame_index=f,
                       seed=w.seed, ert_threshold=w.ert_threshold, samples_per_iter=w.samples_per_iter, mode=mode,
                       dtype=dtype, cache=cache, stats=None if stats is None else stats[i], out=out)
    return img


def psnr(a, b):
    mse = float(((a - b) ** 2).mean())
    return float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse)


def decode_throughput(vol, w, dtype, n_bricks, reps=5):
    import numpy as np
    import torch
    from paper_2504_18001_amd import synth
    cs = w.cache
    nb, _ = vol.geometry(cs.brick, cs.n_lods)
    reqs = torch.from_numpy(synth.random_requests(nb.tolist(), n_bricks, seed=11)).cuda()
    out = torch.empty((n_bricks, cs.brick, cs.brick, cs.brick), dtype=torch.float32, device="cuda")
    vol.decode_bricks(reqs, cs.brick, dtype, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        vol.decode_bricks(reqs, cs.brick, dtype, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return n_bricks / (ms * 1e-3), ms


def request_count_leg(vol, cams, tfs, w, Wm, K, dtype, n_req=40):
    """The headline window with the request list of Sec. 6.1's length (40
    bricks per frame): the cache fills more slowly, so more samples fall back
    to coarser LoDs."""
    import torch
    from paper_2504_18001_amd import cinr
    c = new_cache(vol, w, max_requests=n_req)
    r = cinr.Renderer()
    out = torch.empty((w.height, w.width, 4), dtype=torch.float32, device="cuda")
    st = torch.zeros((K, len(cinr.STAT_FIELDS)), dtype=torch.int64, device="cuda")
    run_frames(r, vol, cams, tfs, w, range(Wm), cinr.CACHED, dtype, c, out=out)
    torch.cuda.synchronize()
    vol.set_timing(True, march_only=True)
    t0 = time.perf_counter()
    run_frames(r, vol, cams, tfs, w, range(Wm, Wm + K), cinr.CACHED, dtype, c, stats=st, out=out)
    torch.cuda.synchronize()
    fps = K / (time.perf_counter() - t0)
    vol.set_timing(False)
    ms, n = vol.collect_timing()["march"]
    tot = st.sum(0).cpu().numpy()
    res = {"max_requests": n_req, "fps": round(fps, 2), "march_ms_per_launch": round(ms / max(n, 1), 4),
           "fallbacks_per_frame": int(tot[cinr.STAT_FIELDS.index("fallbacks")]) // K,
           "samples_per_frame": int(tot[cinr.STAT_FIELDS.index("samples")]) // K}
    del c
    return res


def virtual_pt_leg(vol, cams, tfs, w, Wm, K, dtype, ref_img):
    """The headline sequence through the two-level page table (a directory
    entry per 8^3 bricks, blocks of 512 entries): frame rate and sampler time
    against the flat table's, and the image, which must be identical."""
    import numpy as np
    import torch
    from paper_2504_18001_amd import cinr
    c = new_cache(vol, w, virtual_pt=True)
    r = cinr.Renderer()
    out = torch.empty((w.height, w.width, 4), dtype=torch.float32, device="cuda")
    run_frames(r, vol, cams, tfs, w, range(Wm), cinr.CACHED, dtype, c, out=out)
    torch.cuda.synchronize()
    vol.set_timing(True, march_only=True)
    t0 = time.perf_counter()
    run_frames(r, vol, cams, tfs, w, range(Wm, Wm + K), cinr.CACHED, dtype, c, out=out)
    torch.cuda.synchronize()
    fps = K / (time.perf_counter() - t0)
    vol.set_timing(False)
    ms, n = vol.collect_timing()["march"]
    st = c.dump(cinr.DUMP_PT_STATE)
    used = int((c.dump(cinr.DUMP_PT_DIRECTORY) >= 0).sum())
    res = {"fps": round(fps, 2), "march_ms_per_launch": round(ms / max(n, 1), 4),
           "image_equal_to_flat_table": bool(np.array_equal(ref_img, out.cpu().numpy())),
           "directory_entries": st["directory_per_volume"], "blocks_in_use": used,
           "block_pool": st["blocks"], "table_bytes_in_use": 4 * st["directory_per_volume"] + 2048 * used,
           "flat_table_bytes": 4 * c.n_keys}
    del c
    return res


def pool_f16_leg(vol, cams, tfs, w, Wm, K, dtype, ref_img):
    """The headline sequence over a binary16 pool: the same slot count (half
    the bytes) and the same bytes (twice the slots), against the FP32 pool;
    then LoD-dependent mixed precision with the same slot count, half of the
    slots binary16: LoDs 1 and up in binary16 (LoD 0 kept in binary32), and
    the reverse."""
    import torch
    from paper_2504_18001_amd import cinr
    P = w.cache.pool_bricks
    coarse = ((1 << w.cache.n_lods) - 1) & ~1
    res = {}
    for name, slots, mask in (("same_slots", P, 0), ("same_bytes", 2 * P, 0), ("mixed_lod0_f32", P, coarse),
                              ("mixed_lod0_f16", P, 1)):
        if mask:
            c = new_cache(vol, w, pool_bricks=slots, f16_lods=mask, pool_bricks_f16=slots // 2)
        else:
            c = new_cache(vol, w, pool_dtype="f16", pool_bricks=slots)
        r = cinr.Renderer()
        out = torch.empty((w.height, w.width, 4), dtype=torch.float32, device="cuda")
        st = torch.zeros((K, len(cinr.STAT_FIELDS)), dtype=torch.int64, device="cuda")
        run_frames(r, vol, cams, tfs, w, range(Wm), cinr.CACHED, dtype, c, out=out)
        torch.cuda.synchronize()
        vol.set_timing(True, march_only=True)
        t0 = time.perf_counter()
        run_frames(r, vol, cams, tfs, w, range(Wm, Wm + K), cinr.CACHED, dtype, c, stats=st, out=out)
        torch.cuda.synchronize()
        fps = K / (time.perf_counter() - t0)
        vol.set_timing(False)
        ms, n = vol.collect_timing()["march"]
        tot = st.sum(0).cpu().numpy()
        res[name] = {"fps": round(fps, 2), "pool_slots": slots,
                     "pool_gib": round(c.pool.numel() * c.pool.element_size() / 2 ** 30, 3),
                     "march_ms_per_launch": round(ms / max(n, 1), 4),
                     "true_misses_per_frame": int(tot[cinr.STAT_FIELDS.index("misses")]) // K,
                     "psnr_vs_f32_pool_db": round(psnr(ref_img, out.cpu().numpy()), 2)}
        if mask:
            res[name]["f16_lods"] = mask
            res[name]["binary16_slots"] = slots // 2
        del c
    return res


def lod_context_leg(vol, cams, tfs, w, Wm, K, dtype, laps=21):
    """The headline sequence with the context-aware LoD (macro-cell value
    ranges scale the LoD distance): fps, requests and misses per frame, and
    PSNR of the last frame against the uncached renderer (LoD 0 everywhere),
    both after the headline's warm-up and after `laps` orbits, when 40 bricks
    per frame have loaded every brick of the volume (the pool holds them all)."""
    import torch
    from paper_2504_18001_amd import cinr
    nst = len(cinr.STAT_FIELDS)
    last = Wm + K - 1  # the same orbit frame at every lap
    ru = cinr.Renderer()
    ref = ru.render(vol, cams[last % w.n_frames], tfs[last % w.n_frames], w.step, w.lod_scale, frame_index=last,
                    seed=w.seed, ert_threshold=w.ert_threshold, samples_per_iter=w.samples_per_iter,
                    mode=cinr.UNCACHED_DIRECT, dtype="f32").cpu().numpy()
    Wl = laps * w.n_frames
    res = {"converged_after_frames": Wl + Wm}
    for kappa in (0.0, 0.5, 1.0):
        c = new_cache(vol, w)
        r = cinr.Renderer()
        out = torch.empty((w.height, w.width, 4), dtype=torch.float32, device="cuda")
        st = torch.zeros((K, nst), dtype=torch.int64, device="cuda")

        def frames(rng, stats=None):
            for i, f in enumerate(rng):
                r.render(vol, cams[f % w.n_frames], tfs[f % w.n_frames], w.step, w.lod_scale, frame_index=f,
                         seed=w.seed, ert_threshold=w.ert_threshold, samples_per_iter=w.samples_per_iter,
                         mode=cinr.CACHED, dtype=dtype, cache=c, out=out, stats=None if stats is None else stats[i],
                         lod_context=kappa)

        def timed(first):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            frames(range(first, first + K), st)
            torch.cuda.synchronize()
            fps = K / (time.perf_counter() - t0)
            tot = dict(zip(cinr.STAT_FIELDS, st.sum(0).cpu().numpy().tolist()))
            return {"fps": round(fps, 2), "requested_per_frame": tot["requested"] // K,
                    "true_misses_per_frame": tot["misses"] // K, "fallbacks_per_frame": tot["fallbacks"] // K,
                    "psnr_vs_uncached_db": round(psnr(ref, out.cpu().numpy()), 2)}

        frames(range(Wm))
        early = timed(Wm)
        frames(range(Wm + K, Wl + Wm))
        late = timed(Wl + Wm)
        res[f"kappa_{kappa}"] = {"after_warmup": early, "converged": late}
        del c
    return res


def path_leg(vol, cams, tfs, w, Wm, K, dtype, K_unc, oracle=True):
    """Path tracing of the headline orbit (Woodcock delta tracking through the
    same sampler and cache): cached frames (the headline cache, bricks decoded
    in `dtype`) against uncached frames (every tentative collision inferred in
    FP32), as the two path-tracing columns of Table 1."""
    import torch
    from paper_2504_18001_amd import cinr, configs
    path = configs.PATH_HD512.as_dict()
    nst = len(cinr.STAT_FIELDS)

    def frames(r, c, rng, mode, dt, st=None, out=None):
        for i, f in enumerate(rng):
            r.render(vol, cams[f % w.n_frames], tfs[f % w.n_frames], w.step, w.lod_scale, frame_index=f, seed=w.seed,
                     samples_per_iter=w.samples_per_iter, mode=mode, dtype=dt, cache=c, out=out,
                     stats=None if st is None else st[i], path=path)

    def cached(pool_dtype):
        c = new_cache(vol, w, pool_dtype=pool_dtype)
        r = cinr.Renderer()
        out = torch.empty((w.height, w.width, 4), dtype=torch.float32, device="cuda")
        st = torch.zeros((K, nst), dtype=torch.int64, device="cuda")
        frames(r, c, range(Wm), cinr.CACHED, dtype, out=out)
        torch.cuda.synchronize()
        vol.set_timing(True, march_only=True)
        t0 = time.perf_counter()
        frames(r, c, range(Wm, Wm + K), cinr.CACHED, dtype, st, out)
        torch.cuda.synchronize()
        fps = K / (time.perf_counter() - t0)
        vol.set_timing(False)
        ms, n = vol.collect_timing()["march"]
        tot = {k: int(v) for k, v in zip(cinr.STAT_FIELDS, st.sum(0).cpu().numpy())}
        del c
        return fps, ms, n, tot, out

    fps, ms, n, tot, out = cached("f32")
    # the same paths over a binary16 pool: half the bytes per brick line for
    # the path tracer's incoherent lookups
    fps16, ms16, _, _, out16 = cached("f16")
    half = {"fps_cached": round(fps16, 2), "path_kernel_ms_per_frame": round(ms16 / K, 4),
            "psnr_vs_f32_pool_db": round(psnr(out.cpu().numpy(), out16.cpu().numpy()), 2)}
    ru = cinr.Renderer()
    outu = torch.empty_like(out)
    stu = torch.zeros((K_unc, nst), dtype=torch.int64, device="cuda")
    frames(ru, None, range(Wm, Wm + 1), cinr.UNCACHED_DIRECT, "f32", out=outu)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    frames(ru, None, range(Wm, Wm + K_unc), cinr.UNCACHED_DIRECT, "f32", stu, outu)
    torch.cuda.synchronize()
    fps_u = K_unc / (time.perf_counter() - t0)
    totu = {k: int(v) for k, v in zip(cinr.STAT_FIELDS, stu.sum(0).cpu().numpy())}
    res = {"params": path, "fps_cached": round(fps, 2), "fps_uncached_fp32": round(fps_u, 2),
           "speedup": round(fps / fps_u, 3),
           "lookups_per_frame": tot["samples"] // K, "true_misses_per_frame": tot["misses"] // K,
           "iterations_per_frame": round(tot["iterations"] / K, 2),
           "path_kernel_ms_per_frame": round(ms / K, 4), "path_launches_per_frame": round(n / K, 2),
           "binary16_pool": half,
           "uncached_inferred_per_frame": totu["misses"] // K_unc,
           "uncached_iterations_per_frame": round(totu["iterations"] / K_unc, 2)}
    if oracle:
        res["oracle"] = path_oracle(w, cams, tfs, Wm, path)
    return res


def path_oracle(w, cams, tfs, f, path):
    """The CPU oracle's uncached path tracer on every 4th pixel of every 4th
    row of frame f (1/16 of the pixels): pixels per second."""
    import numpy as np
    from oracle import oracle as O
    from paper_2504_18001_amd import synth
    table, weights = synth.random_inr_params(w.arch, w.inr_seed)
    s, o = load_value_range(f"inr512/{w.inr_seed}")
    m = O.OracleInr(w.arch, table, weights, s, o)
    jj, ii = np.meshgrid(np.arange(0, w.height, 4), np.arange(0, w.width, 4), indexing="ij")
    px = (jj * w.width + ii).reshape(-1).astype(np.int32)
    p = O.make_params(w.step, w.lod_scale, seed=w.seed, frame_index=f, samples_per_iter=w.samples_per_iter,
                      mode=O.UNCACHED_DIRECT, path=path)
    tf = tfs[f % w.n_frames].cpu().numpy()
    t0 = time.perf_counter()
    O.render_pixels(m, cams[f % w.n_frames], tf, p, px)
    dt = time.perf_counter() - t0
    return {"pixels_per_s": round(px.size / dt, 1), "cores": O.get_threads(), "kind": "oracle",
            "sample": f"uncached path tracing of 1/16 of the pixels of frame {f} ({px.size} pixels, {dt:.2f} s)"}


def multiview_leg(warmup, steps, dtype, oracle=True, waves=0):
    """Frames of 16 views of 4 INRs through one shared cache (one cache
    manager pass and one multi-INR decode launch per frame)."""
    import torch
    from paper_2504_18001_amd import cinr, configs, synth
    mv = configs.MULTIVIEW
    vols = []
    for i in range(mv.n_inrs):
        table, weights = synth.random_inr_params(mv.arch, i)
        s, o = load_value_range(f"inr512/{i}")
        base = cinr.Volume(mv.arch, table, weights, s, o)
        mm = base.build_macrocells(16, "f32")
        vols.append(cinr.Volume(mv.arch, base.table, base.weights, s, o, macrocells=mm, macro_cell=16))
    cs = mv.cache
    cache = cinr.Cache(vols, cs.brick, cs.n_lods, cs.pool_bricks, cs.max_requests, preload_period=cs.preload_period)
    r = cinr.MultiViewRenderer(mv.n_views)
    tfs = {k: torch.as_tensor(mv.tf(k)).cuda() for k in (0, 30)}
    outs = [torch.empty((mv.view_size(v), mv.view_size(v), 4), device="cuda") for v in range(mv.n_views)]

    def frame(f):
        views = [(vols[mv.view_inr(v)], mv.camera(v, f), tfs[0 if f % 60 < 30 else 30]) for v in range(mv.n_views)]
        r.render(cache, views, mv.step, mv.lod_scale, frame_index=f, seed=mv.seed, ert_threshold=mv.ert_threshold,
                 samples_per_iter=mv.samples_per_iter, dtype=dtype, outs=outs, waves_per_simd=waves)

    for f in range(warmup):
        frame(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(warmup, warmup + steps):
        frame(f)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the same frames again with stage timing (events around every stage)
    for v in vols:
        v.set_timing(True)
    for f in range(warmup + steps, warmup + 2 * steps):
        frame(f)
    torch.cuda.synchronize()
    stages = {}
    for v in vols:
        for k, (ms, n) in v.collect_timing().items():
            a = stages.setdefault(k, [0.0, 0])
            a[0] += ms
            a[1] += n
        v.set_timing(False)
    st = r.last_stats()
    pixels = sum(mv.view_size(v) ** 2 for v in range(mv.n_views))
    # the same sequence as captured frames (cinr_frame_graph) on a fresh cache;
    # the launch shapes were tuned by the frames above
    gcache = cinr.Cache(vols, cs.brick, cs.n_lods, cs.pool_bricks, cs.max_requests, preload_period=cs.preload_period)
    fg = cinr.FrameGraph(gcache, [(vols[mv.view_inr(v)], mv.camera(v, 0), tfs[0]) for v in range(mv.n_views)],
                         mv.step, mv.lod_scale, seed=mv.seed, ert_threshold=mv.ert_threshold,
                         samples_per_iter=mv.samples_per_iter, dtype=dtype, waves_per_simd=waves)

    def gframe(f):
        if f % 30 == 0:
            for t in fg.tfs:
                t.copy_(tfs[0 if f % 60 < 30 else 30])
        fg.render([mv.camera(v, f) for v in range(mv.n_views)], f)

    for f in range(warmup):
        gframe(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(warmup, warmup + steps):
        gframe(f)
    torch.cuda.synchronize()
    dtg = time.perf_counter() - t0
    n_graph, n_eager, n_tail = fg.counts()
    # decoding throughput of the shared cache: a prefill of bricks of all INRs in one launch
    K = cache.keys_per_volume
    fresh = cinr.Cache(vols, cs.brick, cs.n_lods, 8192, 256)
    import numpy as np
    keys = torch.from_numpy(np.concatenate([np.arange(256, dtype=np.int32) + i * K for i in range(mv.n_inrs)])).cuda()
    fresh.prefill(keys[:256], 0, dtype)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    fresh.prefill(keys[256:], 0, dtype)
    e1.record()
    torch.cuda.synchronize()
    dec = (keys.numel() - 256) / (e0.elapsed_time(e1) * 1e-3)
    cpu = multiview_oracle(mv) if oracle else None
    return {"workload": mv.name, "views": mv.n_views, "inrs": mv.n_inrs, "pixels_per_frame": pixels,
            "frames": steps, "frame_ms": round(dt / steps * 1e3, 4),
            "aggregate_view_fps": round(mv.n_views * steps / dt, 2),
            "pixels_per_s": round(pixels * steps / dt, 1),
            "stage_ms_per_frame": {k: round(v[0] / steps, 4) for k, v in stages.items()},
            "graph_frame_ms": round(dtg / steps * 1e3, 4),
            "graph_aggregate_view_fps": round(mv.n_views * steps / dtg, 2),
            "graph_frames_replayed_eager_tail": [n_graph, n_eager, n_tail],
            "requested_selected_last_frame": [st[0]["requested"], st[0]["selected"]],
            "multi_inr_decode_bricks_per_s": round(dec, 1),
            "cpu_oracle": cpu}


def multiview_oracle(mv):
    """The CPU oracle on frame 0 of the 16 views (cold shared cache) at 1/8 x
    1/8 of each view's pixels: view pixels per second of the oracle."""
    import numpy as np
    from oracle import oracle as O
    from paper_2504_18001_amd import synth
    ms = []
    for i in range(mv.n_inrs):
        table, weights = synth.random_inr_params(mv.arch, i)
        s, o = load_value_range(f"inr512/{i}")
        ms.append(O.OracleInr(mv.arch, table, weights, s, o))
    cs = mv.cache
    # one frame from a cold cache inserts at most max_requests bricks: a small
    # pool gives the same frame (the 32 GiB FP32 pool would be 64 GiB in FP64)
    oc = O.OracleCache(ms, brick=cs.brick, n_lods=cs.n_lods, pool_bricks=4096, max_requests=cs.max_requests,
                       preload_period=cs.preload_period)
    views, params, pixels = [], [], 0
    for v in range(mv.n_views):
        cam = mv.camera(v, 0)
        cam.width, cam.height = cam.width // 8, cam.height // 8
        pixels += cam.width * cam.height
        views.append((mv.view_inr(v), cam, mv.tf(0)))
        params.append(O.make_params(mv.step, mv.lod_scale, seed=mv.seed, frame_index=0, ert_threshold=mv.ert_threshold,
                                    samples_per_iter=mv.samples_per_iter))
    t0 = time.perf_counter()
    oc.render_views(views, params)
    dt = time.perf_counter() - t0
    return {"view_pixels_per_s": round(pixels / dt, 1), "cores": O.get_threads(), "kind": "oracle",
            "sample": f"frame 0 of the 16 views from a cold cache at 1/8 x 1/8 of their sizes ({pixels} pixels, "
                      f"{dt:.2f} s)"}


def training_leg(warmup, steps, oracle=True):
    """GPU training of the learned INR (16 levels x 2, T = 2^20, 32-64-64-1,
    BF16 MLP) on the 1024^3 Fourier field: 2^18 Philox points per step.
    Reports the step time and a breakdown (batch, gradients, Adam) with the
    Adam update's streamed bytes against HBM."""
    import torch
    from paper_2504_18001_amd import cinr, configs, synth
    arch = configs.ARCH_LEARN
    grid = synth.fourier_field(1024, synth.fourier_modes(512, 128, seed=0), device="cuda")
    table, weights = synth.random_inr_params(arch, 0)
    vol = cinr.Volume(arch, table, weights, 1.0, 0.0)
    batch = 1 << 18
    tr = cinr.Trainer(vol, batch=batch, lr=1e-2, seed=0, dtype="bf16")
    loss = torch.empty(1, device="cuda")
    for s in range(warmup):
        tr.step(grid, s, loss)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e[0].record()
    for s in range(warmup, warmup + steps):
        tr.step(grid, s, loss)
    e[1].record()
    torch.cuda.synchronize()
    step_ms = e[0].elapsed_time(e[1]) / steps

    def timed(fn, reps=10):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    u, t = tr.points(warmup + steps, grid)
    pts_ms = timed(lambda: tr.points(warmup + steps, grid))
    grad_ms = timed(lambda: tr.gradients(u, t))
    n = vol.table.numel() + vol.weights.numel()
    p_, m_, v_, g_ = (torch.zeros(n, device="cuda") for _ in range(4))
    adam_ms = timed(lambda: cinr.adam_update(p_, m_, v_, g_, 1, clear_grad=True))
    adam_bytes = 32 * n  # reads p, m, v, g; writes p, m, v and the cleared g
    adam_gbs = adam_bytes / (adam_ms * 1e-3) / 1e9
    cpu = None
    if oracle:
        # the CPU oracle's loss and gradients (FP64) on the first 4096 points of a batch
        import numpy as np
        from oracle import oracle as O
        m = O.OracleInr(arch, table, weights)
        un = u[:4096].double().cpu().numpy()
        tn = t[:4096].double().cpu().numpy()
        t0 = time.perf_counter()
        O.loss_grad(m, un, tn)
        dt = time.perf_counter() - t0
        cpu = {"points_per_s": round(4096 / dt, 1), "cores": O.get_threads(), "kind": "oracle",
               "sample": f"loss and all gradients of 4096 points of one batch in FP64 ({dt:.2f} s, with the "
                         f"16 M-entry table gradient)"}
    return {"workload": "learn1024_inr16x2_T2^20", "points_per_step": batch, "steps": steps,
            "step_ms": round(step_ms, 4), "points_per_s": round(batch / (step_ms * 1e-3), 1),
            "batch_ms": round(pts_ms, 4), "gradients_ms": round(grad_ms, 4), "adam_ms": round(adam_ms, 4),
            "adam_roofline": {"bound": "hbm", "achieved": round(adam_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(adam_gbs / HBM_PEAK_GBS, 4), "bytes_per_launch": adam_bytes,
                              "note": "4 arrays of 16.06 M floats (257 MB) updated back to back: part of them stays "
                                      "in the 256 MB Infinity Cache between launches, so the rate can pass the HBM "
                                      "peak"},
            "final_batch_loss": float(loss.item()), "cpu_oracle": cpu}


def cpu_baseline(w, budget_s):
    """The CPU oracle on a bounded sample of the same workload: cached frames
    from a cold cache at 1/8 x 1/8 of the resolution."""
    import numpy as np
    from oracle import oracle as O
    from paper_2504_18001_amd import synth
    table, weights = synth.random_inr_params(w.arch, w.inr_seed)
    s, o = load_value_range(f"inr512/{w.inr_seed}")
    m = O.OracleInr(w.arch, table, weights, s, o)
    cs = w.cache
    oc = O.OracleCache(m, brick=cs.brick, n_lods=cs.n_lods, pool_bricks=cs.pool_bricks, max_requests=cs.max_requests,
                       rank_window=cs.rank_window, ranking=cs.ranking, preload_period=cs.preload_period)
    W, H = w.width // 8, w.height // 8
    times = []
    t_start = time.perf_counter()
    f = 0
    while f < 12 and (time.perf_counter() - t_start) < budget_s:
        cam = w.camera(f)
        cam.width, cam.height = W, H
        p = O.make_params(w.step, w.lod_scale, seed=w.seed, frame_index=f, ert_threshold=w.ert_threshold,
                          samples_per_iter=w.samples_per_iter)
        t0 = time.perf_counter()
        oc.render(cam, w.tf(f), p)
        times.append(time.perf_counter() - t0)
        f += 1
    med = float(np.median(times))
    return {"value": 1.0 / (64.0 * med), "unit": "frames/s", "cores": O.get_threads(), "kind": "oracle",
            "sample": f"cached frames 0-{len(times) - 1} from a cold cache at {W}x{H} (1/64 of the pixels, no "
                      f"macro-cells); value = 1 / (64 x median frame time {med:.3f} s), i.e. the per-pixel work "
                      f"extrapolated to 1080p"}


def residency_at_frame_start(cache, frame):
    """Keys resident at the start of `frame`, the last frame rendered through
    `cache`: the slot owners now, without the keys its frame end inserted
    (the request list) and with the keys those insertions evicted."""
    import numpy as np
    from paper_2504_18001_amd import cinr
    owners = cache.dump(cinr.DUMP_SLOT_OWNER)
    inserted = set(cache.dump(cinr.DUMP_REQUEST_LIST).tolist())
    ev = cache.dump(cinr.DUMP_EVICTION_LOG).reshape(-1, 4)
    evicted = [int(r[2]) for r in ev if int(r[0]) == frame + 1 and int(r[2]) >= 0]
    keys = [int(k) for k in owners if k >= 0 and int(k) not in inserted] + evicted
    return np.array(sorted(keys), np.int32)


def oracle_image_check(w, keys, frame, img, n_pix=4096):
    """The last timed frame against the FP64 oracle: an oracle cache holding
    the GPU cache's residency at the start of that frame renders sampled
    pixels (its own early termination); max abs RGBA error and PSNR of the
    GPU's pixels against them."""
    import numpy as np
    from oracle import oracle as O
    from paper_2504_18001_amd import synth
    table, weights = synth.random_inr_params(w.arch, w.inr_seed)
    s, o = load_value_range(f"inr512/{w.inr_seed}")
    m = O.OracleInr(w.arch, table, weights, s, o)
    cs = w.cache
    oc = O.OracleCache(m, brick=cs.brick, n_lods=cs.n_lods, pool_bricks=cs.pool_bricks, max_requests=cs.max_requests,
                       rank_window=cs.rank_window, ranking=cs.ranking, preload_period=cs.preload_period)
    t0 = time.perf_counter()
    oc.prefill(keys, 0)
    mm = img["macrocells"]
    p = O.make_params(w.step, w.lod_scale, seed=w.seed, frame_index=frame, ert_threshold=w.ert_threshold,
                      samples_per_iter=w.samples_per_iter, macro_cell=w.macro_cell, macro_minmax=mm)
    px = np.random.default_rng(frame).choice(w.width * w.height, size=n_pix, replace=False).astype(np.int32)
    ref = O.render_pixels(m, w.camera(frame), w.tf(frame), p, px, cache=oc)
    got = img["rgba"].reshape(-1, 4)[px].astype(np.float64)
    d = np.abs(got - ref)
    mse = float((d ** 2).mean())
    return {"frame": frame, "pixels": n_pix, "resident_bricks": int(keys.size),
            "max_abs_rgba": float(d.max()), "psnr_db": round(10 * math.log10(1.0 / mse), 2) if mse > 0 else None,
            "oracle_s": round(time.perf_counter() - t0, 2)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dtype", default="bf16x3",
                    help="MLP arithmetic of the headline run: bf16x3 (BF16 MFMA with split operands), bf16, f16, f32")
    ap.add_argument("--precisions", default="f32,bf16,f16",
                    help="other MLP precisions run on the same cached sequence (own caches) for comparison")
    ap.add_argument("--uncached-steps", type=int, default=None)
    ap.add_argument("--decode-bricks", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-cached", action="store_true", help="skip the comparison precisions")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-multiview", action="store_true", help="skip the 16-view shared-cache leg")
    ap.add_argument("--no-adaptive", action="store_true", help="skip the adaptive sampling leg")
    ap.add_argument("--no-pool-f16", action="store_true", help="skip the binary16 pool leg")
    ap.add_argument("--no-virtual-pt", action="store_true", help="skip the two-level page table leg")
    ap.add_argument("--no-path", action="store_true", help="skip the path-tracing leg")
    ap.add_argument("--no-lod-context", action="store_true", help="skip the context-aware LoD leg")
    ap.add_argument("--path-uncached-steps", type=int, default=5)
    ap.add_argument("--multiview-steps", type=int, default=60)
    ap.add_argument("--no-training", action="store_true", help="skip the INR training leg")
    ap.add_argument("--training-steps", type=int, default=50)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain elementwise copy of this many MiB (y = x * 1) five times, to scale "
                         "hardware traffic counters, and exit")
    args = ap.parse_args()
    if args.calibrate_copy_mib:
        import torch
        n = args.calibrate_copy_mib * (1 << 20) // 4
        x = torch.rand(n, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "elementwise copy", "bytes_read": 4 * n, "bytes_written": 4 * n,
                          "launches": 5}))
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (--gpus {args.gpus} requested); multi-GPU sort-first "
              f"rendering is not part of it", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2504_18001_amd import cinr, configs

    torch.cuda.set_device(0)
    w = configs.HD512
    K, Wm = args.steps, args.warmup
    log(f"[bench] workload {w.name}: warmup {Wm} frames, timed {K} frames")
    vol, cams, tfs = make_scene(w)
    # decoding launch shape: the autotuner times every shape on a request list
    # of the frame's length (random bricks of every LoD), before the frames
    nb, _ = vol.geometry(w.cache.brick, w.cache.n_lods)
    from paper_2504_18001_amd import synth
    tune_reqs = torch.from_numpy(synth.random_requests(nb.tolist(), w.cache.max_requests, seed=12)).cuda()
    decode_shape, decode_shape_ms = vol.tune_decode(tune_reqs, w.cache.brick, args.dtype)
    log(f"[bench] decode shape {decode_shape}: {decode_shape_ms}")
    torch.cuda.synchronize()
    # sampler launch shape: the online tuner settles on a scratch cache over the
    # same orbit before the headline's frames, as the decoding shape above
    tcache, tr = new_cache(vol, w), cinr.Renderer()
    vol.set_timing(True, march_only=True)
    tune_frames = 0
    while cinr.tuned_launch(vol, w.width, w.height)[2] > 0 and tune_frames < 400:
        run_frames(tr, vol, cams, tfs, w, range(tune_frames, tune_frames + 10), cinr.CACHED, args.dtype, tcache)
        tune_frames += 10
    torch.cuda.synchronize()
    vol.set_timing(False)
    tune_launches = vol.collect_timing()["march"][1]
    del tcache, tr
    log(f"[bench] sampler launch shape {cinr.tuned_launch(vol, w.width, w.height)} after {tune_frames} frames")

    # --- cached, reduced-precision MLP: the headline run ---------------------
    cache = new_cache(vol, w)
    r = cinr.Renderer()
    out = torch.empty((w.height, w.width, 4), dtype=torch.float32, device="cuda")
    vol.set_timing(True)
    run_frames(r, vol, cams, tfs, w, range(Wm), cinr.CACHED, args.dtype, cache, out=out)
    torch.cuda.synchronize()
    vol.set_timing(False)
    warm_stages = vol.collect_timing()
    log("[bench] warm-up done")
    stats = torch.zeros((K, len(cinr.STAT_FIELDS)), dtype=torch.int64, device="cuda")
    # the timed region: HIP events bracket the sampler launches only
    vol.set_timing(True, march_only=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_frames(r, vol, cams, tfs, w, range(Wm, Wm + K), cinr.CACHED, args.dtype, cache, stats=stats, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    vol.set_timing(False)
    stages = vol.collect_timing()
    cached_img = out.clone()
    last_residency = residency_at_frame_start(cache, Wm + K - 1)
    # stage breakdown: the next orbit lap with every stage bracketed
    vol.set_timing(True)
    run_frames(r, vol, cams, tfs, w, range(Wm + K, Wm + 2 * K), cinr.CACHED, args.dtype, cache)
    torch.cuda.synchronize()
    vol.set_timing(False)
    all_stages = vol.collect_timing()
    fps = K / (t1 - t0)
    st = stats.cpu().numpy()
    tot = {k: int(st[:, i].sum()) for i, k in enumerate(cinr.STAT_FIELDS)}
    log(f"[bench] cached {args.dtype}: {fps:.1f} fps; stages {stages}; totals {tot}")

    # roofline of the dominant kernel (the sampler)
    march_ms, march_n = stages["march"]
    alg_bytes = (BYTES_SERVED * (tot["hits"] + tot["fallbacks"]) + BYTES_MISS * tot["misses"] +
                 BYTES_RAY * tot["rays"])
    achieved = alg_bytes / (march_ms * 1e-3) / 1e9 if march_ms > 0 else 0.0

    # --- the same cached sequence as captured frames (cinr_frame_graph) --------
    gcache = new_cache(vol, w)
    fg = cinr.FrameGraph(gcache, [(vol, cams[0], tfs[0])], w.step, w.lod_scale, seed=w.seed,
                         ert_threshold=w.ert_threshold, samples_per_iter=w.samples_per_iter, dtype=args.dtype)

    def graph_frames(frames):
        for f in frames:
            fg.tfs[0].copy_(tfs[f % w.n_frames])
            fg.render([cams[f % w.n_frames]], f)

    graph_frames(range(Wm))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    graph_frames(range(Wm, Wm + K))
    torch.cuda.synchronize()
    fps_graph = K / (time.perf_counter() - t0)
    graph_same = bool(torch.equal(fg.outs[0], cached_img))
    graph_counts = fg.counts()
    del fg, gcache
    log(f"[bench] captured frames {args.dtype}: {fps_graph:.1f} fps; image equal to eager: {graph_same}; "
        f"counts {graph_counts}")
    # the same with wavefront iterations queued on the device behind the first
    # march (true-miss frames of up to that many more iterations need no host
    # round trip); the steady state pays for the empty launches
    dev_iters = {}
    for k_dev in (2,):
        gcache = new_cache(vol, w)
        fg = cinr.FrameGraph(gcache, [(vol, cams[0], tfs[0])], w.step, w.lod_scale, seed=w.seed,
                             ert_threshold=w.ert_threshold, samples_per_iter=w.samples_per_iter, dtype=args.dtype)
        fg.set_device_iterations(k_dev)
        graph_frames(range(Wm))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        graph_frames(range(Wm, Wm + K))
        torch.cuda.synchronize()
        fps_k = K / (time.perf_counter() - t0)
        dev_iters[str(k_dev)] = {"fps": round(fps_k, 2), "image_equal": bool(torch.equal(fg.outs[0], cached_img)),
                                 "frames_graph_eager_tail": list(fg.counts())}
        del fg, gcache
    log(f"[bench] captured frames with device iterations: {dev_iters}")

    # --- adaptive sampling rate (Section 5.2) ----------------------------------
    # the same orbit with the TFs' opacity scaled by 0.1 (a semi-transparent
    # rendering, where the macro-cells' maximum opacities are low), fixed step
    # (E = 0) against steps of up to 2^E grid samples
    tfs_low = []
    for t in tfs:
        t2 = t.clone()
        t2[:, 3] *= 0.1
        tfs_low.append(t2)
    adaptive = {}
    ref_low = None
    for E in () if args.no_adaptive else (0, 1, 2, 3):
        c3 = new_cache(vol, w)
        r3 = cinr.Renderer()
        out3 = torch.empty_like(out)
        st3 = torch.zeros((K, len(cinr.STAT_FIELDS)), dtype=torch.int64, device="cuda")

        def adaptive_frames(frames, stats=None):
            for i, f in enumerate(frames):
                r3.render(vol, cams[f % w.n_frames], tfs_low[f % w.n_frames], w.step, w.lod_scale, frame_index=f,
                          seed=w.seed, ert_threshold=w.ert_threshold, samples_per_iter=w.samples_per_iter,
                          mode=cinr.CACHED, dtype=args.dtype, cache=c3, out=out3,
                          stats=None if stats is None else stats[i], adapt_max_exp=E)

        adaptive_frames(range(Wm))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        adaptive_frames(range(Wm, Wm + K), st3)
        torch.cuda.synchronize()
        fps_e = K / (time.perf_counter() - t0)
        img = out3.cpu().numpy()
        if E == 0:
            ref_low = img
        adaptive[f"E{E}"] = {"fps": round(fps_e, 2),
                             "samples_per_frame": int(st3[:, cinr.STAT_FIELDS.index("samples")].sum()) // K,
                             "psnr_vs_fixed_step_db": round(psnr(ref_low, img), 2)}
        del c3
    log(f"[bench] adaptive sampling rate (TF opacity x 0.1): {adaptive}")

    # --- the paper's request-list length ----------------------------------------
    req40 = None if w.cache.max_requests == 40 else request_count_leg(vol, cams, tfs, w, Wm, K, args.dtype)
    if req40:
        log(f"[bench] 40 requests per frame: {req40}")

    # --- two-level (virtualised) page table ------------------------------------
    vpt = None
    if not args.no_virtual_pt:
        vpt = virtual_pt_leg(vol, cams, tfs, w, Wm, K, args.dtype, cached_img.cpu().numpy())
        log(f"[bench] two-level page table: {vpt}")

    # --- binary16 brick pool (reduced-precision pool) -------------------------
    pool16 = None
    if not args.no_pool_f16:
        pool16 = pool_f16_leg(vol, cams, tfs, w, Wm, K, args.dtype, cached_img.cpu().numpy())
        log(f"[bench] binary16 pool: {pool16}")

    # --- context-aware LoD from the macro-cells' value ranges ------------------
    lodc = None
    if not args.no_lod_context:
        lodc = lod_context_leg(vol, cams, tfs, w, Wm, K, args.dtype)
        log(f"[bench] context-aware LoD: {lodc}")

    # --- path tracing through the same sampler and cache ----------------------
    pt = None
    if not args.no_path:
        pt = path_leg(vol, cams, tfs, w, Wm, K, args.dtype, args.path_uncached_steps,
                      oracle=not args.no_cpu_baseline)
        log(f"[bench] path tracing: {pt}")

    # --- uncached FP32 INR renderer on the same frames ------------------------
    KU = args.uncached_steps or K
    r2 = cinr.Renderer()
    out2 = torch.empty_like(out)
    run_frames(r2, vol, cams, tfs, w, range(Wm, Wm + 2), cinr.UNCACHED_DIRECT, "f32", None, out=out2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_frames(r2, vol, cams, tfs, w, range(Wm, Wm + KU), cinr.UNCACHED_DIRECT, "f32", None, out=out2)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fps_unc = KU / (t1 - t0)
    # same frame as the last cached one
    run_frames(r2, vol, cams, tfs, w, [Wm + K - 1], cinr.UNCACHED_DIRECT, "f32", None, out=out2)
    torch.cuda.synchronize()
    q_unc = psnr(cached_img.cpu().numpy(), out2.cpu().numpy())
    log(f"[bench] uncached f32: {fps_unc:.1f} fps; PSNR cached vs uncached {q_unc:.2f} dB")

    # --- the same cached sequence with the other MLP precisions -----------------
    other = {}
    if not args.no_fp32_cached:
        ref_img = cached_img.cpu().numpy()
        for dt in [d for d in args.precisions.split(",") if d and d != args.dtype]:
            c2 = new_cache(vol, w)
            r3 = cinr.Renderer()
            out3 = torch.empty_like(out)
            run_frames(r3, vol, cams, tfs, w, range(Wm), cinr.CACHED, dt, c2, out=out3)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run_frames(r3, vol, cams, tfs, w, range(Wm, Wm + K), cinr.CACHED, dt, c2, out=out3)
            torch.cuda.synchronize()
            other[dt] = {"fps": round(K / (time.perf_counter() - t0), 2),
                         "psnr_vs_headline_db": round(psnr(ref_img, out3.cpu().numpy()), 2)}
            del c2
            log(f"[bench] cached {dt}: {other[dt]}")

    # --- brick decoding throughput -------------------------------------------
    bps = {}
    for dt in dict.fromkeys([args.dtype, "bf16", "f16", "f32"]):
        bps[dt], _ = decode_throughput(vol, w, dt, args.decode_bricks)
    log(f"[bench] decode bricks/s {bps}")

    multi = None
    if not args.no_multiview:
        multi = multiview_leg(60, args.multiview_steps, args.dtype, oracle=not args.no_cpu_baseline)
        log(f"[bench] multiview {multi}")

    train = None
    if not args.no_training:
        train = training_leg(10, args.training_steps, oracle=not args.no_cpu_baseline)
        log(f"[bench] training {train}")

    cpu = None
    vs_oracle = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_budget)
        log(f"[bench] cpu baseline {cpu}")
        vs_oracle = oracle_image_check(w, last_residency, Wm + K - 1,
                                       {"rgba": cached_img.cpu().numpy(), "macrocells": vol.macrocells.cpu().numpy()})
        log(f"[bench] last timed frame against the FP64 oracle: {vs_oracle}")

    line = {
        "metric": METRIC,
        "value": round(fps, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": round(1000.0 / fps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded random-init INR; the paper's datasets are not used)",
        "config": {"workload": w.name, "width": w.width, "height": w.height, "volume": list(w.arch.dims),
                   "hash_grid": "16 levels x 2 features, T=2^19", "mlp": "32-64-64-1", "brick": w.cache.brick,
                   "n_lods": w.cache.n_lods, "pool_bricks": w.cache.pool_bricks,
                   "max_requests": w.cache.max_requests, "step": w.step, "ert": w.ert_threshold,
                   "orbit_frames": w.n_frames},
        "captured_frames_fps": round(fps_graph, 2),
        "captured_frames_image_equal": graph_same,
        "captured_frames_device_iterations": dev_iters,
        "uncached_fp32_fps": round(fps_unc, 2),
        "speedup_vs_uncached_fp32": round(fps / fps_unc, 3),
        "mlp_precision": {"bf16x3": "BF16 MFMA, operands split into hi+lo BF16, FP32 accumulation",
                          "bf16": "BF16 MFMA, FP32 accumulation", "f16": "FP16 MFMA, FP32 accumulation",
                          "f32": "FP32 MFMA"}.get(args.dtype, args.dtype),
        "cached_other_precisions": other,
        "adaptive_sampling": {"tf": "the orbit's TFs with opacity x 0.1", "by_max_exponent": adaptive},
        "binary16_pool": pool16,
        "two_level_page_table": vpt,
        "requests_40_per_frame": req40,
        "path_tracing": pt,
        "context_aware_lod": lodc,
        "bricks_per_s": {k: round(v, 1) for k, v in bps.items()},
        "decode_shape": {"chosen": {"parts_per_brick": decode_shape[0], "stage_kib": decode_shape[1]},
                         "ms_per_request_list": {f"{p}x{k}": round(t, 4) for (p, k), t in decode_shape_ms.items()},
                         "request_list": w.cache.max_requests, "dtype": args.dtype},
        "psnr_cached_vs_uncached_db": round(q_unc, 2),
        "vs_fp64_oracle": vs_oracle,
        "per_frame_in_timed_window": {k: round(tot[k] / K, 1) for k in ("rays", "samples", "hits", "fallbacks",
                                                                         "misses", "requested", "selected")},
        "stage_ms_per_frame": {k: round(v[0] / K, 4) for k, v in all_stages.items()},
        "frame_totals": tot,
        "roofline": {"kernel": "k_march", "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                     "algorithmic_bytes_per_launch": round(alg_bytes / max(march_n, 1)),
                     "launches": march_n, "avg_launch_ms": round(march_ms / max(march_n, 1), 5),
                     "launches_before_timed": tune_launches + warm_stages["march"][1],
                     "launch_shape": dict(zip(("pipe_depth", "xcd_bands", "trials_left", "waves_per_simd"),
                                              cinr.tuned_launch(vol, w.width, w.height))),
                     "launch_shape_tuned_over_frames": tune_frames},
        "multiview": multi,
        "training": train,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
