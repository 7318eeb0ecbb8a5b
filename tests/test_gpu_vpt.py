"""The two-level (virtualised) page table of Section 4.3.1 on the GPU.

A directory entry per block of 8^3 bricks of a LoD points to a block of 512
slot entries taken from a block pool.  The paper fixes what the table maps
(brick -> slot), not which block serves which directory entry, so the tests
compare what is unique and check that the rest is valid:
 - against the oracle's flat page table, bit for bit, with every other piece
   of cache state and the images (the flat view is resolved from the
   directory and the blocks);
 - against the GPU's own flat table on a reduced volume of the tera-scale
   shape (10240 x 7680 x 1536 scaled by 1/8, 6 LoDs);
 - the table's own invariants: a directory entry holds a block exactly when
   one of the block's bricks is mapped, a block's count is its mapped
   entries, blocks no entry holds are free and unmapped, none is shared.
"""
import numpy as np
import pytest
import torch

from paper_2504_18001_amd import configs, synth
from tests.helpers import inr_params, value_range
from tests.test_gpu_parity import run_cached_sequence

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_18001_amd import cinr
    cinr.lib()


def check_two_level_table(cache):
    """Invariants of the directory and block pool; returns the blocks in use."""
    from paper_2504_18001_amd import cinr
    d = cache.dump(cinr.DUMP_PT_DIRECTORY)
    blocks = cache.dump(cinr.DUMP_PT_BLOCKS)
    st = cache.dump(cinr.DUMP_PT_STATE)
    used = d[d >= 0]
    assert (d >= -1).all()
    assert len(np.unique(used)) == len(used), "a block serves two directory entries"
    assert (used < st["blocks"]).all()
    mapped = (blocks >= 0).sum(axis=1)
    assert (mapped[used] > 0).all(), "a directory entry holds an empty block"
    free = np.setdiff1d(np.arange(st["blocks"]), used)
    assert (mapped[free] == 0).all(), "a free block still maps bricks"
    assert st["free_blocks"] == len(free)
    owner = cache.dump(cinr.DUMP_SLOT_OWNER)
    assert mapped.sum() == (owner >= 0).sum(), "mapped entries differ from occupied slots"
    return len(used), st


def test_vpt_small_parity_with_eviction():
    # 64^3, 128x128, B = 8, 2 LoDs, 96 slots, 16 requests per frame: the pool
    # fills after 6 frames, and LRU eviction then empties and refills blocks
    caches = []
    run_cached_sequence(configs.SMALL, range(12), 128, 128, virtual_pt=True, caches=caches)
    n_used, st = check_two_level_table(caches[0])
    assert n_used > 0 and st["unmapped_for_want_of_a_block"] == 0


def test_vpt_512_arch_reduced_with_preload():
    w = configs.scaled(configs.HD512, 80, 45, orbit_radius=260.0, lod_scale=1.0 / 180.0)
    caches = []
    run_cached_sequence(w, range(8), 80, 45, dims=(120, 104, 96), pool=300, max_req=12, preload=2, virtual_pt=True,
                        caches=caches)
    check_two_level_table(caches[0])


def _tera_scene():
    from paper_2504_18001_amd import cinr
    arch = configs.ARCH_TERA
    t, w = inr_params(arch, 0)
    s, o = value_range(arch, 0)
    dims = (1280, 960, 192)
    return cinr.Volume(arch, t, w, s, o, dims=dims), dims


def test_vpt_tera_shape_against_flat_table():
    """The tera-scale shape at 1/8 (1280 x 960 x 192), B = 16, 6 LoDs, a
    300-slot pool with eviction, perspective frames over a zoom-in: images,
    statistics and every piece of cache state equal to the flat table's."""
    from paper_2504_18001_amd import cinr
    vol, dims = _tera_scene()
    kw = dict(brick=16, n_lods=6, pool_bricks=300, max_requests=40, preload_period=2, miss_log_capacity=1 << 20,
              evict_log_capacity=1 << 14, keep_request_counts=True)
    flat = cinr.Cache(vol, **kw)
    virt = cinr.Cache(vol, virtual_page_table=True, **kw)
    ra, rb = cinr.Renderer(), cinr.Renderer()
    centre = np.array([(d - 1) / 2.0 for d in dims])
    tf = synth.tf_ramp()
    for f in range(16):
        dist = 1800.0 * (0.8 ** f) + 60.0
        eye = centre + dist * np.array([0.35, 0.5, 0.79]) / np.linalg.norm([0.35, 0.5, 0.79])
        cam = synth.look_at(synth.PERSPECTIVE, eye, centre, 112, 80, 45.0)
        kw_r = dict(lod_scale=1.0 / 400.0, frame_index=f, seed=3, ert_threshold=0.999, samples_per_iter=16,
                    mode=cinr.CACHED, dtype="bf16x3", pipe_depth=1, xcd_bands=1)
        print(f"[vpt] tera frame {f}", flush=True)
        ia = ra.render(vol, cam, tf, 1.0, cache=flat, **kw_r)
        ib = rb.render(vol, cam, tf, 1.0, cache=virt, **kw_r)
        torch.cuda.synchronize()
        assert ra.last_stats() == rb.last_stats(), f
        assert torch.equal(ia, ib), f"frame {f}: max abs {(ia - ib).abs().max().item()}"
        for k in ("DUMP_PAGE_TABLE", "DUMP_SLOT_OWNER", "DUMP_LAST_USED", "DUMP_RANK", "DUMP_REQ_COUNT",
                  "DUMP_REQUEST_LIST", "DUMP_EVICTION_LOG"):
            a, b = flat.dump(getattr(cinr, k)), virt.dump(getattr(cinr, k))
            assert np.array_equal(a, b), (f, k)
    ev = virt.dump(cinr.DUMP_EVICTION_LOG)
    assert (ev[:, 2] >= 0).any(), "the sequence evicts"
    n_used, st = check_two_level_table(virt)
    print("[vpt] tera blocks in use", n_used, st, flush=True)
    # the directory is 512 times smaller than the flat table
    nb, off = vol.geometry(16, 6)
    assert st["directory_per_volume"] * 64 < int(off[-1])


def test_vpt_short_block_pool_leaves_bricks_unmapped():
    """A block pool below its bound (here 1 block, while the LoD-0 bricks
    the frames request span 8 directory entries): insertions that find no
    block are counted and leave their brick unmapped; the table stays
    consistent and frames keep running."""
    from paper_2504_18001_amd import cinr
    w = configs.SMALL
    t, wt = inr_params(w.arch, 0)
    s, o = value_range(w.arch, 0)
    vol = cinr.Volume(w.arch, t, wt, s, o)
    c = cinr.Cache(vol, 8, 2, 96, 16, virtual_page_table=True, pt_blocks=1)
    r = cinr.Renderer()
    for f in range(8):
        cam = w.camera(f)
        cam.width, cam.height = 64, 64
        # LoD distance scale 0: every sample at LoD 0, whose 9^3 bricks span 8 directory entries
        r.render(vol, cam, w.tf(f), w.step, 0.0, frame_index=f, seed=w.seed, samples_per_iter=8,
                 mode=cinr.CACHED, cache=c)
    torch.cuda.synchronize()
    st = c.dump(cinr.DUMP_PT_STATE)
    print("[vpt] short block pool", st, flush=True)
    assert st["blocks"] == 1 and st["unmapped_for_want_of_a_block"] > 0
    d = c.dump(cinr.DUMP_PT_DIRECTORY)
    assert (d >= 0).sum() <= 1
    ev = c.dump(cinr.DUMP_EVICTION_LOG)
    pt = c.dump(cinr.DUMP_PAGE_TABLE)
    owner = c.dump(cinr.DUMP_SLOT_OWNER)
    # every occupied slot's brick is either mapped to that slot or left unmapped
    occ = np.nonzero(owner >= 0)[0]
    assert all(pt[owner[s]] in (s, -1) for s in occ)
    assert (pt >= 0).sum() + st["unmapped_for_want_of_a_block"] >= len(occ) > (pt >= 0).sum()
    assert len(ev) >= len(occ)
    blocks = c.dump(cinr.DUMP_PT_BLOCKS)
    assert ((blocks >= 0).sum(axis=1)[d[d >= 0]] > 0).all()
