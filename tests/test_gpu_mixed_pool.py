"""GPU parity of the LoD-dependent mixed-precision pool (binary32 and
binary16 slot classes, each LoD stored in one class, eviction within the
class) against the oracle through the C ABI.

Decision-plane state (page table, owners, stamps, ranks, request counts,
request lists, miss lists, eviction logs) bit-exact; images within the
tolerance of the MLP precision.  Pool values: binary32 slots within the
INR-value tolerance of the oracle's FP64 decode; binary16 slots within that
plus one binary16 spacing (the oracle rounds its FP64 value, the decoder
its FP32 value, so a value near a rounding tie may land on either side).
"""
import numpy as np
import pytest
import torch

from paper_2504_18001_amd import configs
from tests.helpers import oracle_inr
from tests.test_gpu_parity import VTOL, gpu_volume, run_cached_sequence

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_18001_amd import cinr
    cinr.lib()


def _check_pool(gc, oc, split, dtype):
    from paper_2504_18001_amd import cinr
    owner = gc.dump(cinr.DUMP_SLOT_OWNER)
    np.testing.assert_array_equal(owner, oc.owner())
    with np.errstate(invalid="ignore"):  # free slots hold arbitrary bits
        got = gc.dump(cinr.DUMP_POOL).astype(np.float64)
    ref = oc.pool()
    used = owner >= 0
    assert used[:split].any() and used[split:].any()
    e32 = np.abs(got[:split][used[:split]] - ref[:split][used[:split]]).max()
    e16 = np.abs(got[split:][used[split:]] - ref[split:][used[split:]]).max()
    # binary16 slots hold binary16 numbers
    hi = got[split:][used[split:]]
    np.testing.assert_array_equal(hi.astype(np.float16).astype(np.float64), hi)
    print("pool error: binary32 class", e32, "binary16 class", e16)
    assert e32 <= VTOL[dtype] and e16 <= VTOL[dtype] + 2.0 ** -11


@pytest.mark.parametrize("mask,P,P16", [(0b01, 80, 30), (0b10, 60, 35)])
def test_cached_sequence_mixed_pool_small(mask, P, P16):
    # 64^3, B = 8, 2 LoDs, 24 requests per frame at a LoD scale that requests
    # both LoDs: both classes fill and evict
    w = configs.scaled(configs.SMALL, 40, 32, lod_scale=0.3 * configs.SMALL.lod_scale)
    caches = []
    run_cached_sequence(w, range(10), 40, 32, pool=P, max_req=24, f16_lods=mask, pool_bricks_f16=P16, caches=caches)
    gc, oc = caches
    from paper_2504_18001_amd import cinr
    ev = gc.dump(cinr.DUMP_EVICTION_LOG)
    evicted = ev[ev[:, 2] >= 0]
    assert (evicted[:, 1] < P - P16).any() and (evicted[:, 1] >= P - P16).any()
    _check_pool(gc, oc, P - P16, "f32")


def test_cached_sequence_mixed_pool_split_bf16_macrocells_adaptive():
    # split-BF16 MLP (most samples of these frames are true misses: plain
    # BF16 inference alone takes the images to the edge of their bound)
    w = configs.scaled(configs.SMALL, 48, 40, lod_scale=0.3 * configs.SMALL.lod_scale)
    caches = []
    run_cached_sequence(w, range(8), 48, 40, dtype="bf16x3", macro=True, adapt=2, pool=70, max_req=20,
                        f16_lods=0b10, pool_bricks_f16=30, caches=caches)
    _check_pool(*caches, 40, "bf16x3")


@pytest.mark.parametrize("mask", [0b0011, 0b1100])
def test_cached_sequence_mixed_pool_512_arch(mask):
    # the 512^3 architecture on a 120x104x96 virtual volume, B = 16 (the
    # sampler's 16^3-brick path), 4 LoDs, pre-load of the coarse LoDs
    w = configs.scaled(configs.HD512, 80, 45, orbit_radius=260.0, lod_scale=1.0 / 180.0)
    caches = []
    run_cached_sequence(w, range(8), 80, 45, dims=(120, 104, 96), pool=300, max_req=12, preload=2, f16_lods=mask,
                        pool_bricks_f16=150, caches=caches)
    gc, oc = caches
    from paper_2504_18001_amd import cinr
    owner = gc.dump(cinr.DUMP_SLOT_OWNER)
    assert (owner[:150] >= 0).any() and (owner[150:] >= 0).any()


def test_path_tracing_mixed_pool():
    # explicit-grid volume (brick and true-miss values are the same binary32
    # numbers on both sides): decisions bit-exact; the binary16 class holds
    # LoD 0
    from tests.test_gpu_path import run_grid_sequence
    worst, evicted = run_grid_sequence(range(8), S=4, pool=40, req=10, f16_lods=0b01, pool_bricks_f16=20)
    assert evicted > 0


def test_prefill_mixed_pool():
    from oracle import oracle as O
    from paper_2504_18001_amd import cinr
    arch = configs.ARCH_SMALL
    m = oracle_inr(arch, 0)
    vol = gpu_volume(arch, 0)
    gc = cinr.Cache(vol, 8, 2, 40, 8, f16_lods=0b10, pool_bricks_f16=12)
    oc = O.OracleCache(m, brick=8, n_lods=2, pool_bricks=40, max_requests=8, f16_lods=0b10, pool_bricks_f16=12)
    off = gc.key_offset
    # interleaved LoD-0 and LoD-1 keys: each class fills from its lowest slot
    keys = np.array([int(off[1]) + 3, 5, 9, int(off[1]) + 7, 11, int(off[1])], np.int32)
    gc.prefill(torch.from_numpy(keys).cuda())
    oc.prefill(keys)
    np.testing.assert_array_equal(gc.dump(cinr.DUMP_SLOT_OWNER), oc.owner())
    np.testing.assert_array_equal(gc.dump(cinr.DUMP_PAGE_TABLE), oc.page_table())
    _check_pool(gc, oc, 28, "f32")
