"""The binary16 brick pool on the GPU: decoded values are rounded to
binary16 (nearest, ties to even) when stored and interpolated in FP32.

- the FP16 pool is the FP32 pool rounded, bit for bit (same decoder, same
  requests), at half the bytes;
- prefilled FP16 bricks against the oracle's rounded decoding;
- cached sequences against the oracle's FP16-pool cache: images within the
  FP32 bound, statistics, page table, stamps, ranks, request lists, miss and
  eviction logs bit-exact; the generic sampler (B = 8) and the 16^3
  specialisation, the adaptive sampling rate, BF16 MLP decoding.
"""
import numpy as np
import pytest
import torch

from paper_2504_18001_amd import configs, synth
from tests.helpers import oracle_inr
from tests.test_gpu_parity import gpu_volume, run_cached_sequence

pytestmark = pytest.mark.gpu


def _prefill_pair(arch, B, n_lods, pool, dtype):
    from paper_2504_18001_amd import cinr
    vol = gpu_volume(arch, 0)
    c32 = cinr.Cache(vol, B, n_lods, pool, 8)
    c16 = cinr.Cache(vol, B, n_lods, pool, 8, pool_dtype="f16")
    rng = np.random.default_rng(4)
    keys = np.sort(rng.choice(c32.n_keys, size=min(pool, c32.n_keys), replace=False)).astype(np.int32)
    for c in (c32, c16):
        c.prefill(torch.from_numpy(keys).cuda(), stamp=0, dtype=dtype)
    return vol, c32, c16, keys


@pytest.mark.parametrize("arch,B,n_lods", [(configs.ARCH_SMALL, 8, 2), (configs.ARCH_512, 16, 4)])
@pytest.mark.parametrize("dtype", ["f32", "bf16x3"])
def test_f16_pool_is_the_rounded_f32_pool(arch, B, n_lods, dtype):
    from paper_2504_18001_amd import cinr
    _, c32, c16, keys = _prefill_pair(arch, B, n_lods, 200, dtype)
    assert c16.pool.dtype == torch.float16 and c16.pool.numel() == c32.pool.numel()
    p32 = c32.dump(cinr.DUMP_POOL)
    p16 = c16.dump(cinr.DUMP_POOL)
    assert p16.dtype == np.float16 and p16.nbytes * 2 == p32.nbytes
    np.testing.assert_array_equal(p16.view(np.uint16), p32.astype(np.float16).view(np.uint16))
    np.testing.assert_array_equal(c16.dump(cinr.DUMP_SLOT_OWNER), c32.dump(cinr.DUMP_SLOT_OWNER))


def test_f16_pool_against_oracle_decoding():
    from oracle import oracle as O
    from paper_2504_18001_amd import cinr
    arch = configs.ARCH_512
    B, nl, pool = 16, 4, 120
    _, _, c16, keys = _prefill_pair(arch, B, nl, pool, "f32")
    oc = O.OracleCache(oracle_inr(arch, 0), brick=B, n_lods=nl, pool_bricks=pool, max_requests=8, pool_f16=True)
    oc.prefill(keys, 0)
    np.testing.assert_array_equal(c16.dump(cinr.DUMP_SLOT_OWNER), oc.owner())
    got = c16.dump(cinr.DUMP_POOL).astype(np.float64)
    ref = oc.pool()
    # both round an INR value to binary16; the FP32 and FP64 decodings differ
    # by at most 1e-4, so the rounded values differ by that plus one quantum
    quantum = np.maximum(2.0 ** (np.floor(np.log2(np.maximum(np.abs(ref), 2.0 ** -24))) - 10), 2.0 ** -24)
    err = np.abs(got - ref)
    print("f16 pool vs oracle: max abs", err.max(), "equal", float((err == 0).mean()))
    assert np.all(err <= 1e-4 + quantum)
    assert (err == 0).mean() > 0.9


def test_cached_sequence_f16_pool():
    # 64^3, B = 8 (the generic sampler), 96 slots: eviction from frame 6 on
    w = configs.SMALL
    worst = run_cached_sequence(w, range(12), 72, 56, pool_dtype="f16")
    print("f16 pool worst", worst)


def test_cached_sequence_f16_pool_bf16_macrocells_adaptive():
    w = configs.SMALL
    run_cached_sequence(w, range(6), 64, 48, dtype="bf16", macro=True, adapt=2, pool_dtype="f16",
                        tf_fn=lambda f: synth.tf_window(60, 255))


def test_cached_sequence_f16_pool_512_arch():
    # the 512^3 architecture on a 120x104x96 volume: 16^3 bricks (the
    # sampler's 16^3 specialisation), 4 LoDs with pre-load, eviction
    w = configs.scaled(configs.HD512, 80, 45, orbit_radius=260.0, lod_scale=1.0 / 180.0)
    run_cached_sequence(w, range(8), 80, 45, dims=(120, 104, 96), pool=300, max_req=12, preload=2,
                        pool_dtype="f16")


def test_cached_sequence_f16_pool_512_arch_macrocells_adaptive():
    w = configs.scaled(configs.HD512, 80, 45, orbit_radius=260.0, lod_scale=1.0 / 180.0)
    run_cached_sequence(w, range(6), 80, 45, dims=(120, 104, 96), pool=300, max_req=12, preload=2, macro=True,
                        adapt=2, pool_dtype="f16", tf_fn=lambda f: synth.tf_window(40, 255))
