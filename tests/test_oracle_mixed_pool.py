"""Oracle pins of the LoD-dependent mixed-precision pool (a direction Section 7
leaves open: encodings chosen per LoD).  The pool has a binary32 class of
slots [0, split) and a binary16 class [split, pool_bricks); the LoDs whose
bit is set in f16_lods are stored in the binary16 class (values rounded to
the nearest binary16 value, ties to even), the others in the binary32 class,
and a brick evicts only within its class.

- every slot holds a brick of its class's LoDs, and its values are the
  decode of its owner: exactly (binary32 class) or rounded by numpy's
  float64 -> float16 conversion (binary16 class);
- the per-class slot choice (the class's lowest free slot, else its least
  recently used slot by (last_used, slot) among slots not filled in the
  batch) against a brute-force replay of the request lists;
- special cases: when only LoD-0 bricks are ever requested (lod_scale 0),
  a pool whose binary16 class holds LoD 1 renders exactly as a one-class
  binary32 pool of the binary32 class's size, and a pool whose binary16
  class holds LoD 0 exactly as a one-class binary16 pool of the binary16
  class's size (slots shifted by split);
- invalid descriptions are rejected.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2504_18001_amd import configs
from tests.helpers import oracle_inr


def _key_lod_brick(off, nb, key):
    L = int(np.searchsorted(off, key, side="right") - 1)
    local = int(key - off[L])
    nbx, nby = int(nb[L][0]), int(nb[L][1])
    return L, (local % nbx, (local // nbx) % nby, local // (nbx * nby))


def _check_classes_and_values(c, m, B, n_lods, split, mask):
    _, nb, off = O.lod_geometry(m.dims, B, n_lods)
    owner, pool = c.owner(), c.pool()
    used = np.nonzero(owner >= 0)[0]
    reqs = []
    for s in used:
        L, b = _key_lod_brick(off, nb, owner[s])
        assert ((mask >> L) & 1) == (1 if s >= split else 0), (s, L)
        reqs.append([L, *b])
    ref = m.decode_bricks(np.asarray(reqs, np.int32), B, n_lods)
    for i, s in enumerate(used):
        want = ref[i].astype(np.float16).astype(np.float64) if s >= split else ref[i]
        np.testing.assert_array_equal(pool[s], want, err_msg=f"slot {s}")
    return len(used)


@pytest.mark.parametrize("mask,P,P16", [(0b01, 80, 30), (0b10, 60, 35)])
def test_rendered_classes_hold_their_lods(mask, P, P16):
    # 64^3, B = 8, 2 LoDs, 24 requests per frame, a LoD scale at which both
    # LoDs are requested: both classes fill and evict
    w = configs.SMALL
    m = oracle_inr(w.arch, 0)
    c = O.OracleCache(m, brick=8, n_lods=2, pool_bricks=P, max_requests=24, f16_lods=mask, pool_bricks_f16=P16)
    evicted = {0: 0, 1: 0}
    for f in range(10):
        cam = w.camera(f)
        cam.width, cam.height = 40, 32
        p = O.make_params(w.step, 0.3 * w.lod_scale, seed=w.seed, frame_index=f,
                          samples_per_iter=w.samples_per_iter, mode=O.CACHED, ert_threshold=2.0)
        c.render(cam, w.tf(f), p)
        _check_classes_and_values(c, m, 8, 2, P - P16, mask)
        for rec in c.evict_log():
            if rec[0] == f + 1 and rec[2] >= 0:
                evicted[int(rec[1] >= P - P16)] += 1
    assert evicted[0] > 0 and evicted[1] > 0, evicted


def _replay(owner, last_used, keys, key_class, split, stamp):
    """Brute force: each key in list order takes its class's lowest free slot,
    else the class slot with the smallest (last_used, slot) not filled in this
    batch."""
    filled = set()
    log = []
    for k in keys:
        rng = range(split, len(owner)) if key_class(k) else range(0, split)
        free = [s for s in rng if owner[s] < 0]
        if free:
            s = free[0]
        else:
            s = min((s for s in rng if s not in filled), key=lambda s: (last_used[s], s))
        log.append((stamp, s, owner[s], k))
        owner[s], last_used[s] = k, stamp
        filled.add(s)
    return log


def test_per_class_lru_against_brute_force():
    m = oracle_inr(configs.ARCH_SMALL, 0)
    B, nl, P, P16 = 8, 2, 20, 9
    split = P - P16
    c = O.OracleCache(m, brick=B, n_lods=nl, pool_bricks=P, max_requests=6, f16_lods=0b10, pool_bricks_f16=P16)
    _, nb, off = O.lod_geometry(m.dims, B, nl)
    key_class = lambda k: 1 if k >= off[1] else 0
    rng = np.random.default_rng(5)
    owner = [-1] * P
    last_used = [-1] * P
    n_checked = 0
    for f in range(40):
        # requests for unmapped keys of both LoDs, then reads of random slots
        pt = c.page_table()
        cand = np.nonzero(pt < 0)[0]
        keys = rng.choice(cand, size=8, replace=False)
        c.inject_requests(keys, rng.integers(1, 5, size=8))
        for s in rng.choice(P, size=5, replace=False):
            c.touch(int(s), f)
            last_used[s] = f
        n_log = len(c.evict_log())
        c.end_frame(f)
        want = _replay(owner, last_used, [int(k) for k in c.request_list()], key_class, split, f + 1)
        got = [tuple(int(x) for x in r) for r in c.evict_log()[n_log:]]
        assert got == want, f
        np.testing.assert_array_equal(c.owner(), owner)
        np.testing.assert_array_equal(c.last_used(), last_used)
        n_checked += sum(1 for r in want if r[2] >= 0)
    assert n_checked > 40  # evictions in both classes


def _lod0_sequence(cache, frames=8):
    w = configs.SMALL
    out = []
    for f in range(frames):
        cam = w.camera(f)
        cam.width, cam.height = 36, 28
        # lod_scale 0: every sample selects LoD 0, so only LoD-0 bricks are requested
        p = O.make_params(w.step, 0.0, seed=w.seed, frame_index=f, samples_per_iter=w.samples_per_iter,
                          mode=O.CACHED, ert_threshold=2.0)
        img, st = cache.render(cam, w.tf(f), p)
        out.append((img, st, cache.page_table(), cache.owner(), cache.evict_log()))
    return out


def test_unused_binary16_class_is_a_binary32_pool():
    m = oracle_inr(configs.ARCH_SMALL, 0)
    P32, P16 = 40, 16
    mixed = O.OracleCache(m, brick=8, n_lods=2, pool_bricks=P32 + P16, max_requests=12, f16_lods=0b10,
                          pool_bricks_f16=P16)
    plain = O.OracleCache(m, brick=8, n_lods=2, pool_bricks=P32, max_requests=12)
    evicted = 0
    for (ia, sa, pa, oa, la), (ib, sb, pb, ob, lb) in zip(_lod0_sequence(mixed), _lod0_sequence(plain)):
        np.testing.assert_array_equal(ia, ib)
        assert sa == sb
        np.testing.assert_array_equal(pa, pb)
        np.testing.assert_array_equal(oa[:P32], ob)
        assert np.all(oa[P32:] == -1)
        np.testing.assert_array_equal(la, lb)
        evicted += sa["evicted"]
    assert evicted > 0


def test_binary16_lod0_is_a_binary16_pool():
    m = oracle_inr(configs.ARCH_SMALL, 0)
    P32, P16 = 16, 40
    mixed = O.OracleCache(m, brick=8, n_lods=2, pool_bricks=P32 + P16, max_requests=12, f16_lods=0b01,
                          pool_bricks_f16=P16)
    half = O.OracleCache(m, brick=8, n_lods=2, pool_bricks=P16, max_requests=12, pool_f16=True)
    evicted = 0
    for (ia, sa, pa, oa, la), (ib, sb, pb, ob, lb) in zip(_lod0_sequence(mixed), _lod0_sequence(half)):
        np.testing.assert_array_equal(ia, ib)
        assert sa == sb
        np.testing.assert_array_equal(pa, np.where(pb >= 0, pb + P32, -1))
        assert np.all(oa[:P32] == -1)
        np.testing.assert_array_equal(oa[P32:], ob)
        shifted = lb.copy()
        shifted[:, 1] += P32
        np.testing.assert_array_equal(la, shifted)
        evicted += sa["evicted"]
    assert evicted > 0
    np.testing.assert_array_equal(mixed.pool()[P32:], half.pool())


def test_prefill_per_class():
    m = oracle_inr(configs.ARCH_SMALL, 0)
    _, nb, off = O.lod_geometry(m.dims, 8, 2)
    c = O.OracleCache(m, brick=8, n_lods=2, pool_bricks=12, max_requests=4, f16_lods=0b10, pool_bricks_f16=4)
    lod1 = np.arange(off[1], off[1] + 5, dtype=np.int32)
    with pytest.raises(ValueError):
        c.prefill(lod1)  # five LoD-1 bricks, four binary16 slots
    keys = np.concatenate([np.arange(0, 8, dtype=np.int32), lod1[:4]])
    c.prefill(keys)
    owner = c.owner()
    np.testing.assert_array_equal(owner, keys)  # both classes filled from their lowest slot, in order
    _check_classes_and_values(c, m, 8, 2, 8, 0b10)


@pytest.mark.parametrize("kw", [
    dict(f16_lods=0b10, pool_bricks_f16=8, pool_f16=True),   # the classes need a binary32 pool
    dict(f16_lods=0b11, pool_bricks_f16=8),                  # every LoD in binary16: a one-class pool
    dict(f16_lods=0b100, pool_bricks_f16=8),                 # LoD 2 does not exist
    dict(f16_lods=0b10, pool_bricks_f16=0),
    dict(f16_lods=0b10, pool_bricks_f16=20),                 # no binary32 slot left
    dict(f16_lods=0b10, pool_bricks_f16=3),                  # fewer slots than requests per frame
])
def test_invalid_mixed_descriptions(kw):
    m = oracle_inr(configs.ARCH_SMALL, 0)
    with pytest.raises(ValueError):
        O.OracleCache(m, brick=8, n_lods=2, pool_bricks=20, max_requests=4, **kw)
