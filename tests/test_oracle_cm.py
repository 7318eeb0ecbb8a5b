"""Oracle pins: the cache manager (Section 4.3.3 priority ranking, Sarton's
timestamp/key order) and LRU insertion with eviction (Figure 1 step (5)).
Every expected order below is derived by hand from the rules in the comments.

Ranking rule: a brick requested c times in frame f gets rank f + c - 1 when
first seen, otherwise rank + c; ranks are clamped to f + window.  The request
list is the top-n bricks requested in frame f by (rank desc, key asc).
Insertion: lowest free slot, else least (last_used, slot); the victim's
page-table entry is unmapped and its rank forgotten; new bricks are stamped f+1.
"""
import numpy as np

from oracle import oracle as O
from paper_2504_18001_amd import configs
from tests.helpers import oracle_inr

DIMS = (24, 24, 24)


def _cache(pool, n_req, ranking=1, window=1000):
    m = oracle_inr(configs.ARCH_SMALL, 0, dims=DIMS)
    return O.OracleCache(m, brick=5, n_lods=2, pool_bricks=pool, max_requests=n_req, rank_window=window,
                         ranking=ranking)


def test_priority_ranking_scenario():
    c = _cache(pool=8, n_req=1)
    # frame 0: counts (5, 1, 1) for keys (3, 7, 9) -> ranks 4, 0, 0 -> key 3 selected
    c.inject_requests([3, 7, 9], [5, 1, 1])
    st = c.end_frame(0)
    assert c.request_list().tolist() == [3] and st["requested"] == 3
    r = c.rank()
    assert (r[3], r[7], r[9]) == (4, 0, 0)
    # frame 1: counts (3, 1) for keys (7, 9) -> ranks 3, 1 -> key 7
    c.inject_requests([7, 9], [3, 1])
    c.end_frame(1)
    assert c.request_list().tolist() == [7]
    r = c.rank()
    assert (r[7], r[9]) == (3, 1)
    # frame 2: key 9 alone (rank 2) and a new key 11 seen 3 times (rank 2 + 2 = 4) -> 11
    c.inject_requests([9, 11], [1, 3])
    c.end_frame(2)
    assert c.request_list().tolist() == [11]
    # page table: 3 mapped at frame 1 start, 7 at frame 2, 11 at frame 3
    pt = c.page_table()
    assert pt[3] == 0 and pt[7] == 1 and pt[11] == 2 and pt[9] == -1
    assert c.last_used()[:3].tolist() == [1, 2, 3]


def test_ties_break_by_key():
    c = _cache(pool=8, n_req=2)
    c.inject_requests([20, 5, 13], [2, 2, 2])
    c.end_frame(4)
    assert c.request_list().tolist() == [5, 13]


def test_sarton_order_is_by_key():
    c = _cache(pool=8, n_req=2, ranking=0)
    c.inject_requests([12, 30, 4], [1, 9, 1])
    c.end_frame(0)
    assert c.request_list().tolist() == [4, 12]
    p = _cache(pool=8, n_req=2, ranking=1)
    p.inject_requests([12, 30, 4], [1, 9, 1])
    p.end_frame(0)
    assert p.request_list().tolist() == [30, 4]


def test_rank_clamp_above_timestamp():
    c = _cache(pool=8, n_req=0)
    c.inject_requests([6], [5000])
    c.end_frame(0)
    assert c.rank()[6] == 1000
    c.inject_requests([6], [10])
    c.end_frame(1)
    assert c.rank()[6] == 1001
    # one request per frame adds one per frame: the rank keeps pace with the
    # timestamp and the clamp (f + window) never binds
    c3 = _cache(pool=8, n_req=0, window=10)
    for f in range(50):
        c3.inject_requests([1], [1])
        c3.end_frame(f)
    assert c3.rank()[1] == 49  # 0 + 49 increments, never clamped (stays <= f + 10)


def test_requests_only_from_current_frame_are_eligible():
    c = _cache(pool=8, n_req=1)
    c.inject_requests([2, 3], [50, 1])
    c.end_frame(0)  # 2 selected
    c.inject_requests([4], [1])
    c.end_frame(1)
    # key 3 (rank 0) is not requested in frame 1, so 4 (rank 1) is taken
    assert c.request_list().tolist() == [4]


def test_lru_eviction_scenario():
    c = _cache(pool=2, n_req=1)
    c.inject_requests([10], [1])
    c.end_frame(0)  # 10 -> slot 0, stamp 1
    c.inject_requests([11], [1])
    c.end_frame(1)  # 11 -> slot 1, stamp 2
    assert c.owner().tolist() == [10, 11] and c.last_used().tolist() == [1, 2]
    # frame 2 reads slot 1 only; key 12 evicts the least recently used slot 0
    c.touch(1, 2)
    c.inject_requests([12], [1])
    c.end_frame(2)
    assert c.owner().tolist() == [12, 11] and c.last_used().tolist() == [3, 2]
    pt, rk = c.page_table(), c.rank()
    assert pt[10] == -1 and rk[10] == -1 and pt[12] == 0
    # frame 3 reads both slots (stamps equal) -> tie broken by the lower slot
    c.touch(0, 3)
    c.touch(1, 3)
    c.inject_requests([13], [1])
    c.end_frame(3)
    assert c.owner().tolist() == [13, 11]
    log = c.evict_log().tolist()
    assert log == [[1, 0, -1, 10], [2, 1, -1, 11], [3, 0, 10, 12], [4, 0, 12, 13]]


def test_batch_never_evicts_its_own_slots():
    c = _cache(pool=3, n_req=3)
    c.inject_requests([1, 2, 3], [3, 2, 1])
    c.end_frame(0)
    c.touch(0, 1)
    c.touch(1, 1)
    c.touch(2, 1)
    c.inject_requests([4, 5, 6], [3, 2, 1])
    c.end_frame(1)
    # all three old slots stamped 1: victims in slot order; new ones stamped 2
    assert c.owner().tolist() == [4, 5, 6] and c.last_used().tolist() == [2, 2, 2]


def test_request_list_bounded_by_pool():
    c = _cache(pool=2, n_req=5)
    c.inject_requests([1, 2, 3, 4], [4, 3, 2, 1])
    st = c.end_frame(0)
    assert c.request_list().tolist() == [1, 2] and st["selected"] == 2


def test_cache_state_invariants_over_a_sequence():
    # I5: hits + fallbacks + misses + skipped = samples;  I6: page table and
    # owner are inverse on mapped entries;  I7: occupancy <= pool.
    w = configs.SMALL
    m = oracle_inr(configs.ARCH_SMALL, 0)
    c = O.OracleCache(m, brick=8, n_lods=2, pool_bricks=40, max_requests=16, preload_period=1)
    for f in range(5):
        cam = w.camera(f)
        cam.width = cam.height = 24
        p = O.make_params(0.5, w.lod_scale, seed=3, frame_index=f, samples_per_iter=8)
        _, st = c.render(cam, w.tf(f), p)
        assert st["hits"] + st["fallbacks"] + st["misses"] + st["skipped"] == st["samples"]
        pt, own = c.page_table(), c.owner()
        mapped = np.nonzero(pt >= 0)[0]
        assert len(mapped) <= 40
        for k in mapped:
            assert own[pt[k]] == k
        for s, k in enumerate(own):
            if k >= 0:
                assert pt[k] == s
