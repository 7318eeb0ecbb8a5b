"""Oracle pins for a cache shared by several volumes and frames of several
views: a single view reduces to the single-view frame, request counts add
up over the views of a frame, and bricks of volume v are volume v's decoded
at the local key."""
import numpy as np

from oracle import oracle as O
from paper_2504_18001_amd import configs, synth
from tests.helpers import oracle_inr

W = configs.SMALL


def _params(f, **kw):
    return O.make_params(W.step, W.lod_scale, seed=W.seed, frame_index=f, samples_per_iter=W.samples_per_iter, **kw)


def _cam(f, w=48, h=40):
    c = W.camera(f)
    c.width, c.height = w, h
    return c


def _state(oc):
    return (oc.page_table(), oc.owner(), oc.last_used(), oc.rank(), oc.req_count(), oc.request_list())


def test_one_view_equals_the_single_view_frame():
    m = oracle_inr(W.arch, 0)
    a = O.OracleCache(m, brick=8, n_lods=2, pool_bricks=40, max_requests=8)
    b = O.OracleCache([m], brick=8, n_lods=2, pool_bricks=40, max_requests=8)
    for f in range(5):
        ia, sa = a.render(_cam(f), W.tf(f), _params(f))
        (ib, sb), = b.render_views([(0, _cam(f), W.tf(f))], [_params(f)])
        np.testing.assert_array_equal(ia, ib)
        assert sa == sb
        for x, y in zip(_state(a), _state(b)):
            np.testing.assert_array_equal(x, y)


def test_request_counts_of_a_frame_add_over_its_views():
    m0, m1 = oracle_inr(W.arch, 0), oracle_inr(W.arch, 1)
    views = [(0, _cam(0), W.tf(0)), (1, _cam(2, 40, 32), W.tf(0)), (0, _cam(3, 32, 32), W.tf(0))]
    shared = O.OracleCache([m0, m1], brick=8, n_lods=2, pool_bricks=60, max_requests=0)
    res = shared.render_views(views, [_params(0)] * 3)
    total = shared.req_count()
    K = shared.n_keys // 2
    # each view alone on a fresh cache: counts land in its volume's key range
    acc = np.zeros_like(total)
    for i, (vi, cam, tf) in enumerate(views):
        c = O.OracleCache([m0, m1], brick=8, n_lods=2, pool_bricks=60, max_requests=0)
        (img, st), = c.render_views([(vi, cam, tf)], [_params(0)])
        np.testing.assert_array_equal(img, res[i][0])
        rc = c.req_count()
        assert rc[(1 - vi) * K:(2 - vi) * K].sum() == 0
        acc += rc
    np.testing.assert_array_equal(total, acc)


def test_bricks_of_each_volume_are_decoded_from_that_volume():
    m0, m1 = oracle_inr(W.arch, 0), oracle_inr(W.arch, 1)
    oc = O.OracleCache([m0, m1], brick=8, n_lods=2, pool_bricks=10, max_requests=4)
    K = oc.n_keys // 2
    keys = np.array([3, K + 3, K + 700, 11], np.int32)
    oc.prefill(keys, 0)
    pool = oc.pool()
    pt = oc.page_table()
    _, nb, off = O.lod_geometry(W.arch.dims, 8, 2)
    for key in keys:
        vol, local = divmod(int(key), K)
        L = 0 if local < off[1] else 1
        r = local - off[L]
        b = (r % nb[L][0], (r // nb[L][0]) % nb[L][1], r // (nb[L][0] * nb[L][1]))
        ref = (m0, m1)[vol].decode_bricks(np.array([[L, *b]], np.int32), 8, 2)[0]
        np.testing.assert_array_equal(pool[pt[key]], ref)
    # the same local key of the two volumes holds different bricks
    assert not np.array_equal(pool[pt[3]], pool[pt[K + 3]])
