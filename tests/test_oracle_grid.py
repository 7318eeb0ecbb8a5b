"""Oracle pins for the explicit-grid value source (the learned part's
fallback and reference): samples at voxel centres, exact reproduction of
trilinear fields, clamping, bricks made of grid samples, and the uncached
image of a constant grid in closed form."""
import numpy as np

from oracle import oracle as O
from paper_2504_18001_amd import synth


def _grid_of(fn, dims):
    z, y, x = np.meshgrid(*[np.arange(d, dtype=np.float64) for d in dims[::-1]], indexing="ij")
    return fn(x, y, z).astype(np.float32)


def test_grid_values_at_samples_and_clamped_outside():
    g = np.random.default_rng(0).uniform(size=(5, 6, 7)).astype(np.float32)  # [z][y][x]
    m = O.OracleInr.from_grid(g)
    i = np.array([[0, 0, 0], [6, 5, 4], [3, 2, 1]], np.float64)
    np.testing.assert_array_equal(m.value(i), g[[0, 4, 1], [0, 5, 2], [0, 6, 3]].astype(np.float64))
    np.testing.assert_array_equal(m.value(np.array([[-3.0, -1.0, -9.0], [99.0, 99.0, 99.0]])), [g[0, 0, 0], g[4, 5, 6]])


def test_grid_values_reproduce_trilinear_fields():
    dims = (9, 7, 5)
    fn = lambda x, y, z: 0.1 + 0.03 * x + 0.02 * y + 0.01 * z + 0.001 * x * y * z  # stays inside [0, 1]
    m = O.OracleInr.from_grid(_grid_of(fn, dims))
    x = np.random.default_rng(1).uniform(size=(300, 3)) * (np.array(dims) - 1)
    np.testing.assert_allclose(m.value(x), fn(x[:, 0], x[:, 1], x[:, 2]), rtol=0, atol=1e-7)


def test_grid_bricks_hold_grid_samples():
    g = synth.blob_volume((20, 18, 16), seed=3)
    m = O.OracleInr.from_grid(g)
    B = 8
    out = m.decode_bricks(np.array([[0, 1, 0, 1], [1, 0, 1, 0]], np.int32), B, 2)
    # LoD 0, brick (1, 0, 1): samples x = 7..14, y = 0..7, z = 7..14 (stride B-1)
    np.testing.assert_array_equal(out[0], g[7:15, 0:8, 7:15].astype(np.float64))
    # LoD 1, brick (0, 1, 0): samples at 2*(0..7) in x and z, 2*(7..14) in y, clamped to V-1
    xs = np.minimum(2 * np.arange(8), 19)
    ys = np.minimum(2 * (7 + np.arange(8)), 17)
    zs = np.minimum(2 * np.arange(8), 15)
    np.testing.assert_array_equal(out[1], g[np.ix_(zs, ys, xs)].astype(np.float64))


def test_constant_grid_renders_the_closed_form():
    # every sample has value c: after n samples A = 1 - (1 - a')^n
    c = 0.5
    g = np.full((16, 16, 16), c, np.float32)
    m = O.OracleInr.from_grid(g)
    cam = synth.orbit_camera(synth.ORTHOGRAPHIC, (16, 16, 16), 40.0, 0.0, 0.0, 8, 8, ortho_w=8.0, ortho_h=8.0)
    tf = np.full((256, 4), 0.25, np.float32)
    p = O.make_params(0.5, 0.0, mode=O.UNCACHED_DIRECT)
    img, st = O.render_uncached(m, cam, tf, p)
    # central rays cross the full box along z: t in [0, 15], samples at k*0.5, k = 0..30
    n = 31
    ap = 1.0 - (1.0 - 0.25) ** 0.5
    A = 1.0 - (1.0 - ap) ** n
    np.testing.assert_allclose(img[4, 4, 3], A, rtol=0, atol=1e-12)
    np.testing.assert_allclose(img[4, 4, 0], 0.25 * A, rtol=0, atol=1e-12)
