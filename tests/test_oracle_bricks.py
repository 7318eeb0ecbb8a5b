"""Oracle pins: LoD lattice, bricks and brick decoding (Section 4.3.2), the
memory arithmetic of Section 6.3 and macro-cells (Section 5.2)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2504_18001_amd import configs, synth
from tests.helpers import coordinate_inr, oracle_inr


def test_literal_worked_example_origin():
    # Section 4.3.2: request (0,1,2) at LoD 1, side 40 -> origin (0, 79, 159).
    assert O.brick_origin_literal((0, 1, 2), 1, 40) == (0, 79, 159)


def test_brick_counts_of_named_configs():
    _, _, off = O.lod_geometry((64, 64, 64), 8, 2)
    assert off[-1] == 9 ** 3 + 5 ** 3 == 854
    _, _, off = O.lod_geometry((512, 512, 512), 16, 4)
    assert off[-1] == 35 ** 3 + 18 ** 3 + 9 ** 3 + 5 ** 3 == 49561
    _, nb, off = O.lod_geometry((10240, 7680, 1536), 16, 6)
    assert nb[0].tolist() == [683, 512, 103]
    assert off[-1] == 41223072


def test_decoded_sample_positions_follow_shared_sample_stride():
    # With an INR whose value is the normalised coordinate, decoding reveals
    # the voxel position of every stored sample.  Request (0,1,2) at LoD 1
    # with B = 40: stride 2, origin (0, 78, 156) (one shared sample per face),
    # each brick spanning (B-1)*2 = 78 voxels; positions clamp at V-1.
    V = (256, 256, 256)
    B = 40
    for axis in range(3):
        m = coordinate_inr(V, axis)
        br = m.decode_bricks(np.array([[1, 0, 1, 2]]), B, 3)[0]
        x = br * V[axis] - 0.5  # recover the coordinate
        line = {0: br[0, 0, :], 1: br[0, :, 0], 2: br[:, 0, 0]}[axis] * V[axis] - 0.5
        origin = (0, 78, 156)[axis]
        expect = np.minimum(origin + 2 * np.arange(B), V[axis] - 1)
        np.testing.assert_allclose(line, expect, atol=1e-9)
        assert x.shape == (B, B, B)
    # last brick along x at LoD 0 clamps to V-1
    m = coordinate_inr((100, 100, 100), 0)
    _, nb, _ = O.lod_geometry((100, 100, 100), 16, 1)
    br = m.decode_bricks(np.array([[0, nb[0, 0] - 1, 0, 0]]), 16, 1)[0]
    xs = br[0, 0, :] * 100 - 0.5
    start = (nb[0, 0] - 1) * 15
    np.testing.assert_allclose(xs, np.minimum(start + np.arange(16), 99), atol=1e-9)


def test_brick_coverage_doubles_per_lod():
    # Each brick spans (B-1) * 2^L voxels: 39, 78, 156 for B = 40.
    V = (400, 400, 400)
    m = coordinate_inr(V, 0)
    for L, span in [(0, 39), (1, 78), (2, 156)]:
        br = m.decode_bricks(np.array([[L, 0, 0, 0]]), 40, 3)[0]
        xs = br[0, 0, :] * 400 - 0.5
        assert xs[-1] - xs[0] == pytest.approx(span, abs=1e-9)


def test_neighbour_bricks_share_their_face():
    m = oracle_inr(configs.ARCH_SMALL, 0)
    B = 8
    reqs = np.array([[0, 2, 3, 4], [0, 3, 3, 4], [0, 2, 4, 4], [0, 2, 3, 5], [1, 1, 1, 1], [1, 2, 1, 1]])
    br = m.decode_bricks(reqs, B, 2)
    np.testing.assert_array_equal(br[0][:, :, B - 1], br[1][:, :, 0])
    np.testing.assert_array_equal(br[0][:, B - 1, :], br[2][:, 0, :])
    np.testing.assert_array_equal(br[0][B - 1, :, :], br[3][0, :, :])
    np.testing.assert_array_equal(br[4][:, :, B - 1], br[5][:, :, 0])


def test_decode_equals_values_at_lattice_positions():
    m = oracle_inr(configs.ARCH_SMALL, 0)
    B = 8
    req = np.array([[1, 4, 2, 0]])
    br = m.decode_bricks(req, B, 2)[0]
    i = np.arange(B)
    zz, yy, xx = np.meshgrid(i, i, i, indexing="ij")
    x = np.stack([(4 * 7 + xx) * 2, (2 * 7 + yy) * 2, (0 * 7 + zz) * 2], -1).reshape(-1, 3)
    x = np.minimum(x, 63).astype(np.float64)
    np.testing.assert_array_equal(br.reshape(-1), m.value(x))


def test_invalid_requests_rejected():
    m = oracle_inr(configs.ARCH_SMALL, 0)
    with pytest.raises(ValueError):
        m.decode_bricks(np.array([[2, 0, 0, 0]]), 8, 2)
    with pytest.raises(ValueError):
        m.decode_bricks(np.array([[1, 5, 0, 0]]), 8, 2)


def test_memory_arithmetic_of_section_6_3():
    # 30^3 bricks of 40^3 FP32 voxels: 1.728e9 voxels, just under 7 GB.
    vox = 30 ** 3 * 40 ** 3
    assert vox == 1_728_000_000
    assert vox * 4 == 6_912_000_000 < 7e9
    # request buffer of 40 bricks of 40^3 FP32 values: 40^4 * 4 B = 10.24 MB
    assert 40 * 40 ** 3 * 4 == 10_240_000
    # macro-cells of a 4096^3 volume, FP32 (min, max) per cell
    for N, mb in [(16, 134.2), (32, 16.8), (64, 2.1)]:
        cells = (4096 // N) ** 3
        assert cells * 8 / 1e6 == pytest.approx(mb, abs=0.05)
    assert (4096 // 16) ** 3 == pytest.approx(16.8e6, rel=0.01)


def test_macrocells_bound_lattice_values():
    # every lattice point lies inside the closed region of each cell that
    # contains it, so its value is within that cell's [min, max]
    m = oracle_inr(configs.ARCH_SMALL, 0)
    mm = m.macrocells(16)
    assert mm.shape == (4, 4, 4, 2)

    def cells(p):
        c = {min(p // 16, 3)}
        if p % 16 == 0 and p > 0:
            c.add(p // 16 - 1)
        return c

    rng = np.random.default_rng(0)
    x = rng.integers(0, 64, size=(500, 3))
    x[:50] = rng.integers(0, 5, size=(50, 3)) * 16 - (rng.integers(0, 5, size=(50, 3)) == 4)
    x = np.clip(x, 0, 63)
    v = m.value(x.astype(np.float64))
    for p, val in zip(x, v):
        for cz in cells(p[2]):
            for cy in cells(p[1]):
                for cx in cells(p[0]):
                    lo, hi = mm[cz, cy, cx]
                    assert lo - 1e-6 <= val <= hi + 1e-6


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_macrocells_of_a_coordinate_field_closed_form(axis):
    # v = (x_axis + 0.5) / V_axis: a cell's range along its axis is fixed by
    # the closed region [c N, min((c + 1) N, V - 1)] of the lattice, and does
    # not depend on the other two cell indices (cells are stored z, y, x)
    dims = (40, 37, 50)
    N = 16
    m = coordinate_inr(dims, axis)
    mm = m.macrocells(N)
    M = [(d + N - 1) // N for d in dims]
    assert mm.shape == (M[2], M[1], M[0], 2)
    V = dims[axis]
    c = np.arange(M[axis])
    lo = (c * N + 0.5) / V
    hi = (np.minimum((c + 1) * N, V - 1) + 0.5) / V
    shape = [1, 1, 1]
    shape[2 - axis] = M[axis]
    exp_lo = np.broadcast_to(lo.reshape(shape), mm.shape[:3])
    exp_hi = np.broadcast_to(hi.reshape(shape), mm.shape[:3])
    np.testing.assert_allclose(mm[..., 0], exp_lo, rtol=0, atol=2e-7)
    np.testing.assert_allclose(mm[..., 1], exp_hi, rtol=0, atol=2e-7)


def test_macrocell_flags_hand_cases():
    tf = synth.tf_ramp()
    tf[:100, 3] = 0.0
    mm = np.array([[0.1, 0.3], [0.1, 0.4], [0.0, 0.0], [0.9, 1.0]], np.float32)
    # rows [25, 77] all transparent; [25, 102] reaches row 100; [0,0]; [229, 255]
    assert O.macrocell_flags(mm, tf).tolist() == [0, 1, 0, 1]
