"""GPU training of the INR (the learned part) against the CPU oracle.

Points and targets of a step, the loss and every gradient (MLP weights and
hash-table entries), and the Adam update are compared with the oracle's FP64
implementation; a short run checks that training fits a field."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2504_18001_amd import cinr, configs, synth
from paper_2504_18001_amd.synth import InrArch

pytestmark = pytest.mark.gpu

ADAM = dict(lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15)


def train_volume(arch, seed, dims=None):
    table, weights = synth.random_inr_params(arch, seed)
    return cinr.Volume(arch, table, weights, 1.0, 0.0, dims=dims), table, weights


def rel_err(got, ref):
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30))


def test_points_and_targets_match_oracle():
    vol, _, _ = train_volume(configs.ARCH_SMALL, 0)
    grid = synth.blob_volume((33, 29, 17), seed=2)  # [z][y][x] = 17 x 29 x 33
    n = 5000
    tr = cinr.Trainer(vol, batch=n, seed=0xABCDEF0123, dtype="f32")
    for step in (0, 7, 123456):
        u, t = tr.points(step, torch.from_numpy(grid).cuda())
        ru = O.train_points(0xABCDEF0123, step, n)
        np.testing.assert_array_equal(u.cpu().numpy().astype(np.float64), ru)
        rt = O.grid_trilinear(grid, ru)
        err = np.abs(t.cpu().numpy() - rt).max()
        print("step", step, "target max abs", err)
        assert err < 2e-6


ARCH_TINY_HASH = InrArch(dims=(64, 64, 64), n_levels=8, n_features=2, log2_table=10, n_min=4, growth=1.5,
                         widths=(16, 32, 32, 1))


@pytest.mark.parametrize("name,arch,dtype", [("small", configs.ARCH_SMALL, "f32"),
                                             ("small_tiny_table", ARCH_TINY_HASH, "f32"),
                                             ("inr512", configs.ARCH_512, "f32"),
                                             ("small", configs.ARCH_SMALL, "bf16"),
                                             ("inr512", configs.ARCH_512, "bf16")])
def test_gradients_match_oracle(name, arch, dtype):
    vol, table, weights = train_volume(arch, 3)
    m = O.OracleInr(arch, table, weights)
    rng = np.random.default_rng(11)
    n = 1000  # 31 full tiles of 32 points and a ragged tail
    u = rng.uniform(0.0, 1.0, size=(n, 3)).astype(np.float32)
    t = rng.uniform(0.0, 1.0, size=n).astype(np.float32)
    tr = cinr.Trainer(vol, batch=n, dtype=dtype)
    loss, gt, gw = tr.gradients(torch.from_numpy(u).cuda(), torch.from_numpy(t).cuda())
    rl, rgt, rgw = O.loss_grad(m, u.astype(np.float64), t.astype(np.float64))
    gt, gw = gt.cpu().numpy().astype(np.float64), gw.cpu().numpy().astype(np.float64)
    el, ew, et = abs(float(loss.item()) - rl) / rl, rel_err(gw, rgw), rel_err(gt, rgt)
    print(name, dtype, "loss", loss.item(), rl, "rel errors: loss", el, "weights", ew, "table", et)
    if dtype == "f32":
        assert el < 1e-5 and ew < 1e-4 and et < 1e-4
        # element-wise on the entries that matter
        assert np.abs(gw - rgw).max() < 1e-4 * np.abs(rgw).max()
        assert np.abs(gt - rgt).max() < 1e-4 * np.abs(rgt).max()
    else:
        # against the FP64 gradient: BF16 operands (8 significant bits) with FP32 accumulation
        assert el < 2e-2 and ew < 5e-2 and et < 8e-2
        cos_w = float(gw.ravel() @ rgw.ravel() / (np.linalg.norm(gw) * np.linalg.norm(rgw)))
        cos_t = float(gt.ravel() @ rgt.ravel() / (np.linalg.norm(gt) * np.linalg.norm(rgt)))
        assert cos_w > 0.998 and cos_t > 0.998
        # element by element against the oracle with the same BF16 operands: what
        # remains is FP32 against FP64 accumulation (about 1e-6 of an element's
        # terms) and operands whose FP32 and FP64 values round to neighbouring
        # BF16 values (one BF16 unit, 2^-8, of one term).  Bound per element:
        # 2^-8 |g| + 2^-11 max|g| of the tensor (weights of each layer, table);
        # measured: at most 1e-4 max|g| on both shapes.
        bl, bgt, bgw = O.loss_grad(m, u.astype(np.float64), t.astype(np.float64), bf16_operands=True)
        assert abs(float(loss.item()) - bl) <= 1e-4 * bl
        H, IN = arch.widths[1], arch.widths[0]
        cuts = [0, H * IN, H * IN + H * H, gw.size]
        for name_, got, ref in [("W%d" % (k + 1), gw[cuts[k]:cuts[k + 1]], bgw[cuts[k]:cuts[k + 1]]) for k in range(3)] + \
                [("table", gt.ravel(), bgt.ravel())]:
            d = np.abs(got - ref)
            bound = 2.0 ** -8 * np.abs(ref) + 2.0 ** -11 * np.abs(ref).max()
            print(name_, "max |d| / max |g|", d.max() / np.abs(ref).max(), "worst d / bound", (d / bound).max(),
                  "elements over 1e-4 max|g|", int((d > 1e-4 * np.abs(ref).max()).sum()), "of", d.size)
            assert (d <= bound).all(), name_


def test_gradients_of_no_points_are_zero():
    vol, _, _ = train_volume(configs.ARCH_SMALL, 0)
    tr = cinr.Trainer(vol, batch=16, dtype="f32")
    e = torch.empty((0, 3), device="cuda")
    loss, gt, gw = tr.gradients(e, torch.empty(0, device="cuda"))
    assert float(gt.abs().max()) == 0.0 and float(gw.abs().max()) == 0.0


def test_adam_matches_oracle():
    rng = np.random.default_rng(5)
    n = 10007
    p = rng.normal(size=n)
    m1 = np.zeros(n)
    m2 = np.zeros(n)
    P = torch.tensor(p, dtype=torch.float32, device="cuda")
    M = torch.zeros(n, dtype=torch.float32, device="cuda")
    Vv = torch.zeros(n, dtype=torch.float32, device="cuda")
    for step in range(1, 4):
        g = rng.normal(size=n).astype(np.float32)
        G = torch.from_numpy(g).cuda()
        cinr.adam_update(P, M, Vv, G, step, clear_grad=True, **ADAM)
        assert float(G.abs().max()) == 0.0
        O.lib().orc_adam_step(O._ptr(p), O._ptr(m1), O._ptr(m2), O._ptr(g.astype(np.float64)), n, step,
                              ADAM["lr"], ADAM["beta1"], ADAM["beta2"], ADAM["eps"])
    np.testing.assert_allclose(P.cpu().numpy(), p, rtol=0, atol=2e-6)
    np.testing.assert_allclose(M.cpu().numpy(), m1, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(Vv.cpu().numpy(), m2, rtol=1e-5, atol=1e-8)


def test_one_training_step_equals_points_gradients_and_adam():
    arch = configs.ARCH_SMALL
    grid = synth.blob_volume((64, 64, 64), seed=0)
    G = torch.from_numpy(grid).cuda()
    n = 4096
    # eps well above the rounding noise of the atomically summed table gradient,
    # so that entries with a vanishing gradient move by a vanishing amount
    adam = dict(ADAM, eps=1e-6)
    vol_a, table, weights = train_volume(arch, 1)
    tr = cinr.Trainer(vol_a, batch=n, seed=9, dtype="f32", **adam)
    loss = torch.empty(1, device="cuda")
    tr.step(G, 0, loss)
    # the same step through the separate entry points
    vol_b, _, _ = train_volume(arch, 1)
    tb = cinr.Trainer(vol_b, batch=n, seed=9, dtype="f32", **adam)
    u, t = tb.points(0, G)
    l2, gt, gw = tb.gradients(u, t)
    for prm, g in ((vol_b.table, gt), (vol_b.weights, gw)):
        cinr.adam_update(prm.view(-1), torch.zeros_like(g).view(-1), torch.zeros_like(g).view(-1), g.view(-1), 1,
                         **adam)
    torch.cuda.synchronize()
    assert abs(loss.item() - l2.item()) <= 1e-6 * abs(l2.item())
    # Adam's first step moves each parameter by at most lr; atomics may reorder the
    # table gradient, so compare with a tolerance far below lr
    assert float((vol_a.weights - vol_b.weights).abs().max()) < 1e-5
    assert float((vol_a.table - vol_b.table).abs().max()) < 1e-5


def lattice_psnr(vol, grid, dtype="f32"):
    V = grid.shape[0]
    ii = torch.arange(V, device="cuda", dtype=torch.float32)
    z, y, x = torch.meshgrid(ii, ii, ii, indexing="ij")
    pos = torch.stack([x, y, z], dim=-1).reshape(-1, 3).contiguous()
    v = vol.infer_points(pos, dtype).reshape(V, V, V)
    mse = float(((v - grid) ** 2).mean())
    return 10.0 * np.log10(1.0 / mse)


def test_training_fits_a_small_field():
    arch = configs.ARCH_SMALL
    V = 64
    grid = synth.fourier_field(V, synth.fourier_modes(64, 8, seed=4), device="cuda")
    vol, _, _ = train_volume(arch, 0)
    p0 = lattice_psnr(vol, grid)
    tr = cinr.Trainer(vol, batch=1 << 14, seed=1, dtype="bf16")
    loss = torch.empty(1, device="cuda")
    losses = []
    for s in range(500):
        tr.step(grid, s, loss)
        if s % 50 == 0 or s == 499:
            losses.append(loss.item())
    p1 = lattice_psnr(vol, grid)
    print("losses", losses, "PSNR random init", p0, "trained", p1)
    assert losses[-1] < 0.01 * losses[0]
    assert p1 > p0 + 20.0
