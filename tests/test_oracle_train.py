"""Oracle pins for the learned part: analytic gradients of the MSE loss
through MLP and hash grid against central finite differences, and Adam
against torch.optim.Adam (float64, CPU) as a library cross-check."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2504_18001_amd.synth import InrArch, random_inr_params

TINY = InrArch(dims=(16, 16, 16), n_levels=3, n_features=2, log2_table=6, n_min=2, growth=1.7, widths=(6, 8, 8, 1))


def _loss(arch, table, weights, u, g):
    m = O.OracleInr(arch, table, weights)
    y = m.mlp(m.encode(u))
    return np.mean((y - g) ** 2)


def test_gradients_match_central_differences():
    table, weights = random_inr_params(TINY, 4)
    # table values are float32 in the descriptor; work with exactly representable perturbations
    rng = np.random.default_rng(0)
    u = rng.uniform(0, 1, size=(64, 3))
    g = rng.uniform(0, 1, size=64)
    m = O.OracleInr(TINY, table, weights)
    loss, gt, gw = O.loss_grad(m, u, g)
    assert loss == pytest.approx(_loss(TINY, table, weights, u, g), rel=1e-12)
    h = 2.0 ** -12
    # a sample of weights
    for i in rng.choice(weights.size, size=25, replace=False):
        wp, wm = weights.copy(), weights.copy()
        wp[i] += h
        wm[i] -= h
        fd = (_loss(TINY, table, wp, u, g) - _loss(TINY, table, wm, u, g)) / (2 * h)
        assert gw[i] == pytest.approx(fd, rel=1e-5, abs=1e-9)
    # a sample of table entries that received gradient (hashed and dense levels)
    nz = np.argwhere(np.abs(gt) > 1e-6)
    for r, c in nz[rng.choice(len(nz), size=25, replace=False)]:
        tp, tm = table.copy(), table.copy()
        tp[r, c] += h
        tm[r, c] -= h
        fd = (_loss(TINY, tp, weights, u, g) - _loss(TINY, tm, weights, u, g)) / (2 * h)
        assert gt[r, c] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_adam_matches_torch_optim_adam():
    rng = np.random.default_rng(1)
    n = 50
    p = rng.normal(size=n)
    m1 = np.zeros(n)
    m2 = np.zeros(n)
    tp = torch.tensor(p.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.99), eps=1e-15)
    for step in range(1, 6):
        g = rng.normal(size=n)
        O.lib().orc_adam_step(O._ptr(p), O._ptr(m1), O._ptr(m2), O._ptr(g), n, step, 1e-2, 0.9, 0.99, 1e-15)
        opt.zero_grad()
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)
