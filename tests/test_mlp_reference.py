"""The CPU reference network used to check the GPU gradients is itself checked
against central finite differences (FP64, no rounding)."""
import numpy as np

import mlp_reference as mr


def test_reference_gradient_vs_finite_differences():
    rng = np.random.default_rng(0)
    p = rng.normal(0, 0.3, 9217)
    X = rng.normal(size=(40, 12))
    y = rng.normal(size=40) * 3
    mean, std = np.zeros(12), np.ones(12)
    _, g, _ = mr.loss_and_grad(p, X, y, mean, std, 0.9, rounding=False)
    h = 1e-6
    for i in rng.choice(9217, 60, replace=False):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mr.loss_and_grad(pp, X, y, mean, std, 0.9, False)[0] -
              mr.loss_and_grad(pm, X, y, mean, std, 0.9, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-5 * abs(g[i]) + 1e-9, (i, fd, g[i])
