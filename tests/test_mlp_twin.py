"""The FP64 MLP twin against central finite differences (its gradient pin)."""
import numpy as np

import mlp


def test_param_count():
    assert mlp.NPARAMS == 38657


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = mlp.init_params(1) * 0.5 + rng.normal(scale=0.01, size=mlp.NPARAMS)
    X = rng.normal(size=(64, 42))
    y = (rng.random(64) < 0.2).astype(float)
    loss, g = mlp.loss_and_grad(p, X, y, 5.0)
    idx = rng.choice(mlp.NPARAMS, 300, replace=False)
    idx = np.concatenate([idx, [mlp.NPARAMS - 1, 5376, 5376 + 128]])  # b4, b1[0], W2[0,0]
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.NPARAMS)
        e[i] = h
        fd = (mlp.loss_and_grad(p + e, X, y, 5.0)[0] - mlp.loss_and_grad(p - e, X, y, 5.0)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(g[i]), (i, fd, g[i])
