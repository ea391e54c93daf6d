"""The oracle MLP gradient is pinned by central finite differences (FP64)."""
import numpy as np

from oracle import mlp


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    n_in, width, n_out = 5, 7, 4
    npar = width * n_in + width + width * width + width + n_out * width + n_out
    theta = rng.standard_normal(npar) * 0.5
    X = rng.standard_normal((9, n_in))
    T = rng.standard_normal((9, n_out))
    loss, g = mlp.loss_grad(theta, X, T, n_in, width, n_out)
    h = 1e-6
    fd = np.empty(npar)
    for k in range(npar):
        e = np.zeros(npar)
        e[k] = h
        fd[k] = (mlp.loss_grad(theta + e, X, T, n_in, width, n_out)[0] -
                 mlp.loss_grad(theta - e, X, T, n_in, width, n_out)[0]) / (2 * h)
    assert np.abs(fd - g).max() < 1e-8 * max(1.0, np.abs(g).max())
    assert loss > 0
