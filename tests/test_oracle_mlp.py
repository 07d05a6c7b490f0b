"""Pins of the FP64 network reference: its gradient against central finite differences."""

import numpy as np

from oracle import mlp


def _setup(width, B, seed):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-0.5, 0.5, mlp.n_params(width))
    X = rng.uniform(-1, 1, (B, mlp.D_IN))
    r = rng.normal(size=B)
    return p, X, r


def test_gradient_matches_finite_differences():
    """Every parameter of a width-8 net: the chain-rule gradient equals the central difference of
    the loss with the log-error targets frozen at the base point (that is the stated loss)."""
    width = 8
    p, X, r = _setup(width, 13, 0)
    Y, _ = mlp.forward(p, X, width)
    c = np.log(np.abs(Y[:, 0] - r) + mlp.EPS)
    _, g = mlp.loss_and_grad(p, X, r, width, c=c)
    h = 1e-6
    fd = np.empty_like(p)
    for k in range(p.size):
        e = np.zeros_like(p)
        e[k] = h
        fd[k] = (mlp.loss_and_grad(p + e, X, r, width, c=c)[0] - mlp.loss_and_grad(p - e, X, r, width, c=c)[0]) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))


def test_forward_special_cases():
    """Zero weights give the output bias; silu(0) = 0 and silu'(0) = 1/2."""
    width = 5
    p = np.zeros(mlp.n_params(width))
    p[-2:] = [0.25, -3.0]
    Y, _ = mlp.forward(p, np.ones((4, mlp.D_IN)), width)
    assert np.all(Y == [0.25, -3.0])
    assert mlp.silu(0.0) == 0.0 and mlp.silu_prime(0.0) == 0.5
    assert abs(mlp.silu(30.0) - 30.0) < 1e-10


def test_loss_is_zero_when_exact():
    """If y0 = r exactly and y1 = log(eps), the loss and its gradient vanish."""
    width = 4
    p = np.zeros(mlp.n_params(width))
    p[-1] = np.log(mlp.EPS)
    r = np.zeros(6)
    loss, g = mlp.loss_and_grad(p, np.zeros((6, mlp.D_IN)), r, width)
    assert loss == 0.0 and np.all(g == 0.0)
