"""FP64 reference of the touching-pair surrogate's network (test infrastructure only).

The network maps 6 features to 2 outputs through two hidden layers of `width` units with the
SiLU activation silu(z) = z / (1 + e^-z):

    H1 = silu(X W1 + b1),  H2 = silu(H1 W2 + b2),  Y = H2 W3 + b3.

Parameters are one flat vector in the order W1 [6 x width] (row-major, input-major), b1, W2
[width x width], b2, W3 [width x 2], b3. The training loss of a batch with targets r is

    L = mean_i (y_i0 - r_i)^2 + w * mean_i (y_i1 - c_i)^2,   c_i = log(|y_i0 - r_i| + eps),

where c_i is treated as a constant (the second output learns the size of the first output's
miss). The gradient is written out by the chain rule, layer by layer.
"""

import numpy as np

D_IN, D_OUT = 6, 2
W_ERR, EPS = 0.1, 1e-5


def unpack(p, width):
    p = np.asarray(p, dtype=np.float64)
    shapes = [(D_IN, width), (width,), (width, width), (width,), (width, D_OUT), (D_OUT,)]
    out, at = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(p[at:at + n].reshape(s))
        at += n
    assert at == p.size
    return out


def n_params(width):
    return D_IN * width + width + width * width + width + width * D_OUT + D_OUT


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_prime(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p, X, width):
    W1, b1, W2, b2, W3, b3 = unpack(p, width)
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ W1 + b1
    H1 = silu(Z1)
    Z2 = H1 @ W2 + b2
    H2 = silu(Z2)
    return H2 @ W3 + b3, (X, Z1, H1, Z2, H2)


def loss_and_grad(p, X, r, width, c=None):
    """Loss and its gradient; c (the log-error targets) defaults to the value at p."""
    W1, b1, W2, b2, W3, b3 = unpack(p, width)
    Y, (X, Z1, H1, Z2, H2) = forward(p, X, width)
    r = np.asarray(r, dtype=np.float64)
    B = len(r)
    d = Y[:, 0] - r
    if c is None:
        c = np.log(np.abs(d) + EPS)
    e = Y[:, 1] - c
    loss = np.mean(d * d) + W_ERR * np.mean(e * e)
    dY = np.stack([2.0 * d / B, 2.0 * W_ERR * e / B], axis=1)
    gW3 = H2.T @ dY
    gb3 = dY.sum(axis=0)
    dZ2 = (dY @ W3.T) * silu_prime(Z2)
    gW2 = H1.T @ dZ2
    gb2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2.T) * silu_prime(Z1)
    gW1 = X.T @ dZ1
    gb1 = dZ1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g
