"""FP64 reference of the coarse-stencil surrogate network (a project
addition; no passage of the paper defines it).

Architecture: 3 inputs -> 64 -> 64 -> n_out outputs, SiLU activations,
three affine layers.  Inputs are standardised (eta_c = h_c k, order p,
damping ratio); the outputs are the standardised y_m = log(max(-e_m, 0) +
1e-13) where e_m is the relative fine dispersion error (r_m / kh - 1): in 2-D
(n_out = 2) at the QSFEM directions t_1 = pi/16, t_2 = 3 pi/16, in 3-D
(n_out = 3) along the three directions of the 27-point fit.  Loss: mean
squared error over samples and outputs.  Optimiser: Adam (Kingma & Ba 2015)
with bias correction.

Parameter layout (flat, the order the device code uses):
  W1 (64 x 3, row-major), b1 (64), W2 (64 x 64), b2 (64), W3 (n_out x 64), b3 (n_out).
"""
from __future__ import annotations

import numpy as np

N_IN, WIDTH, N_OUT = 3, 64, 2
E_FLOOR = 1e-13


def shapes(n_out: int = N_OUT):
    return [(WIDTH, N_IN), (WIDTH,), (WIDTH, WIDTH), (WIDTH,), (n_out, WIDTH), (n_out,)]


def n_params(n_out: int = N_OUT) -> int:
    return sum(int(np.prod(s)) for s in shapes(n_out))


N_PARAMS = n_params(N_OUT)


def n_out_of(theta) -> int:
    """Number of outputs of a flat parameter vector."""
    n_out = (len(theta) - n_params(0)) // (WIDTH + 1)
    assert n_params(n_out) == len(theta)
    return n_out


def unpack(theta: np.ndarray):
    out, o = [], 0
    for s in shapes(n_out_of(theta)):
        n = int(np.prod(s))
        out.append(theta[o:o + n].reshape(s))
        o += n
    return out


def silu(a):
    return a / (1.0 + np.exp(-a))


def dsilu(a):
    s = 1.0 / (1.0 + np.exp(-a))
    return s * (1.0 + a * (1.0 - s))


def forward(theta, x):
    """x: (n, 3) standardised inputs -> (n, n_out) outputs and the cache."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    a1 = x @ W1.T + b1
    h1 = silu(a1)
    a2 = h1 @ W2.T + b2
    h2 = silu(a2)
    y = h2 @ W3.T + b3
    return y, (x, a1, h1, a2, h2)


def loss_and_grad(theta, x, t):
    """Mean squared error over all n * n_out outputs and its gradient."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    y, (x, a1, h1, a2, h2) = forward(theta, x)
    n = x.shape[0]
    d = y - t
    loss = float(np.mean(d * d))
    dy = 2.0 * d / (n * y.shape[1])
    gW3 = dy.T @ h2
    gb3 = dy.sum(axis=0)
    dh2 = dy @ W3
    da2 = dh2 * dsilu(a2)
    gW2 = da2.T @ h1
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * dsilu(a1)
    gW1 = da1.T @ x
    gb1 = da1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam_step(theta, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def targets_from_errors(e):
    return np.log(np.maximum(-np.asarray(e, dtype=float), 0.0) + E_FLOOR)


def errors_from_targets(y):
    return -(np.exp(np.asarray(y, dtype=float)) - E_FLOOR)
