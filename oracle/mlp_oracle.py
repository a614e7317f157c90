"""FP64 reference of the learned sub-sample TDoA stage (test infrastructure).

Only the test-suite imports this module; the GPU library never calls it.

A small multilayer perceptron maps the rank-D projection coefficients of one
pair-frame (eq. 9: z_k = a_k + j b_k, k = 1 .. D) to a sub-sample TDoA and a
confidence:

    u   = (a_1, b_1, ..., a_D, b_D) / ||(a, b)||_2            (scale-free input)
    h1  = gelu(u W1 + b1),  h2 = gelu(h1 W2 + b2)              (hidden width H)
    (mu, s) = h2 W3 + b3                                       (mu: TDoA in samples)

s is the log-variance of a Gaussian error model, clipped to [-S_CLIP, S_CLIP]
(the clip is part of the model; its gradient is zero outside).  The training
loss of a batch of R rows with true delays delta is the mean negative
log-likelihood  L = (1/R) sum_r 0.5 (exp(-s_r) (mu_r - delta_r)^2 + s_r).
The confidence of a prediction is exp(-s / 2), the inverse predicted
standard deviation.

gelu is the tanh form of Hendrycks and Gimpel (2016):
    gelu(x) = 0.5 x (1 + tanh(c (x + 0.044715 x^3))),  c = sqrt(2 / pi).

Parameters are one flat float64 vector in the order W1 [in][H], b1 [H],
W2 [H][H], b2 [H], W3 [H][2], b3 [2] (row-major), the same layout the GPU
library uses.
"""
from __future__ import annotations

import math

import numpy as np

S_CLIP = 8.0
GELU_C = math.sqrt(2.0 / math.pi)
GELU_A = 0.044715


def num_params(in_dim: int, hidden: int) -> int:
    return in_dim * hidden + hidden + hidden * hidden + hidden + hidden * 2 + 2


def unpack(theta, in_dim: int, hidden: int):
    theta = np.asarray(theta, dtype=np.float64)
    shapes = [(in_dim, hidden), (hidden,), (hidden, hidden), (hidden,), (hidden, 2), (2,)]
    out, o = [], 0
    for sh in shapes:
        n = int(np.prod(sh))
        out.append(theta[o:o + n].reshape(sh))
        o += n
    assert o == theta.size
    return out


def init_params(in_dim: int, hidden: int, seed: int) -> np.ndarray:
    """He-style normal initialisation, zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((in_dim, hidden)) * math.sqrt(2.0 / in_dim)
    W2 = rng.standard_normal((hidden, hidden)) * math.sqrt(2.0 / hidden)
    W3 = rng.standard_normal((hidden, 2)) * math.sqrt(1.0 / hidden)
    parts = [W1, np.zeros(hidden), W2, np.zeros(hidden), W3, np.zeros(2)]
    return np.concatenate([p.ravel() for p in parts])


def gelu(x):
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * x * (1.0 + np.tanh(GELU_C * (x + GELU_A * x ** 3)))


def gelu_grad(x):
    x = np.asarray(x, dtype=np.float64)
    t = np.tanh(GELU_C * (x + GELU_A * x ** 3))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * GELU_A * x * x)


def features(coef):
    """Rows of coefficients scaled to unit length (zero rows stay zero)."""
    c = np.asarray(coef, dtype=np.float64)
    n = np.sqrt((c * c).sum(-1, keepdims=True))
    return np.where(n > 0, c / np.where(n > 0, n, 1.0), 0.0)


def forward(theta, coef, hidden: int):
    """Returns (mu, s_clipped, cache)."""
    u = features(coef)
    W1, b1, W2, b2, W3, b3 = unpack(theta, u.shape[-1], hidden)
    z1 = u @ W1 + b1
    h1 = gelu(z1)
    z2 = h1 @ W2 + b2
    h2 = gelu(z2)
    o = h2 @ W3 + b3
    mu, s_raw = o[:, 0], o[:, 1]
    s = np.clip(s_raw, -S_CLIP, S_CLIP)
    return mu, s, (u, z1, h1, z2, h2, s_raw)


def loss_and_grad(theta, coef, delta, hidden: int):
    """Mean Gaussian negative log-likelihood and its gradient w.r.t. theta."""
    delta = np.asarray(delta, dtype=np.float64)
    mu, s, (u, z1, h1, z2, h2, s_raw) = forward(theta, coef, hidden)
    R = mu.size
    W1, b1, W2, b2, W3, b3 = unpack(theta, u.shape[-1], hidden)
    e = mu - delta
    w = np.exp(-s)
    L = float(np.mean(0.5 * (w * e * e + s)))
    dmu = w * e / R
    ds = 0.5 * (1.0 - w * e * e) / R
    ds = np.where((s_raw > -S_CLIP) & (s_raw < S_CLIP), ds, 0.0)
    do = np.stack([dmu, ds], axis=1)
    gW3 = h2.T @ do
    gb3 = do.sum(0)
    dz2 = (do @ W3.T) * gelu_grad(z2)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2.T) * gelu_grad(z1)
    gW1 = u.T @ dz1
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return L, g


def adam_step(theta, m, v, g, step: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma and Ba, 2015) with bias correction; returns new state."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
