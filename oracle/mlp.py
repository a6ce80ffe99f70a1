"""Float64 reference of the surrogate network used as a control variate.

TEST INFRASTRUCTURE (CPU oracle; see oracle/__init__.py).

The paper has no learned component; this is the reference for the
control-variate extension: features are the sine and cosine of every angle
of U and V, the network has three SiLU hidden layers and one linear output,
and the loss is the mean squared error (1/B) sum_i (y_i - t_i)^2.  Forward
and backward are written out layer by layer; tests pin the backward pass
with central finite differences.

Parameter vector layout (as the library's): W1 (n_in x H, row-major), b1 (H),
W2 (H x H), b2, W3 (H x H), b3, w4 (H), b4 (1).  Feature order: circuit U
then V, layer l, qubit q, angle (theta, phi), then (sin, cos).
"""

import numpy as np


def param_count(n_in, h):
    return n_in * h + h + 2 * (h * h + h) + h + 1


def unpack(p, n_in, h):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    out = []
    for shape in [(n_in, h), (h,), (h, h), (h,), (h, h), (h,), (h,), (1,)]:
        n = int(np.prod(shape))
        out.append(p[o:o + n].reshape(shape))
        o += n
    return out


def features(theta_u, phi_u, theta_v, phi_v):
    """(batch, L, n) angle arrays of both circuits -> (batch, 8 n L) features."""
    parts = []
    for th, ph in ((theta_u, phi_u), (theta_v, phi_v)):
        a = np.stack([th, ph], axis=-1)                       # (B, L, n, 2)
        sc = np.stack([np.sin(a), np.cos(a)], axis=-1)        # (B, L, n, 2, 2)
        parts.append(sc.reshape(sc.shape[0], -1))
    return np.concatenate(parts, axis=1)


def _silu(z):
    return z / (1.0 + np.exp(-z))


def _dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p, x, n_in, h):
    w1, b1, w2, b2, w3, b3, w4, b4 = unpack(p, n_in, h)
    z1 = x @ w1 + b1
    h1 = _silu(z1)
    z2 = h1 @ w2 + b2
    h2 = _silu(z2)
    z3 = h2 @ w3 + b3
    h3 = _silu(z3)
    y = h3 @ w4 + b4[0]
    return y, (z1, h1, z2, h2, z3, h3)


def loss_and_grad(p, x, t, n_in, h):
    w1, b1, w2, b2, w3, b3, w4, b4 = unpack(p, n_in, h)
    y, (z1, h1, z2, h2, z3, h3) = forward(p, x, n_in, h)
    bsz = x.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / bsz
    gw4 = h3.T @ dy
    gb4 = np.array([dy.sum()])
    dz3 = np.outer(dy, w4) * _dsilu(z3)
    gw3 = h2.T @ dz3
    gb3 = dz3.sum(axis=0)
    dz2 = (dz3 @ w3.T) * _dsilu(z2)
    gw2 = h1.T @ dz2
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ w2.T) * _dsilu(z1)
    gw1 = x.T @ dz1
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gw1.ravel(), gb1, gw2.ravel(), gb2, gw3.ravel(), gb3, gw4, gb4])
    return loss, g


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
