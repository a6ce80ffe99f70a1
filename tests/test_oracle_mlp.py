"""Pin of the oracle's surrogate-network backward pass: central finite differences (CPU)."""

import numpy as np

import synth
from oracle import mlp


def test_backward_matches_finite_differences():
    n_in, h, b = 7, 5, 6
    p = synth.normal(1, mlp.param_count(n_in, h), std=0.5)
    x = synth.normal(2, (b, n_in))
    t = synth.normal(3, b)
    loss, g = mlp.loss_and_grad(p, x, t, n_in, h)
    eps = 1e-6
    for i in range(p.size):
        d = np.zeros_like(p)
        d[i] = eps
        lp, _ = mlp.loss_and_grad(p + d, x, t, n_in, h)
        lm, _ = mlp.loss_and_grad(p - d, x, t, n_in, h)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_forward_definition_small():
    # one hidden unit per layer, identity-like weights: y = silu(silu(silu(x)))
    p = np.array([1.0, 0.0, 1.0, 0.0, 1.0, 0.0, 1.0, 0.0])
    x = np.array([[0.3], [-1.2]])
    y, _ = mlp.forward(p, x, 1, 1)
    s = lambda z: z / (1 + np.exp(-z))
    assert np.allclose(y, s(s(s(x[:, 0]))), rtol=1e-15)


def test_features_order():
    th_u = np.array([[[0.1, 0.2]]])
    ph_u = np.array([[[0.3, 0.4]]])
    th_v = np.array([[[0.5, 0.6]]])
    ph_v = np.array([[[0.7, 0.8]]])
    f = mlp.features(th_u, ph_u, th_v, ph_v)[0]
    # U: (q0: th sin cos, ph sin cos), (q1: ...), then V
    want = []
    for th, ph in ((th_u, ph_u), (th_v, ph_v)):
        for q in range(2):
            for a in (th[0, 0, q], ph[0, 0, q]):
                want += [np.sin(a), np.cos(a)]
    assert np.allclose(f, want)
