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


# Pins of the oracle's Adam update against Kingma & Ba (2015), Algorithm 1:
# m_t = b1 m + (1-b1) g, v_t = b2 v + (1-b2) g^2, bias-corrected by 1 - b^t,
# step lr * m_hat / (sqrt(v_hat) + eps).  Values below are worked by hand.

def test_adam_first_step_is_lr_times_sign():
    # t = 1 from zero moments: m_hat = g and v_hat = g^2 exactly, so the step
    # is lr * g / (|g| + eps), about lr in size whatever the gradient's scale.
    p = np.array([0.5, -2.0, 3.0])
    g = np.array([4.0, -1e-3, 250.0])
    q, m, v = mlp.adam(p, g, np.zeros(3), np.zeros(3), 1, 0.01, eps=0.0)
    assert np.allclose(q, p - 0.01 * np.sign(g), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g, rtol=1e-15) and np.allclose(v, 0.001 * g * g, rtol=1e-12)


def test_adam_eps_outside_the_square_root():
    # g = 1e-9, eps = 1e-8: the first step is lr * 1e-9 / (1e-9 + 1e-8) = lr / 11.
    # With eps under the root it would be about lr * 1e-5.
    q, _, _ = mlp.adam(np.zeros(1), np.array([1e-9]), np.zeros(1), np.zeros(1), 1, 1.0, eps=1e-8)
    assert abs(q[0] + 1.0 / 11.0) < 1e-12


def test_adam_two_steps_by_hand():
    # g1 = +1, g2 = -1, b1 = 0.9, b2 = 0.999, eps = 0:
    #   m1 = 0.1, v1 = 0.001; m2 = 0.09 - 0.1 = -0.01, v2 = 0.000999 + 0.001 = 0.001999
    #   m_hat2 = -0.01 / (1 - 0.81) = -1/19, v_hat2 = 0.001999 / (1 - 0.998001) = 1
    # so p2 = p0 - lr + lr / 19.
    lr = 0.25
    p1, m, v = mlp.adam(np.array([1.0]), np.array([1.0]), np.zeros(1), np.zeros(1), 1, lr, eps=0.0)
    p2, m, v = mlp.adam(p1, np.array([-1.0]), m, v, 2, lr, eps=0.0)
    assert abs(m[0] + 0.01) < 1e-15 and abs(v[0] - 0.001999) < 1e-15
    assert abs(p2[0] - (1.0 - lr + lr / 19.0)) < 1e-14


def test_adam_constant_gradient_moves_lr_each_step():
    # With a constant gradient the bias-corrected moments equal g and g^2 at
    # every step, so every step moves by lr * sign(g) (eps = 0).
    p, m, v = np.array([0.0, 0.0]), np.zeros(2), np.zeros(2)
    g = np.array([3.0, -0.02])
    for t in range(1, 8):
        p, m, v = mlp.adam(p, g, m, v, t, 0.1, eps=0.0)
        assert np.allclose(p, -0.1 * t * np.sign(g), rtol=0, atol=1e-12), t
