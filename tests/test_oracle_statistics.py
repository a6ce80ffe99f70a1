"""Pins of the oracle's statistics (bootstrap, quantiles, fit region, layers
to epsilon, sample-size rule) -- CPU."""

import math

import numpy as np
import pytest

import synth
from oracle import statistics as st
from oracle.philox import key_from_seed, philox4x32_10


def test_resample_index_is_the_high_word_of_u_times_n():
    # floor(u N / 2^64) with Python integers, u the 64-bit word of the draw
    n, r, seed = 1000003, 7, 12345
    idx = st.resample_indices(n, r, seed)
    for i in (0, 1, 2, 3, 1000, 1000001, 1000002):
        b = i >> 1
        x = philox4x32_10(np.array([[b & 0xFFFFFFFF, b >> 32, r, st.BOOT_TAG]], dtype=np.uint64),
                          key_from_seed(seed))[0]
        u = int(x[0]) + (int(x[1]) << 32) if i % 2 == 0 else int(x[2]) + (int(x[3]) << 32)
        assert idx[i] == (u * n) >> 64
    assert idx.min() >= 0 and idx.max() < n


def test_resample_indices_uniform():
    n = 50
    counts = np.zeros(n)
    for r in range(200):
        counts += np.bincount(st.resample_indices(n, r, 3), minlength=n)
    e = counts.sum() / n
    chi2 = float(np.sum((counts - e) ** 2 / e))
    assert chi2 < 95.0  # 49 degrees of freedom, p ~ 1e-4


def test_bootstrap_constant_and_spread():
    z = np.full(40, 1.5 + 0.5j)
    b = st.bootstrap_philox(z, 2, 30, 9)
    assert np.allclose(b[0], 2.5, rtol=0, atol=1e-15) and np.allclose(b[1], 6.25, rtol=0, atol=1e-14)
    # the spread of the resample means is the standard error of the mean
    z = synth.heavy_tailed_traces(4, 4000)
    a = np.abs(z) ** 2
    b = st.bootstrap_philox(z, 1, 300, 11)[0]
    se = a.std(ddof=1) / math.sqrt(a.size)
    assert abs(b.std(ddof=1) / se - 1.0) < 0.2
    assert abs(b.mean() - a.mean()) < 4 * se / math.sqrt(300) + 1e-12


def test_quantile_linear_interpolation():
    v = np.sort(synth.normal(5, 300))
    for q in (0.0, 0.025, 0.5, 0.975, 1.0):
        assert st.quantile(v, q) == pytest.approx(float(np.quantile(v, q)), rel=0, abs=1e-14)
    assert st.quantile([1.0, 2.0, 3.0, 10.0], 0.5) == 2.5


def test_layers_to_epsilon_on_an_exact_exponential():
    # F - F_Haar = A^2 exp(-2 l / C) with A = 3, C = 1.7; n = 4, q = 2, k = 2
    A, C, fh = 3.0, 1.7, 2.0
    layers = np.arange(1, 12)
    f = fh + A * A * np.exp(-2.0 * layers / C)
    m = st.fit_region(f, fh)
    assert list(m) == [bool(d < 5.0) for d in (f - fh) / fh]
    l_eps, a, c = st.layers_to_epsilon(layers, f, fh, 0.1, 4, 2, 2)
    assert a == pytest.approx(A, rel=1e-12) and c == pytest.approx(C, rel=1e-12)
    # the defining condition A exp(-l / C) = epsilon / q^(n k), and the worked number
    assert A * math.exp(-l_eps / C) == pytest.approx(0.1 / 2 ** 8, rel=1e-12)
    assert l_eps == pytest.approx(1.7 * (8 * math.log(2) + math.log(3) + math.log(10)), rel=1e-12)
    # a point far outside the region must not move the fit
    f2 = f.copy()
    f2[0] = fh * 20
    assert st.layers_to_epsilon(layers, f2, fh, 0.1, 4, 2, 2)[0] == pytest.approx(l_eps, rel=1e-12)
    # fewer than two points, or no decay: no estimate
    assert st.layers_to_epsilon([1, 2], [fh * 10, fh * 0.5], fh, 0.1, 4, 2, 2) is None
    assert st.layers_to_epsilon([1, 2, 3], [fh * 1.5, fh * 2, fh * 3], fh, 0.1, 4, 2, 2) is None


def test_adaptive_decision_cases():
    d = st.adaptive_decision
    assert d(2.5, 0.1, 2.0, None, 3.0, 100, 1000, 1.0, 10.0) == st.STOP_RESOLVED   # 5 SE above Haar
    assert d(2.2, 0.1, 2.0, None, 3.0, 100, 1000, 1.0, 10.0) == st.CONTINUE        # 2 SE only
    assert d(1.9, 0.01, 2.0, None, 3.0, 100, 1000, 1.0, 10.0) == st.CONTINUE       # below Haar
    assert d(2.5, 0.1, 2.0, 2.4, 3.0, 100, 1000, 1.0, 10.0) == st.CONTINUE         # above the shallower depth
    assert d(2.5, 0.1, 2.0, 2.6, 3.0, 100, 1000, 1.0, 10.0) == st.STOP_RESOLVED
    assert d(1.9, 0.01, 2.0, None, 3.0, 1000, 1000, 1.0, 10.0) == st.STOP_BUDGET   # pairs spent
    assert d(1.9, 0.01, 2.0, None, 3.0, 100, 1000, 11.0, 10.0) == st.STOP_BUDGET   # time spent
