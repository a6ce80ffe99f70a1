"""Pins for the Haar counts, the exact brickwork transfer and the estimator (CPU only)."""

import math
import os

import numpy as np
import pytest

import synth
from oracle import closed_forms, dense, estimator, sampler
from oracle.haar_moments import haar_frame_potential, lis_length
from oracle.weingarten import brickwork_bound_k2, brickwork_frame_potential

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_lis_length_small():
    assert lis_length([3, 1, 2]) == 2
    assert lis_length([1, 2, 3, 4]) == 4
    assert lis_length([4, 3, 2, 1]) == 1


def test_haar_counts_golden():
    with open(os.path.join(GOLDEN, "lis_counts.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            d, k, c = (int(x) for x in line.split())
            assert haar_frame_potential(k, d) == c


def test_haar_counts_factorial_and_trivial():
    for k in range(1, 7):
        assert haar_frame_potential(k, k) == math.factorial(k)
        assert haar_frame_potential(k, 1) == 1


def test_weingarten_first_moment_is_one():
    for n, d in [(4, 2), (5, 3), (6, 4)]:
        assert brickwork_frame_potential(n, d, 1) == pytest.approx(1.0, rel=1e-10)


def test_weingarten_depth1_product():
    for n in (4, 5, 6):
        for k in (1, 2, 3):
            assert brickwork_frame_potential(n, 1, k) == pytest.approx(
                closed_forms.brickwork_depth1_frame_potential(n, k), rel=1e-12)


def test_weingarten_two_qubits_is_haar():
    for k in range(1, 6):
        for d in (1, 2, 3):
            assert brickwork_frame_potential(2, d, k) == pytest.approx(haar_frame_potential(k, 4), rel=1e-9)


def test_weingarten_below_paper_bound_with_equality_at_one_layer():
    for n in (4, 6):
        assert brickwork_frame_potential(n, 1, 2) == pytest.approx(brickwork_bound_k2(n, 1), rel=1e-12)
        for d in range(2, 7):
            assert brickwork_frame_potential(n, d, 2) < brickwork_bound_k2(n, d)


def test_weingarten_monotone_and_haar_limit():
    vals = [brickwork_frame_potential(4, d, 2) for d in range(1, 9)]
    assert all(vals[i + 1] <= vals[i] + 1e-12 for i in range(len(vals) - 1))
    assert brickwork_frame_potential(4, 40, 2) == pytest.approx(2.0, rel=1e-6)
    assert brickwork_frame_potential(4, 40, 3) == pytest.approx(6.0, rel=1e-6)


def test_weingarten_against_dense_monte_carlo():
    # independent estimate: dense traces of sampled circuits, n = 4, D = 2
    pairs = sampler.sample_pairs(sampler.BRICKWORK, 4, 2, 21, 0, 3000)
    tr = dense.traces(pairs)
    f, se = estimator.frame_potential(tr, 2)
    for k in (1, 2):
        want = brickwork_frame_potential(4, 2, k)
        assert abs(f[k - 1] - want) < 4.5 * se[k - 1], (k, f, se, want)


def test_hea_one_layer_frame_potential_closed_form():
    # F^(k) = (C(2k,k)^2/4^k)^n: E|2cos(a/2)cos(b/2)|^{2k} with uniform a, b
    th = synth.uniform(3, (200000, 2), 0, 2 * np.pi)
    x = (2 * np.cos(th[:, 0] / 2) * np.cos(th[:, 1] / 2)) ** 2
    for k in (1, 2, 3):
        est = np.mean(x ** k)
        se = np.std(x ** k) / np.sqrt(x.size)
        assert abs(est - closed_forms.hea_one_layer_frame_potential(1, k)) < 4.5 * se


def test_estimator_definition():
    tr = np.array([1.0, 1j, 2.0, 0.5 - 0.5j])
    a = np.array([1.0, 1.0, 4.0, 0.5])
    f, se = estimator.frame_potential(tr, 3)
    for k in (1, 2, 3):
        assert f[k - 1] == pytest.approx(np.mean(a ** k))
        assert se[k - 1] == pytest.approx(np.std(a ** k, ddof=1) / 2.0)


def test_control_variate_reduces_to_plain_mean():
    f = synth.normal(4, 100) ** 2
    g_b = np.full(100, 3.0)
    g_c = np.full(1000, 3.0)
    est, _ = estimator.control_variate(f, g_b, g_c, 0.7)
    assert est == pytest.approx(f.mean(), rel=1e-14)
    est0, se0 = estimator.control_variate(f, synth.normal(5, 100), synth.normal(6, 1000), 0.0)
    assert est0 == pytest.approx(f.mean(), rel=1e-14)
    assert se0 == pytest.approx(f.std(ddof=1) / 10.0, rel=1e-12)


def test_bootstrap_centred():
    tr = synth.heavy_tailed_traces(8, 2000)
    b = estimator.bootstrap(tr, 2, resamples=300, seed=1)
    f, se = estimator.frame_potential(tr, 2)
    assert abs(np.median(b) - f[1]) < 3 * se[1]
    assert 0.5 * se[1] < b.std() < 2.0 * se[1]
