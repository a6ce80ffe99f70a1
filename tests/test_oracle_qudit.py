"""Pins of the qudit brickwork oracle (Sec. II.A, generalisation to qudits) -- CPU."""

import math

import numpy as np
import pytest

from oracle import qudit
from oracle.haar_moments import haar_frame_potential


def test_gates_are_unitary_and_batch_split_invariant():
    g = qudit.haar_gates(5, 3, np.arange(4, dtype=np.uint64), 1, 3)
    for m in g.reshape(-1, 9, 9):
        assert np.max(np.abs(m.conj().T @ m - np.eye(9))) <= 1e-13
    h = qudit.haar_gates(5, 3, np.arange(2, 4, dtype=np.uint64), 1, 3)
    assert np.array_equal(g[2:], h)


def test_dense_by_kronecker_products():
    (u, _), = qudit.sample_pairs(4, 3, 3, 9, 0, 1)
    n, q = 4, 3
    m = np.eye(q ** n, dtype=np.complex128)
    for b, g in u["gates"]:
        m = np.kron(np.kron(np.eye(q ** b), g), np.eye(q ** (n - b - 2))) @ m
    assert np.max(np.abs(qudit.dense_unitary(u) - m)) <= 1e-12


@pytest.mark.parametrize("q", [3, 4])
def test_mpo_matches_dense_and_identities(q):
    for n, d in [(2, 1), (3, 2), (4, 3), (5, 2)]:
        if q ** n > 1024:
            continue
        for u, v in qudit.sample_pairs(n, q, d, 17 + n * d, 0, 3):
            t = qudit.dense_trace(u, v)
            assert abs(qudit.mpo_trace(u, v) - t) <= 1e-11 * q ** n
            assert abs(qudit.dense_trace(u, u) - q ** n) <= 1e-10 * q ** n
            if d == 1:
                assert abs(qudit.depth1_trace(u, v) - t) <= 1e-11 * q ** n


def test_two_qutrit_haar_moments():
    # one Haar U(9) gate per circuit: F^(k) = k! for k <= 9
    pr = qudit.sample_pairs(2, 3, 1, 77, 0, 20000)
    a = np.abs(np.array([qudit.depth1_trace(u, v) for u, v in pr])) ** 2
    for k in (1, 2, 3):
        f = a ** k
        assert abs(f.mean() - haar_frame_potential(k, 9)) <= 5 * f.std() / math.sqrt(a.size), (k, f.mean())


def test_first_moment_twirl():
    # every qudit meets a Haar gate: F^(1) = 1
    pr = qudit.sample_pairs(4, 3, 2, 78, 0, 3000)
    a = np.abs(np.array([qudit.mpo_trace(u, v) for u, v in pr])) ** 2
    assert abs(a.mean() - 1.0) <= 5 * a.std() / math.sqrt(a.size)
