"""Pins of the oracle for the paper's hardware-efficient ansatz (Fig. 2c;
Sec. II.C): RY(pi/4) wall, random Pauli rotations, CNOT or CZ walls (CPU)."""

import math

import numpy as np
import pytest

from oracle import ancilla, closed_forms, dense, mpo, sampler

ANS = [sampler.PAULI_CNOT, sampler.PAULI_CZ]


@pytest.mark.parametrize("ans", ANS)
def test_one_layer_closed_form(ans):
    for n in range(2, 7):
        for u, v in sampler.sample_pairs(ans, n, 1, 100 + n, 0, 6):
            want = closed_forms.pauli_one_layer_trace(u, v)
            assert abs(dense.trace_pair(u, v) - want) <= 1e-12 * 2 ** n


@pytest.mark.parametrize("ans", ANS)
def test_fixed_wall_cancels_in_the_trace(ans):
    # a fixed unitary applied first in both circuits drops out of Tr(U^dag V)
    for L in (1, 2, 3):
        for u, v in sampler.sample_pairs(ans, 5, L, 7 + L, 0, 3):
            assert abs(dense.trace_pair(u, v) - dense.trace_pair(u, v, wall=False)) <= 1e-12 * 32
            # the wall does change the unitaries themselves
            assert np.max(np.abs(dense.circuit_unitary(u) - dense.circuit_unitary(u, wall=False))) > 0.1


def _proj(b):
    p = np.zeros((2, 2), dtype=np.complex128)
    p[b, b] = 1.0
    return p


def test_gates_by_kronecker_products():
    # U of three qubits, two layers, built from Kronecker products of 2x2
    # blocks: controlled gates as sum_b |b><b| (x) P^b with P = X (CNOT) or Z (CZ)
    x = np.array([[0.0, 1.0], [1.0, 0.0]], dtype=np.complex128)
    z = np.diag([1.0, -1.0]).astype(np.complex128)
    i2 = np.eye(2, dtype=np.complex128)
    for ans, p in ((sampler.PAULI_CNOT, x), (sampler.PAULI_CZ, z)):
        (u, _), = sampler.sample_pairs(ans, 3, 2, 31, 0, 1)
        ctl01 = sum(np.kron(np.kron(_proj(b), np.linalg.matrix_power(p, b)), i2) for b in (0, 1))
        ctl12 = sum(np.kron(i2, np.kron(_proj(b), np.linalg.matrix_power(p, b))) for b in (0, 1))
        c, s = math.cos(math.pi / 8), math.sin(math.pi / 8)
        ry = np.array([[c, -s], [s, c]], dtype=np.complex128)
        m = np.kron(np.kron(ry, ry), ry)
        for l in range(2):
            rots = []
            for q in range(3):
                th, a = u["theta"][l, q], u["axis"][l, q]
                pa = [x, np.array([[0, -1j], [1j, 0]]), z][a]
                rots.append(math.cos(th / 2) * i2 - 1j * math.sin(th / 2) * pa)
            m = ctl12 @ ctl01 @ np.kron(np.kron(rots[0], rots[1]), rots[2]) @ m
        assert np.max(np.abs(dense.circuit_unitary(u) - m)) <= 1e-13


@pytest.mark.parametrize("ans", ANS)
def test_independent_contractions_agree(ans):
    for n, L in [(2, 2), (4, 2), (5, 3), (6, 2), (4, 4)]:
        pr = sampler.sample_pairs(ans, n, L, 55 + n * L, 0, 3)
        for u, v in pr:
            d = dense.trace_pair(u, v)
            assert abs(mpo.trace_pair(u, v) - d) <= 1e-11 * 2 ** n
            assert abs(ancilla.trace_pair(u, v) - d) <= 1e-11 * 2 ** n


def test_axes_uniform_and_angles_in_range():
    th, ax = sampler.pauli_params(99, 10, 4, np.arange(300, dtype=np.uint64), 1)
    counts = np.bincount(ax.ravel(), minlength=3)
    e = ax.size / 3.0
    chi2 = float(np.sum((counts - e) ** 2 / e))
    assert counts.size == 3 and chi2 < 13.8  # 2 degrees of freedom, p = 0.001
    assert th.min() > 0.0 and th.max() <= 2 * math.pi
    # batch split: the same pair index gives the same draw
    th2, ax2 = sampler.pauli_params(99, 10, 4, np.arange(150, 300, dtype=np.uint64), 1)
    assert np.array_equal(th[150:], th2) and np.array_equal(ax[150:], ax2)


def test_one_layer_frame_potential_formula():
    # Monte Carlo of the one-layer closed form (whose trace is pinned above
    # against the dense oracle) against F^(1) = (4/3)^n, F^(2) = (7/2)^n
    n, npairs = 2, 400000
    pr = np.arange(npairs, dtype=np.uint64)
    tu, au = sampler.pauli_params(5, n, 1, pr, 0)
    tv, av = sampler.pauli_params(5, n, 1, pr, 1)
    same = au[:, 0] == av[:, 0]
    tr = np.where(same, 2 * np.cos((tv[:, 0] - tu[:, 0]) / 2), 2 * np.cos(tu[:, 0] / 2) * np.cos(tv[:, 0] / 2))
    tr = np.prod(tr, axis=1)
    for k in (1, 2):
        f = np.abs(tr) ** (2 * k)
        want = closed_forms.pauli_one_layer_frame_potential(n, k)
        assert abs(f.mean() - want) <= 5 * f.std() / math.sqrt(npairs), (k, f.mean(), want)
    assert closed_forms.pauli_one_layer_frame_potential(3, 1) == pytest.approx((4 / 3) ** 3)
    assert closed_forms.pauli_one_layer_frame_potential(3, 2) == pytest.approx(3.5 ** 3)
