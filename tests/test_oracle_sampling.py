"""Pins for the oracle's generator and samplers (CPU only)."""

import math
import os

import numpy as np
import pytest

from oracle import philox, sampler
from oracle.haar_moments import haar_frame_potential

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    for ctr, key, want in _kat():
        got = philox.philox4x32_10(np.array(ctr, np.uint64), np.array(key, np.uint64))
        assert [int(x) for x in got] == want


def test_philox_vectorised_matches_scalar():
    ctrs = np.array([[i, 7 * i, 3, 0x80000001] for i in range(17)], np.uint64)
    key = np.array([0x12345678, 0x9abcdef0], np.uint64)
    batch = philox.philox4x32_10(ctrs, key)
    for i in range(17):
        assert np.array_equal(batch[i], philox.philox4x32_10(ctrs[i], key))


def test_counter_layout():
    c = philox.make_counter(5, 9, (1 << 40) + 3, 1)
    assert [int(x) for x in c] == [5, 9, 3, (1 << 8) | (1 << 31)]


def test_u53_open_interval_and_resolution():
    lo = sampler.u53(0, 0)
    hi = sampler.u53(0xFFFFFFFF, 0xFFFFFFFF)
    assert lo == 2.0 ** -53
    assert hi == 1.0
    assert 0.0 < lo < hi
    # the two words fill 27 + 26 = 53 bits
    assert sampler.u53(1 << 5, 0) - sampler.u53(0, 0) == pytest.approx(2.0 ** -27)
    assert sampler.u53(0, 1 << 6) - sampler.u53(0, 0) == pytest.approx(2.0 ** -53)


def test_gaussian_moments():
    z = sampler.gaussian_entries(11, np.arange(4000, dtype=np.uint64), 0, 0).ravel()
    x = np.concatenate([z.real, z.imag])
    assert abs(x.mean()) < 0.01
    assert abs(x.var() - 1.0) < 0.02
    # fourth moment of a standard normal is 3
    assert abs(np.mean(x ** 4) - 3.0) < 0.1


def _gram_schmidt(z):
    """Classical Gram-Schmidt on the columns (positive real R diagonal)."""
    q = np.zeros_like(z)
    for j in range(z.shape[1]):
        v = z[:, j].copy()
        for i in range(j):
            v -= np.vdot(q[:, i], z[:, j]) * q[:, i]
        q[:, j] = v / np.linalg.norm(v)
    return q


def test_haar_is_unitary_and_unique_qr_factor():
    z = sampler.gaussian_entries(3, np.arange(50, dtype=np.uint64), 1, 2)
    g = sampler.haar_from_gaussian(z)
    for i in range(50):
        assert np.allclose(g[i].conj().T @ g[i], np.eye(4), atol=1e-13)
        assert np.allclose(g[i], _gram_schmidt(z[i]), atol=1e-10)


def test_haar_u4_moments_match_permutation_counts():
    # E|Tr G|^{2k} over U(4) equals the LIS count (k! for k <= 4).
    z = sampler.gaussian_entries(5, np.arange(40000, dtype=np.uint64), 0, 0)
    g = sampler.haar_from_gaussian(z)
    a = np.abs(np.trace(g, axis1=-2, axis2=-1)) ** 2
    for k in (1, 2, 3):
        x = a ** k
        est, se = x.mean(), x.std() / math.sqrt(x.size)
        want = haar_frame_potential(k, 4)
        assert abs(est - want) < 4.5 * se, (k, est, want, se)


def test_brickwork_layout():
    b = sampler.brickwork_layout(6, 3)
    assert list(b) == [0, 2, 4, 1, 3, 0, 2, 4]
    b = sampler.brickwork_layout(5, 2)
    assert list(b) == [0, 2, 1, 3]


def test_local_random_bonds_uniform():
    bonds = sampler.local_random_bonds(9, 7, 400, np.arange(20, dtype=np.uint64), 0).ravel()
    assert bonds.min() >= 0 and bonds.max() <= 5
    counts = np.bincount(bonds, minlength=6)
    expected = bonds.size / 6.0
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    assert chi2 < 25.0        # 5 dof; p ~ 1e-4


def test_hea_angles_range_and_independence():
    th, ph = sampler.hea_angles(4, 10, 3, np.arange(500, dtype=np.uint64), 1)
    for a in (th, ph):
        assert a.min() > 0.0 and a.max() <= 2 * np.pi
        assert abs(a.mean() - np.pi) < 0.05
    assert abs(np.corrcoef(th.ravel(), ph.ravel())[0, 1]) < 0.02


def test_fp32_storage_rounds_exactly():
    p64 = sampler.sample_pairs(sampler.BRICKWORK, 4, 2, 17, 0, 2, fp32=False)
    p32 = sampler.sample_pairs(sampler.BRICKWORK, 4, 2, 17, 0, 2, fp32=True)
    g64 = p64[0][0]["gates"][0][1]
    g32 = p32[0][0]["gates"][0][1]
    assert np.array_equal(g32, g64.astype(np.complex64).astype(np.complex128))


def test_batch_split_invariance():
    a = sampler.sample_pairs(sampler.LOCAL_RANDOM, 6, 5, 99, 10, 4)
    b = sampler.sample_pairs(sampler.LOCAL_RANDOM, 6, 5, 99, 12, 2)
    for i in range(2):
        for c in range(2):
            ga, gb = a[2 + i][c]["gates"], b[i][c]["gates"]
            assert [x[0] for x in ga] == [x[0] for x in gb]
            assert all(np.array_equal(x[1], y[1]) for x, y in zip(ga, gb))
