"""GPU parity of the paper's hardware-efficient ansatz (Fig. 2c; Sec. II.C):
RY(pi/4) wall, random Pauli rotations, CNOT or CZ walls -- sampler and
contraction against the oracle (dense for n <= 8, MPO-zip beyond), the
one-layer closed forms and the Haar lower bound."""

import math

import numpy as np
import pytest
import torch

import synth
from oracle import closed_forms, dense, sampler
from oracle.haar_moments import haar_frame_potential
import oracle_pool
from tolerance import TOL, floored

pytestmark = pytest.mark.gpu

ANS = [3, 4]  # CNOT walls, CZ walls


@pytest.fixture(scope="module")
def fp():
    import paper_2205_09900_amd as m
    assert torch.cuda.is_available()
    return m


def gpu_traces(fp, ens, n_pairs, seed, prec, first=0):
    g = fp.sample(ens, n_pairs, seed, first, prec)
    return fp.contract(ens, g, n_pairs, prec).cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("ans", ANS)
def test_sampler_matches_oracle(fp, ans, prec):
    ens, npairs, first, seed = (ans, 6, 3), 7, 11, 4321
    buf = fp.sample(ens, npairs, seed, first, prec).cpu().numpy()
    nb = fp.fp_gate_bytes_per_pair(ens, prec)
    real = np.float64 if prec == 0 else np.float32
    want = sampler.sample_pairs(ans, 6, 3, seed, first, npairs, fp32=(prec != 0))
    for p in range(npairs):
        a = np.frombuffer(buf[p * nb:(p + 1) * nb].tobytes(), dtype=real)[: 2 * 3 * 6 * 2]
        a = a.astype(np.float64).reshape(2, 3, 6, 2)
        for c in range(2):
            assert np.array_equal(a[c, :, :, 1].astype(np.int64), want[p][c]["axis"])
            assert np.max(np.abs(a[c, :, :, 0] - want[p][c]["theta"])) <= (1e-15 if prec == 0 else 5e-7)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("ans", ANS)
def test_vs_dense(fp, ans, prec):
    for n, L in [(2, 1), (2, 2), (3, 2), (4, 3), (5, 2), (6, 4), (7, 3), (8, 5), (4, 7), (3, 6)]:
        seed = synth.workload_seed(50 + ans, L) + n
        got = gpu_traces(fp, (ans, n, L), 24, seed, prec)
        want = dense.traces(sampler.sample_pairs(ans, n, L, seed, 0, 24, fp32=(prec != 0)))
        err = floored(got, want, prec)
        assert err.max() <= TOL[prec], (n, L, err.max())


@pytest.mark.parametrize("ans", ANS)
def test_wide_vs_mpo(fp, ans):
    for n, L, prec in [(20, 2, 1), (20, 4, 1), (30, 3, 0), (16, 5, 1), (12, 6, 0)]:
        seed = synth.workload_seed(60 + ans, L) + n
        npairs = 600
        got = gpu_traces(fp, (ans, n, L), npairs, seed, prec)
        pick = sorted(int(x) for x in synth.rng(n * L + ans).choice(npairs, 6, replace=False))
        want = np.array(oracle_pool.traces(ans, n, L, seed, pick, fp32=(prec != 0)))
        err = floored(got[pick], want, prec)
        assert err.max() <= TOL[prec], (n, L, prec, err.max())


def test_bf16x3_vs_dense(fp):
    for ans in ANS:
        seed = 777 + ans
        got = gpu_traces(fp, (ans, 6, 4), 32, seed, 2)
        want = dense.traces(sampler.sample_pairs(ans, 6, 4, seed, 0, 32, fp32=True))
        assert floored(got, want, 0).max() <= 5e-3


@pytest.mark.parametrize("ans", ANS)
def test_one_layer_closed_form_and_moments(fp, ans):
    # per pair against the closed form, and F^(1) = (4/3)^n, F^(2) = (7/2)^n
    n, seed = 4, synth.workload_seed(70, ans)
    got = gpu_traces(fp, (ans, n, 1), 40, seed, 0)
    want = [closed_forms.pauli_one_layer_trace(u, v) for u, v in sampler.sample_pairs(ans, n, 1, seed, 0, 40)]
    assert np.max(np.abs(got - np.array(want))) <= 1e-12 * 2 ** n
    npairs = 4_000_000
    tr = fp.contract((ans, n, 1), fp.sample((ans, n, 1), npairs, seed, 0, fp.C64), npairs, fp.C64)
    f, se = fp.frame_potential(tr, 2)
    for k in (1, 2):
        exact = closed_forms.pauli_one_layer_frame_potential(n, k)
        assert abs(f[k - 1] - exact) <= 5 * se[k - 1], (k, f[k - 1], se[k - 1], exact)


@pytest.mark.parametrize("ans", ANS)
def test_frame_potential_above_haar(fp, ans):
    # any ensemble has F^(k) >= F_Haar^(k) (here 2^n >= k, so k!): deep circuits approach it from above
    n, L, npairs = 4, 7, 400000
    tr = fp.contract((ans, n, L), fp.sample((ans, n, L), npairs, synth.workload_seed(71, ans), 0, fp.C64), npairs,
                     fp.C64)
    f, se = fp.frame_potential(tr, 3)
    for k in (1, 2, 3):
        print(f"ansatz {ans} n={n} L={L}: F^({k}) = {f[k - 1]:.4g} +- {se[k - 1]:.2g} (Haar {haar_frame_potential(k, 16)})")
        assert f[k - 1] >= haar_frame_potential(k, 16) - 5 * se[k - 1]
