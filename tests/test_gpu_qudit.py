"""GPU parity of qudit brickworks (local dimension q = 3, 4, 5; Haar U(q^2)
gates; the paper's generalisation of the trace network to qudits, Sec. II.A):
the sampler against the oracle's draws, the column sweep with base-q digits
against the dense trace (small q^n) and the MPO zip (longer chains), U = V,
the one-layer product of gate traces, split invariance of a batch, and the
Haar moments of a single gate (F^(k) = k! for k <= q^2)."""

import math

import numpy as np
import pytest
import torch

import synth
from oracle import estimator, qudit
from oracle.sampler import brickwork_layout
from tolerance import TOL, floored

pytestmark = pytest.mark.gpu

QUDIT = 5


@pytest.fixture(scope="module")
def fp():
    import paper_2205_09900_amd as m
    assert torch.cuda.is_available()
    return m


def gpu_traces(fp, ens, n_pairs, seed, prec, first=0):
    g = fp.sample(ens, n_pairs, seed, first, prec)
    tr = fp.contract(ens, g, n_pairs, prec)
    torch.cuda.synchronize()
    return tr.cpu().numpy()


def oracle_traces(n, q, depth, seed, n_pairs, prec, first=0, mpo=False):
    pairs = qudit.sample_pairs(n, q, depth, seed, first, n_pairs, fp32=(prec != 0))
    f = qudit.mpo_trace if mpo else qudit.dense_trace
    return np.array([f(u, v) for u, v in pairs])


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("q", [3, 4, 5])
def test_sampler_matches_oracle(fp, q, prec):
    n, depth, npairs, first, seed = 5, 3, 5, 7, 4099
    ens = (QUDIT, n, depth, q)
    G = len(brickwork_layout(n, depth))
    d = q * q
    buf = fp.sample(ens, npairs, seed, first, prec).cpu().numpy()
    nb = fp.fp_gate_bytes_per_pair(ens, prec)
    assert nb == -(-2 * G * d * d * 2 * (8 if prec == 0 else 4) // 64) * 64
    real = np.float64 if prec == 0 else np.float32
    pairs = np.arange(first, first + npairs)
    want = [qudit.haar_gates(seed, q, pairs, c, G) for c in (0, 1)]
    for p in range(npairs):
        a = np.frombuffer(buf[p * nb:(p + 1) * nb].tobytes(), dtype=real)[: 2 * G * d * d * 2]
        a = a.astype(np.float64).reshape(2, G, d, d, 2)
        m = a[..., 0] + 1j * a[..., 1]
        for c in range(2):
            # Gram-Schmidt and Householder QR agree to rounding on the unique
            # factor with a positive R diagonal
            tol = 1e-12 if prec == 0 else 3e-7
            assert np.max(np.abs(m[c] - want[c][p])) <= tol, (p, c)
            if prec == 0:
                for g in range(G):
                    assert np.max(np.abs(m[c, g].conj().T @ m[c, g] - np.eye(d))) <= 1e-13


DENSE_CASES = [(3, 2, 1), (3, 2, 3), (3, 3, 2), (3, 4, 3), (3, 5, 4), (3, 6, 5), (3, 5, 1),
               (4, 2, 2), (4, 3, 3), (4, 4, 4), (4, 4, 1), (5, 2, 3), (5, 3, 2), (5, 4, 3)]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("q,n,depth", DENSE_CASES)
def test_vs_dense(fp, q, n, depth, prec):
    seed = synth.workload_seed(70 + q, depth) + n
    npairs = 19  # not a multiple of anything the launch assumes
    got = gpu_traces(fp, (QUDIT, n, depth, q), npairs, seed, prec)
    want = oracle_traces(n, q, depth, seed, npairs, prec)
    err = floored(got, want, prec)
    assert err.max() <= TOL[prec], (q, n, depth, float(err.max()))


@pytest.mark.parametrize("q,n,depth", [(3, 9, 4), (3, 8, 5), (4, 7, 3), (4, 6, 4), (5, 6, 3)])
def test_vs_mpo(fp, q, n, depth):
    seed = synth.workload_seed(80 + q, depth) + n
    got = gpu_traces(fp, (QUDIT, n, depth, q), 6, seed, 0)
    want = oracle_traces(n, q, depth, seed, 6, 0, mpo=True)
    err = floored(got, want, 0)
    assert err.max() <= TOL[0], float(err.max())


def test_widest_register_c64(fp):
    """q = 5 at depth 4: 5^6 entries, the largest register that fits LDS in
    complex64 (complex128 refuses it)."""
    ens = (QUDIT, 4, 4, 5)
    seed = synth.workload_seed(85, 4)
    got = gpu_traces(fp, ens, 5, seed, 1)
    want = oracle_traces(4, 5, 4, seed, 5, 1)
    assert floored(got, want, 1).max() <= TOL[1]
    with pytest.raises(fp.FPError):
        fp.fp_workspace_bytes(ens, 5, 0)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("q,n,depth", [(3, 7, 4), (4, 5, 3), (5, 3, 3), (3, 12, 2)])
def test_u_equals_v(fp, q, n, depth, prec):
    """Tr(U^dagger U) = q^n: the V half of every pair overwritten with U."""
    ens = (QUDIT, n, depth, q)
    npairs = 9
    g = fp.sample(ens, npairs, 5 + q, 0, prec)
    nb = fp.fp_gate_bytes_per_pair(ens, prec)
    half = len(brickwork_layout(n, depth)) * q ** 4 * 2 * (8 if prec == 0 else 4)
    gv = g.view(npairs, nb)
    gv[:, half:2 * half] = gv[:, :half]
    tr = fp.contract(ens, g, npairs, prec).cpu().numpy()
    want = float(q) ** n
    assert np.max(np.abs(tr - want)) <= (1e-12 if prec == 0 else 2e-6) * want


@pytest.mark.parametrize("q,n", [(3, 6), (3, 7), (4, 5), (5, 4), (5, 3)])
def test_depth_one_closed_form(fp, q, n):
    """One layer: the product of Tr(G_U^dagger G_V) over its gates, times q for
    a qudit no gate touches."""
    seed = synth.workload_seed(90 + q, 1) + n
    got = gpu_traces(fp, (QUDIT, n, 1, q), 16, seed, 0)
    want = np.array([qudit.depth1_trace(u, v) for u, v in qudit.sample_pairs(n, q, 1, seed, 0, 16)])
    assert floored(got, want, 0).max() <= TOL[0]


def test_batch_split_and_empty(fp):
    ens = (QUDIT, 6, 3, 3)
    seed = 1234
    whole = gpu_traces(fp, ens, 37, seed, 0)
    a = gpu_traces(fp, ens, 20, seed, 0)
    b = gpu_traces(fp, ens, 17, seed, 0, first=20)
    assert np.array_equal(whole, np.concatenate([a, b]))
    g = fp.sample(ens, 1, seed, 0, 0)
    tr = torch.empty(2, dtype=torch.float64, device="cuda")
    fp.fp_contract_trace_batch(ens, 0, 0, g, tr, fp.workspace(ens, 1, 0))  # no pairs: nothing to do


@pytest.mark.parametrize("q,depth", [(3, 1), (4, 3)])
def test_single_gate_haar_moments(fp, q, depth):
    """n = 2: every layer acts on the one bond and the layers merge into one
    Haar gate of U(q^2), so F^(k) = k! for k <= q^2 (Diaconis-Shahshahani)."""
    ens = (QUDIT, 2, depth, q)
    n_pairs = 40000
    g = fp.sample(ens, n_pairs, 77 + q, 0, 0)
    tr = fp.contract(ens, g, n_pairs, 0)
    F, se = fp.frame_potential(tr, 3)
    for k in range(3):
        assert abs(F[k] - math.factorial(k + 1)) <= 5 * se[k] + 1e-12, (k, F[k], se[k])
    # the same estimate from the oracle's reduction of the returned traces
    fo, _ = estimator.frame_potential(tr.cpu().numpy(), 3)
    assert np.allclose(F, fo, rtol=1e-12)


@pytest.mark.parametrize("q,n,depth", [(3, 6, 4), (4, 4, 3), (5, 3, 3)])
def test_bf16x3(fp, q, n, depth):
    """BF16x3 arithmetic against the float64 oracle on the same float32 gates
    (about 2^-16 per product)."""
    ens = (QUDIT, n, depth, q)
    seed = synth.workload_seed(95 + q, depth) + n
    got = gpu_traces(fp, ens, 16, seed, 2)
    c64 = gpu_traces(fp, ens, 16, seed, 1)
    want = oracle_traces(n, q, depth, seed, 16, 1)
    rms = math.sqrt(float(np.mean(np.abs(want) ** 2)))
    r = np.abs(got - want) / np.maximum(np.abs(want), 1e-3 * rms)
    assert np.median(r) <= 2e-4 and r.max() <= 5e-3, (float(np.median(r)), float(r.max()))
    assert not np.array_equal(got, c64)
