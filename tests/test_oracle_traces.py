"""Pins for the oracle's trace contractions (CPU only)."""

import numpy as np

import synth
from oracle import ancilla, closed_forms, dense, mpo, sampler

BW, LR, HEA = sampler.BRICKWORK, sampler.LOCAL_RANDOM, sampler.HEA


def _kron_unitary(circ):
    """Independent construction: each gate embedded with np.kron, product in time order."""
    n = circ["n"]
    u = np.eye(2 ** n, dtype=np.complex128)
    for bond, g in circ["gates"]:
        full = np.kron(np.kron(np.eye(2 ** bond), g), np.eye(2 ** (n - bond - 2)))
        u = full @ u
    return u


def _random_circuit(seed, n, ngates):
    g = synth.complex_gaussian(seed, (ngates, 4, 4))
    b = synth.rng(seed + 1).integers(0, n - 1, ngates)
    return {"ansatz": LR, "n": n, "gates": [(int(b[i]), g[i]) for i in range(ngates)]}


def test_dense_matches_kron_construction():
    for seed in range(3):
        cu = _random_circuit(100 + seed, 4, 7)
        cv = _random_circuit(200 + seed, 4, 5)
        want = np.sum(np.conj(_kron_unitary(cu)) * _kron_unitary(cv))
        assert abs(dense.trace_pair(cu, cv) - want) < 1e-10 * abs(want)


def test_dense_trace_single_gate_matches_definition():
    # n = 2, one gate each: Tr(U^dagger V) = sum_ab conj(U_ab) V_ab.
    g1, g2 = synth.complex_gaussian(7, (2, 4, 4))
    cu = {"ansatz": LR, "n": 2, "gates": [(0, g1)]}
    cv = {"ansatz": LR, "n": 2, "gates": [(0, g2)]}
    assert abs(dense.trace_pair(cu, cv) - np.trace(g1.conj().T @ g2)) < 1e-12


def test_identical_circuits_give_dimension():
    p = sampler.sample_pairs(BW, 5, 3, 1, 0, 1)[0]
    assert abs(dense.trace_pair(p[0], p[0]) - 32.0) < 1e-11


def test_one_gate_difference_identity():
    p = sampler.sample_pairs(LR, 6, 12, 2, 0, 2)
    cu = p[0][0]
    cv = {"ansatz": LR, "n": 6, "gates": list(cu["gates"])}
    bond, g = cu["gates"][5]
    g2 = p[1][1]["gates"][0][1]
    cv["gates"][5] = (bond, g2)
    want = closed_forms.one_gate_difference(6, g, g2)
    assert abs(dense.trace_pair(cu, cv) - want) < 1e-11 * max(1.0, abs(want))


def test_brickwork_depth1_product():
    for n in (4, 5):
        for cu, cv in sampler.sample_pairs(BW, n, 1, 3, 0, 3):
            assert abs(dense.trace_pair(cu, cv) - closed_forms.brickwork_depth1_trace(cu, cv)) < 1e-11


def test_hea_one_layer_closed_form():
    for cu, cv in sampler.sample_pairs(HEA, 5, 1, 4, 0, 3):
        want = closed_forms.hea_one_layer_trace(cu, cv)
        assert abs(dense.trace_pair(cu, cv) - want) < 1e-11


def test_ancilla_tensor_identity():
    assert np.allclose(ancilla.bottom_tensor_identity(), 0.5 * np.eye(2))


def test_ancilla_matches_dense():
    cases = [sampler.sample_pairs(BW, 4, 3, 5, 0, 2), sampler.sample_pairs(LR, 5, 9, 6, 0, 2),
             sampler.sample_pairs(HEA, 4, 2, 7, 0, 2)]
    for pairs in cases:
        for cu, cv in pairs:
            a, d = ancilla.trace_pair(cu, cv), dense.trace_pair(cu, cv)
            assert abs(a - d) < 1e-10 * max(1.0, abs(d))


def test_mpo_matches_dense_small():
    cases = [sampler.sample_pairs(BW, 6, 4, 8, 0, 3), sampler.sample_pairs(LR, 7, 14, 9, 0, 3),
             sampler.sample_pairs(HEA, 6, 3, 10, 0, 3)]
    for pairs in cases:
        for cu, cv in pairs:
            m, d = mpo.trace_pair(cu, cv), dense.trace_pair(cu, cv)
            assert abs(m - d) < 1e-10 * max(1.0, abs(d))
    # non-unitary gates: no cancellation from unitarity can hide an error
    for s in range(3):
        cu, cv = _random_circuit(300 + s, 5, 9), _random_circuit(400 + s, 5, 8)
        m, d = mpo.trace_pair(cu, cv), dense.trace_pair(cu, cv)
        assert abs(m - d) < 1e-10 * abs(d)


def test_mpo_wide_identities():
    # one-gate difference deep inside a 30-qubit local random circuit
    p = sampler.sample_pairs(LR, 30, 40, 11, 0, 2)
    cu = p[0][0]
    cv = {"ansatz": LR, "n": 30, "gates": list(cu["gates"])}
    bond, g = cu["gates"][20]
    g2 = p[1][0]["gates"][3][1]
    cv["gates"][20] = (bond, g2)
    want = closed_forms.one_gate_difference(30, g, g2)
    assert abs(mpo.trace_pair(cu, cv) - want) < 1e-9 * abs(want)
    # brickwork depth 1 at n = 50
    cu, cv = sampler.sample_pairs(BW, 50, 1, 12, 0, 1)[0]
    want = closed_forms.brickwork_depth1_trace(cu, cv)
    assert abs(mpo.trace_pair(cu, cv) - want) < 1e-9 * abs(want)
    # HEA one layer at n = 40
    cu, cv = sampler.sample_pairs(HEA, 40, 1, 13, 0, 1)[0]
    want = closed_forms.hea_one_layer_trace(cu, cv)
    assert abs(mpo.trace_pair(cu, cv) - want) < 1e-9 * max(abs(want), 1e-30)
