"""Dense trace oracle: Tr(U^dagger V) from explicit 2^n x 2^n unitaries.

TEST INFRASTRUCTURE (CPU oracle; see oracle/__init__.py).

This is the plain definition: the frame potential is the double average of
|Tr(U^dagger V)|^{2k} (Sec. I.A, frame-potential equation), and the trace of
a product is the Frobenius inner product sum_ab conj(U_ab) V_ab.  Each
circuit's unitary is built by left-multiplying its gates, in time order, onto
the identity.  Basis index = sum_q x_q 2^(n-1-q) (qubit 0 most significant);
a two-qubit gate on bond (q, q+1) uses composite index 2 x_q + x_{q+1} with
rows = outputs and columns = inputs.  Cost O(#gates 4^n): n <= 12.
"""

import numpy as np

from .sampler import HEA, PAULI_HEA, hea_gate_list, pauli_gate_list, CZ


def apply_2q(mat, gate, q, n):
    """mat <- (gate on qubits q, q+1) @ mat, mat of shape (2^n, cols)."""
    cols = mat.shape[1]
    m = mat.reshape(2 ** q, 4, 2 ** (n - q - 2), cols)
    return np.einsum("ij,ajbc->aibc", gate, m).reshape(2 ** n, cols)


def apply_1q(mat, gate, q, n):
    cols = mat.shape[1]
    m = mat.reshape(2 ** q, 2, 2 ** (n - q - 1), cols)
    return np.einsum("ij,ajbc->aibc", gate, m).reshape(2 ** n, cols)


def circuit_unitary(circ, wall=True):
    n = circ["n"]
    u = np.eye(2 ** n, dtype=np.complex128)
    if circ["ansatz"] in PAULI_HEA:
        for kind, q, g in pauli_gate_list(circ, wall):
            u = apply_1q(u, g, q, n) if kind == "1q" else apply_2q(u, g, q, n)
        return u
    if circ["ansatz"] == HEA:
        for op in hea_gate_list(circ):
            if op[0] == "1q":
                u = apply_1q(u, op[2], op[1], n)
            else:
                u = apply_2q(u, CZ, op[1], n)
        return u
    for bond, g in circ["gates"]:
        u = apply_2q(u, np.asarray(g, dtype=np.complex128), bond, n)
    return u


def trace_pair(cu, cv, wall=True):
    """Tr(U^dagger V) for one sampled pair (complex128)."""
    u = circuit_unitary(cu, wall)
    v = circuit_unitary(cv, wall)
    return complex(np.sum(np.conj(u) * v))


def traces(pairs):
    return np.array([trace_pair(a, b) for a, b in pairs], dtype=np.complex128)
