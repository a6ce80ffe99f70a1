"""Ancilla oracle: the trace as a single amplitude (Sec. II.A of the paper).

TEST INFRASTRUCTURE (CPU oracle; see oracle/__init__.py).

The paper prepares n ancilla and n target qubits in |0...0>, applies a
Hadamard to every ancilla and a CNOT from ancilla j to target j (the operator
M), and shows that <Psi| U^dagger V |Psi> = Tr(U^dagger V) / 2^n for
|Psi> = M |0...0>.  This module simulates exactly that 2n-qubit circuit as a
state vector, so it is feasible for n <= 10, and multiplies the amplitude by
2^n (unnormalised trace, so that the Haar value is k!).

Register layout: 2n qubits, ancillas are qubits 0..n-1 and targets are
n..2n-1 (qubit 0 most significant), so the state is a (2^n, 2^n) array
indexed [ancilla basis, target basis].
"""

import numpy as np

from .dense import apply_1q, apply_2q
from .sampler import HEA, PAULI_HEA, hea_gate_list, pauli_gate_list, CZ

H = np.array([[1.0, 1.0], [1.0, -1.0]], dtype=np.complex128) / np.sqrt(2.0)


def _prepare(n):
    """M |0...0>: Hadamards on ancillas, then CNOT(ancilla j -> target j)."""
    psi = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
    psi[0, 0] = 1.0
    # Hadamard on each ancilla acts on axis 0.
    a = psi
    for q in range(n):
        a = apply_1q(a, H, q, n)
    # CNOT ancilla j -> target j: flip target bit j where ancilla bit j is 1.
    out = np.zeros_like(a)
    idx = np.arange(2 ** n)
    for mu in range(2 ** n):
        out[mu, idx ^ mu] = a[mu, idx]
    return out


def _apply_circuit_to_targets(psi, circ, dagger):
    """Apply the circuit (or its inverse) to the target register (axis 1)."""
    n = circ["n"]
    st = psi.T.copy()           # (target, ancilla): gates act on axis 0
    if circ["ansatz"] in PAULI_HEA:
        seq = list(pauli_gate_list(circ))
    elif circ["ansatz"] == HEA:
        ops = hea_gate_list(circ)
        seq = [(op[0], op[1], op[2] if op[0] == "1q" else CZ) for op in ops]
    else:
        seq = [("2q", b, np.asarray(g, dtype=np.complex128)) for b, g in circ["gates"]]
    if dagger:
        seq = [(k, q, np.conj(g).T) for (k, q, g) in reversed(seq)]
    for kind, q, g in seq:
        if kind == "1q":
            st = apply_1q(st, g, q, n)
        else:
            st = apply_2q(st, g, q, n)
    return st.T


def trace_pair(cu, cv):
    n = cu["n"]
    psi = _prepare(n)
    phi = _apply_circuit_to_targets(psi, cv, dagger=False)
    phi = _apply_circuit_to_targets(phi, cu, dagger=True)
    amp = np.vdot(psi.reshape(-1), phi.reshape(-1))
    return complex(amp * 2 ** n)


def traces(pairs):
    return np.array([trace_pair(a, b) for a, b in pairs], dtype=np.complex128)


def bottom_tensor_identity():
    """The bottom tensor of Fig. 3b: sum_m H_{m0} CNOT_{m i 0} CNOT_{m 0 j} H_{0 m}.

    Returns the 2x2 array over (i, j).  CNOT_{k i j} is the three-index CNOT
    tensor of that passage (first index = control, then target output and
    input).  Evaluated with the normalised Hadamard of the same passage the
    sum is delta_ij / 2: the printed right-hand side omits the factor 1/2 per
    qubit that reappears as the 1/2^n of the amplitude-trace relation.
    """
    def cnot(k, i, j):
        return 1.0 if (k == 0 and i == j) or (k == 1 and i != j) else 0.0
    out = np.zeros((2, 2))
    for i in range(2):
        for j in range(2):
            s = 0.0
            for m in range(2):
                s += H[m, 0].real * cnot(m, i, 0) * cnot(m, 0, j) * H[0, m].real
            out[i, j] = s
    return out
