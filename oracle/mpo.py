"""MPO-zip trace oracle for circuits too wide for dense matrices.

TEST INFRASTRUCTURE (CPU oracle; see oracle/__init__.py).

The paper evaluates the trace network of Fig. 3a by contracting along the
qubit direction so that few indices are exposed (Sec. II.A) and notes that
the cost is linear in n and exponential in depth (Sec. II.A, Methods A).
This oracle follows a different route from the GPU sweep on purpose: U and V
are never merged.  Each circuit becomes a matrix product operator by the exact
block split of every two-qubit gate,
    G = sum_{p,q} |p><q| (on qubit j)  (x)  G^{(pq)} (on qubit j+1),
    G^{(pq)}[a, b] = G[2p + a, 2q + b],
(CZ uses its exact rank-2 split |p><p| (x) Z^p, CNOT with control j its split
|p><p| (x) X^p), so qubit j carries the
time-ordered product of its factors, indexed by one bond index per gate on
its left and right.  Then
    Tr(U^dagger V) = sum over bond indices of prod_j Tr(A^U_j^dagger A^V_j),
evaluated left to right with an environment E_j[R^U, R^V].
All arithmetic is complex128.
"""

import numpy as np

from .sampler import CNOT, HEA, PAULI_CNOT, PAULI_HEA, hea_gate_list, pauli_gate_list

_PQ = np.zeros((4, 2, 2), dtype=np.complex128)
for _p in range(2):
    for _q in range(2):
        _PQ[2 * _p + _q, _p, _q] = 1.0
_PP = np.zeros((2, 2, 2), dtype=np.complex128)
_PP[0, 0, 0] = 1.0
_PP[1, 1, 1] = 1.0
_ZP = np.array([np.eye(2), np.diag([1.0, -1.0])], dtype=np.complex128)
_XP = np.array([np.eye(2), [[0.0, 1.0], [1.0, 0.0]]], dtype=np.complex128)


def _events(circ):
    """Time-ordered events: ('1q', q, M) or ('2q', bond, left_stack, right_stack)."""
    ev = []
    if circ["ansatz"] in PAULI_HEA:
        right = _XP if circ["ansatz"] == PAULI_CNOT else _ZP
        for kind, q, g in pauli_gate_list(circ):
            ev.append(("1q", q, g) if kind == "1q" else ("2q", q, _PP, right))
        return ev
    if circ["ansatz"] == HEA:
        for op in hea_gate_list(circ):
            if op[0] == "1q":
                ev.append(("1q", op[1], op[2]))
            else:
                ev.append(("2q", op[1], _PP, _ZP))
        return ev
    for bond, g in circ["gates"]:
        g = np.asarray(g, dtype=np.complex128)
        right = np.empty((4, 2, 2), dtype=np.complex128)
        for p in range(2):
            for q in range(2):
                right[2 * p + q] = g[2 * p:2 * p + 2, 2 * q:2 * q + 2]
        ev.append(("2q", bond, _PQ, right))
    return ev


def site_tensors(circ):
    """Per-qubit MPO tensors as arrays of shape (dim L, dim R, 2, 2)."""
    n = circ["n"]
    ev = _events(circ)
    tens = []
    for j in range(n):
        t = np.eye(2, dtype=np.complex128)
        axes = []                      # ('L' or 'R', event index) per leading axis
        for ei, e in enumerate(ev):
            if e[0] == "1q":
                if e[1] == j:
                    t = np.einsum("ab,...bc->...ac", e[2], t)
            else:
                b = e[1]
                if b == j:             # left part acts on qubit j
                    t = np.einsum("kab,...bc->...kac", e[2], t)
                    axes.append(("R", ei))
                elif b == j - 1:       # right part acts on qubit j
                    t = np.einsum("kab,...bc->...kac", e[3], t)
                    axes.append(("L", ei))
        lax = [i for i, a in enumerate(axes) if a[0] == "L"]
        rax = [i for i, a in enumerate(axes) if a[0] == "R"]
        nl = len(axes)
        t = np.transpose(t, lax + rax + [nl, nl + 1])
        dl = int(np.prod([t.shape[i] for i in range(len(lax))])) if lax else 1
        dr = int(np.prod([t.shape[len(lax) + i] for i in range(len(rax))])) if rax else 1
        tens.append(t.reshape(dl, dr, 2, 2))
    return tens


def trace_pair(cu, cv):
    au = site_tensors(cu)
    av = site_tensors(cv)
    env = np.ones((1, 1), dtype=np.complex128)
    for j in range(cu["n"]):
        a, b = au[j], av[j]
        # x[RU, LV, s, t] = sum_LU conj(a[LU, RU, s, t]) env[LU, LV]
        x = np.tensordot(np.conj(a), env, axes=([0], [0]))        # (RU, s, t, LV)
        # env'[RU, RV] = sum_{LV, s, t} x[RU, s, t, LV] b[LV, RV, s, t]
        env = np.tensordot(x, b, axes=([3, 1, 2], [0, 2, 3]))
    return complex(env[0, 0])


def traces(pairs):
    return np.array([trace_pair(a, b) for a, b in pairs], dtype=np.complex128)
