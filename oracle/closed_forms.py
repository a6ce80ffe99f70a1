"""Closed-form traces and frame potentials for special cases.

TEST INFRASTRUCTURE (CPU oracle; see oracle/__init__.py).

Each identity follows from the trace being the Frobenius inner product of
the two circuit unitaries (frame-potential definition, Sec. I.A):
  * U = V: Tr(U^dagger U) = 2^n.
  * U, V equal except one two-qubit gate G vs G': U^dagger V = Y^dagger
    (G^dagger G' (x) I) Y, so Tr = 2^(n-2) Tr_4(G^dagger G').
  * Brickwork, one layer: Tr = prod_gates Tr_4(G_U^dagger G_V), times 2 per
    qubit no gate touches.  Hence F^(k) = (F_U(4)^(k))^floor(n/2) * 4^(k (n mod 2)).
  * Hardware-efficient ansatz, one layer (the CZ ladders cancel inside the
    trace): Tr = prod_q 2 cos(dphi_q / 2) cos(dtheta_q / 2), and with
    uniform angles F^(k) = (C(2k, k)^2 / 4^k)^n.
  * The paper's Pauli-rotation ansatz, one layer: the RY(pi/4) walls and the
    entangling walls cancel inside the trace, leaving prod_q Tr(R_q^U^dagger
    R_q^V) with R = exp(-i theta P / 2): 2 cos((theta_V - theta_U) / 2) for
    equal axes and 2 cos(theta_U / 2) cos(theta_V / 2) for different ones
    (Tr(P Q) = 0).  With uniform axes and angles, per qubit
    E |Tr|^{2k} = C(2k, k) / 3 + (2/3) C(2k, k)^2 / 4^k, so
    F^(1) = (4/3)^n and F^(2) = (7/2)^n.
"""

import math

import numpy as np

from .haar_moments import haar_frame_potential


def one_gate_difference(n, g, g2):
    g = np.asarray(g, dtype=np.complex128)
    g2 = np.asarray(g2, dtype=np.complex128)
    return 2.0 ** (n - 2) * np.trace(np.conj(g).T @ g2)


def brickwork_depth1_trace(cu, cv):
    n = cu["n"]
    touched = set()
    tr = 1.0 + 0j
    for (bu, gu), (bv, gv) in zip(cu["gates"], cv["gates"]):
        assert bu == bv
        touched.update((bu, bu + 1))
        tr *= np.trace(np.conj(np.asarray(gu)).T @ np.asarray(gv))
    return tr * 2.0 ** (n - len(touched))


def brickwork_depth1_frame_potential(n, k):
    return float(haar_frame_potential(k, 4)) ** (n // 2) * 4.0 ** (k * (n % 2))


def hea_one_layer_trace(cu, cv):
    dth = cv["theta"][0] - cu["theta"][0]
    dph = cv["phi"][0] - cu["phi"][0]
    return complex(np.prod(2.0 * np.cos(dph / 2.0) * np.cos(dth / 2.0)))


def hea_one_layer_frame_potential(n, k):
    return (math.comb(2 * k, k) ** 2 / 4.0 ** k) ** n


def pauli_one_layer_trace(cu, cv):
    tu, tv = cu["theta"][0], cv["theta"][0]
    au, av = cu["axis"][0], cv["axis"][0]
    t = 1.0 + 0.0j
    for q in range(len(tu)):
        if au[q] == av[q]:
            t *= 2.0 * math.cos((tv[q] - tu[q]) / 2.0)
        else:
            t *= 2.0 * math.cos(tu[q] / 2.0) * math.cos(tv[q] / 2.0)
    return t


def pauli_one_layer_frame_potential(n, k):
    c = math.comb(2 * k, k)
    return (c / 3.0 + 2.0 * c * c / (3.0 * 4.0 ** k)) ** n
