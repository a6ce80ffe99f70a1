"""Qudit brickwork oracle: local dimension q > 2 (Sec. II.A of the paper, the
generalisation to qudits with the generalised Hadamard and SUM gates).

TEST INFRASTRUCTURE (CPU oracle; see oracle/__init__.py).

Ensemble: n qudits of dimension q on an open chain; layer t = 1..D acts on
the pairs (j, j+1) with j = t-1 (mod 2); every gate is Haar on U(q^2).  A
two-qudit gate on (j, j+1) uses the composite index q x_j + x_{j+1} (qudit j
the more significant digit), rows = outputs.  Tr(U^dagger V) is the
Frobenius inner product of the dense q^n x q^n unitaries (n small), or the
MPO zip of the two circuits (block split G = sum_{a,b} |a><b| (x) G^{(ab)},
G^{(ab)}[c, d] = G[q a + c, q b + d]).  The Haar value is F^(k) = #{pi in S_k
: longest increasing subsequence <= q^n}, i.e. k! for q^n >= k.

Draws (philox.py counter stream, as for the qubit gates): gate g of circuit
c of pair p takes, for its q^4 complex Gaussian entries w = 0..q^4-1 (entry
(w // q^2, w % q^2)), the block with counter (w, g, pair low, pair high |
c << 31) and key = seed: Box-Muller of U53(x0, x1), U53(x2, x3).  Haar
unitary: the QR factor with a positive real R diagonal (Mezzadri 2007).
"""

import numpy as np

from .philox import key_from_seed, make_counter, philox4x32_10
from .sampler import brickwork_layout, u53

QUDIT_BRICKWORK = 5


def haar_gates(seed, q, pairs, circuit, ngates):
    """(num_pairs, ngates, q^2, q^2) complex128 Haar unitaries."""
    pairs = np.asarray(pairs, dtype=np.uint64)
    d = q * q
    w = np.arange(d * d, dtype=np.uint64)
    g = np.arange(ngates, dtype=np.uint64)
    ctr = make_counter(w[None, None, :], g[None, :, None], pairs[:, None, None], circuit)
    x = philox4x32_10(ctr, key_from_seed(seed))
    u1 = u53(x[..., 0], x[..., 1])
    u2 = u53(x[..., 2], x[..., 3])
    z = np.sqrt(-2.0 * np.log(u1)) * np.exp(2j * np.pi * u2)
    z = z.reshape(pairs.size, ngates, d, d)
    out = np.empty_like(z)
    for i in range(pairs.size):
        for k in range(ngates):
            qm, r = np.linalg.qr(z[i, k])
            ph = np.diag(r) / np.abs(np.diag(r))
            out[i, k] = qm * ph[None, :]
    return out


def sample_pairs(n, q, depth, seed, first_pair, num_pairs, fp32=False):
    """List of (U, V) circuits {'n', 'q', 'gates': [(bond, q^2 x q^2)]}."""
    pairs = np.arange(first_pair, first_pair + num_pairs, dtype=np.uint64)
    bonds = brickwork_layout(n, depth)
    mats = []
    for c in (0, 1):
        m = haar_gates(seed, q, pairs, c, len(bonds))
        if fp32:
            m = m.astype(np.complex64).astype(np.complex128)
        mats.append(m)
    return [tuple({"n": n, "q": q, "gates": [(int(b), mats[c][i, k]) for k, b in enumerate(bonds)]}
                  for c in (0, 1)) for i in range(num_pairs)]


def _apply(mat, gate, j, n, q):
    cols = mat.shape[1]
    m = mat.reshape(q ** j, q * q, q ** (n - j - 2), cols)
    return np.einsum("ij,ajbc->aibc", gate, m).reshape(q ** n, cols)


def dense_unitary(circ):
    n, q = circ["n"], circ["q"]
    u = np.eye(q ** n, dtype=np.complex128)
    for b, g in circ["gates"]:
        u = _apply(u, np.asarray(g, dtype=np.complex128), b, n, q)
    return u


def dense_trace(cu, cv):
    return complex(np.sum(np.conj(dense_unitary(cu)) * dense_unitary(cv)))


def _sites(circ):
    n, q = circ["n"], circ["q"]
    left = np.zeros((q * q, q, q), dtype=np.complex128)
    for a in range(q):
        for b in range(q):
            left[q * a + b, a, b] = 1.0
    tens = []
    for j in range(n):
        t = np.eye(q, dtype=np.complex128)
        axes = []
        for ei, (b, g) in enumerate(circ["gates"]):
            g = np.asarray(g, dtype=np.complex128)
            if b == j:
                t = np.einsum("kab,...bc->...kac", left, t)
                axes.append("R")
            elif b == j - 1:
                right = np.empty((q * q, q, q), dtype=np.complex128)
                for a in range(q):
                    for c in range(q):
                        right[q * a + c] = g[q * a:q * a + q, q * c:q * c + q]
                t = np.einsum("kab,...bc->...kac", right, t)
                axes.append("L")
        lax = [i for i, a in enumerate(axes) if a == "L"]
        rax = [i for i, a in enumerate(axes) if a == "R"]
        na = len(axes)
        t = np.transpose(t, lax + rax + [na, na + 1])
        dl = int(np.prod([t.shape[i] for i in range(len(lax))])) if lax else 1
        dr = int(np.prod([t.shape[len(lax) + i] for i in range(len(rax))])) if rax else 1
        tens.append(t.reshape(dl, dr, q, q))
    return tens


def mpo_trace(cu, cv):
    au, av = _sites(cu), _sites(cv)
    env = np.ones((1, 1), dtype=np.complex128)
    for a, b in zip(au, av):
        x = np.tensordot(np.conj(a), env, axes=([0], [0]))
        env = np.tensordot(x, b, axes=([3, 1, 2], [0, 2, 3]))
    return complex(env[0, 0])


def depth1_trace(cu, cv):
    """One layer: the product of Tr(G_U^dagger G_V) over the gates, times q for an untouched qudit."""
    n, q = cu["n"], cu["q"]
    t = 1.0 + 0.0j
    for (b, gu), (_, gv) in zip(cu["gates"], cv["gates"]):
        t *= np.trace(np.conj(np.asarray(gu)).T @ np.asarray(gv))
    return t * (q if n % 2 else 1)
