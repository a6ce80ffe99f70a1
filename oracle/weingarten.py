"""Exact brickwork frame potential by the Weingarten permutation transfer.

TEST INFRASTRUCTURE (CPU oracle; see oracle/__init__.py).

F^(k) = E_{U,V} |Tr(U^dagger V)|^{2k} = Tr(M^dagger M) with M the k-th
moment operator E[U^{(x)k} (x) conj(U)^{(x)k}] (frame-potential definition,
Sec. I.A).  For a brickwork of independent Haar U(4) gates (Fig. 2a), M is
the product of its layer operators, and each Haar gate contributes the
orthogonal projector onto the span of the permutation operators,
    P = sum_{s,t} Wg(s, t) |s s>> <<t t|,   Wg = pinv(G4),
    G4[s, t] = 4^{cycles(s^-1 t)},   <<t|a>>_(one qubit) = 2^{cycles(t^-1 a)}.
With layer 1 on even bonds, Tr(M^dagger M) = Tr((P_e P_o)^{D-1}) for D >= 2
(the projectors are idempotent) and Tr(P_e) for D = 1.  The trace is
evaluated on the span of per-qubit permutation labels left by P_e P_o, with
the Gram correction Tr(Y^m) = Tr(pinv(G_S) G_S M_S^m) so that linearly
dependent labels (k > d) are handled exactly.

This is an exact (deterministic) value for the ensemble; it is used to check
Monte Carlo estimates, and is itself pinned by F^(1) = 1, the D = 1 product,
the paper's analytic bound for k = 2 (Sec. I.A) and the Haar limit.
"""

import itertools

import numpy as np


def _perms(k):
    return list(itertools.permutations(range(k)))


def _cycles(p):
    seen = [False] * len(p)
    c = 0
    for i in range(len(p)):
        if not seen[i]:
            c += 1
            j = i
            while not seen[j]:
                seen[j] = True
                j = p[j]
    return c


def _inv(p):
    q = [0] * len(p)
    for i, x in enumerate(p):
        q[x] = i
    return tuple(q)


def _compose(a, b):            # (a o b)(i) = a[b[i]]
    return tuple(a[b[i]] for i in range(len(a)))


def gram(k, d):
    ps = _perms(k)
    g = np.empty((len(ps), len(ps)))
    for i, s in enumerate(ps):
        si = _inv(s)
        for j, t in enumerate(ps):
            g[i, j] = float(d) ** _cycles(_compose(si, t))
    return g


def gate_transfer(k):
    """K[s, a, b] = sum_t Wg(s, t) <<t|a>>_2 <<t|b>>_2 for one Haar U(4) gate."""
    g4 = gram(k, 4)
    g2 = gram(k, 2)
    wg = np.linalg.pinv(g4)
    return np.einsum("st,ta,tb->sab", wg, g2, g2)


def _apply_gate(t, kmat, q):
    """Apply a gate on qubits (q, q+1) to a batch of label tensors t[batch, q0..q_{n-1}]."""
    nax = t.ndim
    a, b = 1 + q, 2 + q
    moved = np.moveaxis(t, (a, b), (nax - 2, nax - 1))
    out = np.einsum("sab,...ab->...s", kmat, moved)
    m = kmat.shape[0]
    full = np.zeros(out.shape[:-1] + (m, m))
    idx = np.arange(m)
    full[..., idx, idx] = out
    return np.moveaxis(full, (nax - 2, nax - 1), (a, b))


def brickwork_frame_potential(n, depth, k):
    """Exact F^(k) of the n-qubit brickwork of the given depth (Haar U(4) gates)."""
    m = len(_perms(k))
    g4 = gram(k, 4)
    g2 = gram(k, 2)
    even = list(range(0, n - 1, 2))
    odd = list(range(1, n - 1, 2))
    if depth == 1:
        rank = np.trace(np.linalg.pinv(g4) @ g4)
        return float(rank ** len(even) * (4.0 ** k) ** (n % 2))
    kmat = gate_transfer(k)
    # Spanning set S of range(P_e P_o): one label per even gate, plus one label
    # for a qubit that no even gate touches (odd n: the last qubit).
    free = list(even) + ([n - 1] if n % 2 else [])
    configs = list(itertools.product(range(m), repeat=len(free)))
    ns = len(configs)
    t = np.zeros((ns,) + (m,) * n)
    for ci, cfg in enumerate(configs):
        lab = [0] * n
        for (slot, lbl) in zip(free, cfg):
            lab[slot] = lbl
            if slot in even:
                lab[slot + 1] = lbl
        t[(ci,) + tuple(lab)] = 1.0
    for q in odd:
        t = _apply_gate(t, kmat, q)
    for q in even:
        t = _apply_gate(t, kmat, q)
    # Read coefficients back on S.
    mat = np.empty((ns, ns))
    for ci, cfg in enumerate(configs):
        lab = [0] * n
        for (slot, lbl) in zip(free, cfg):
            lab[slot] = lbl
            if slot in even:
                lab[slot + 1] = lbl
        mat[ci, :] = t[(slice(None),) + tuple(lab)]
    # Gram matrix of S.
    gs = np.ones((ns, ns))
    for fi, slot in enumerate(free):
        gf = g4 if slot in even else g2
        li = np.array([c[fi] for c in configs])
        gs *= gf[np.ix_(li, li)]
    proj = np.linalg.pinv(gs) @ gs
    return float(np.trace(proj @ np.linalg.matrix_power(mat, depth - 1)))


def brickwork_bound_k2(n, layers, q=2):
    """The paper's analytic upper bound on F^(2) for the brickwork (Sec. I.A)."""
    ng = n // 2
    return 2.0 * (1.0 + (2.0 * q / (q * q + 1.0)) ** (2 * (layers - 1))) ** (ng - 1)
