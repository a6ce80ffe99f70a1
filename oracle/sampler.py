"""Oracle sampler: the three random-circuit ensembles of the paper.

TEST INFRASTRUCTURE (CPU oracle; see oracle/__init__.py).

Ensembles (Results, Fig. 2 of the paper; 1D open chain, q = 2):
  * brickwork ("parallel random unitaries"): layer t = 1..D acts on bonds
    (q, q+1) with q = t-1 (mod 2); every gate is a Haar U(4) matrix.
  * local random: each step applies one Haar U(4) gate on a bond chosen
    uniformly among the n-1 neighbouring pairs.
  * hardware-efficient ansatz: each layer is RY(theta) then RZ(phi) on every
    qubit, then CZ on every bond, with theta, phi ~ U[0, 2pi).
  * the paper's hardware-efficient ansatz (Fig. 2c; Sec. II.C): a wall of
    RY(pi/4) rotations, then per layer a random Pauli rotation
    R_P(theta) = exp(-i theta P / 2) on every qubit (P uniform in {X, Y, Z},
    theta ~ U[0, 2pi)) and two walls of entangling gates, first on the bonds
    (q, q+1) with q even, then with q odd -- each layer has two walls of
    two-qubit gates (Sec. II.C) -- CNOT with control q and target q+1, or
    CZ.

Haar U(4) is drawn as complex Gaussian -> QR -> multiply column a of Q by
R[a,a]/|R[a,a]| (Mezzadri 2007), which is the unique QR factor with a
positive real diagonal in R.  The paper uses a 16-phase EUNN parametrisation
(Methods, "Sampling U(d^2)"); both target the same Haar measure.

Random draws follow one counter stream (Philox4x32-10, see philox.py):
  key = (seed low 32, seed high 32)
  counter = (word, item, pair low 32, pair high 31 | circuit << 31)
  circuit: 0 = U, 1 = V.
  Haar gate g of a circuit: item = g, words w = 0..15 give entry (w//4, w%4)
      of the Gaussian matrix: Philox block -> u1 = U53(x0,x1), u2 = U53(x2,x3)
      -> z = sqrt(-2 ln u1) (cos 2 pi u2 + i sin 2 pi u2).
  Local-random bond of step s: item = s, words w = 16, 17, ...: the 32-bit
      outputs in order, first x < 2^32 - (2^32 mod (n-1)) gives bond x mod (n-1).
  HEA angles of (layer l, qubit q): item = l*n + q, word 0:
      theta = 2 pi U53(x0,x1), phi = 2 pi U53(x2,x3).
  Pauli-rotation HEA, (layer l, qubit q): item = l*n + q, word 0: the axis
      is x mod 3 for the first x of (x0, x1) below 2^32 - 1 (0 if neither
      is; 2^32 - 1 = 3 * 1431655765, so x mod 3 is uniform), 0 = X, 1 = Y,
      2 = Z; theta = 2 pi U53(x2, x3).
  U53(a, b) = ((a >> 5) * 2^26 + (b >> 6) + 1) * 2^-53, exact in float64 and
      in (0, 1], so the logarithm of Box-Muller is always finite.
Gates are computed in float64 and then stored in the precision's type.
"""

import numpy as np

from .philox import philox4x32_10, key_from_seed, make_counter

BRICKWORK, LOCAL_RANDOM, HEA, PAULI_CNOT, PAULI_CZ = 0, 1, 2, 3, 4
PAULI_HEA = (PAULI_CNOT, PAULI_CZ)


def u53(a, b):
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    return ((a >> np.uint64(5)).astype(np.float64) * 67108864.0
            + (b >> np.uint64(6)).astype(np.float64) + 1.0) * 2.0 ** -53


def gaussian_entries(seed, pair, circuit, item):
    """Complex Gaussian 4x4 matrices for arrays of (pair, circuit, item)."""
    pair = np.asarray(pair, dtype=np.uint64)
    item = np.asarray(item, dtype=np.uint64)
    circuit = np.asarray(circuit, dtype=np.uint64)
    shape = np.broadcast_shapes(pair.shape, item.shape, circuit.shape)
    w = np.arange(16, dtype=np.uint64).reshape((1,) * len(shape) + (16,))
    ctr = make_counter(w, item[..., None], pair[..., None], circuit[..., None])
    x = philox4x32_10(ctr, key_from_seed(seed))
    u1 = u53(x[..., 0], x[..., 1])
    u2 = u53(x[..., 2], x[..., 3])
    r = np.sqrt(-2.0 * np.log(u1))
    z = r * np.cos(2.0 * np.pi * u2) + 1j * (r * np.sin(2.0 * np.pi * u2))
    return z.reshape(shape + (4, 4))


def haar_from_gaussian(z):
    """QR with the phase fix; z has shape (..., 4, 4)."""
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    ad = np.abs(d)
    ph = np.where(ad > 0, d / np.where(ad > 0, ad, 1.0), 1.0)
    return q * ph[..., None, :]


def brickwork_layout(n, depth):
    """Bond of every gate of one brickwork circuit, in time order."""
    bonds = []
    for t in range(1, depth + 1):
        bonds.extend(range((t - 1) % 2, n - 1, 2))
    return np.array(bonds, dtype=np.int64)


def local_random_bonds(seed, n, steps, pairs, circuit):
    """Unbiased uniform bond per step (rejection from 32-bit words)."""
    m = n - 1
    limit = (1 << 32) - ((1 << 32) % m)
    pairs = np.asarray(pairs, dtype=np.uint64)
    out = np.empty((pairs.size, steps), dtype=np.int64)
    key = key_from_seed(seed)
    for pi, p in enumerate(pairs):
        for s in range(steps):
            w = 16
            found = None
            while found is None:
                x = philox4x32_10(make_counter(w, s, p, circuit), key)
                for v in x:
                    if int(v) < limit:
                        found = int(v) % m
                        break
                w += 1
            out[pi, s] = found
    return out


def hea_angles(seed, n, layers, pairs, circuit):
    """theta, phi of shape (num_pairs, layers, n)."""
    pairs = np.asarray(pairs, dtype=np.uint64)
    l = np.arange(layers, dtype=np.uint64)[:, None]
    q = np.arange(n, dtype=np.uint64)[None, :]
    item = l * np.uint64(n) + q
    ctr = make_counter(0, item[None], pairs[:, None, None], circuit)
    x = philox4x32_10(ctr, key_from_seed(seed))
    theta = 2.0 * np.pi * u53(x[..., 0], x[..., 1])
    phi = 2.0 * np.pi * u53(x[..., 2], x[..., 3])
    return theta, phi


def pauli_params(seed, n, layers, pairs, circuit):
    """theta (float64) and axis (int, 0 = X, 1 = Y, 2 = Z) of shape
    (num_pairs, layers, n) for the Pauli-rotation HEA."""
    pairs = np.asarray(pairs, dtype=np.uint64)
    l = np.arange(layers, dtype=np.uint64)[:, None]
    q = np.arange(n, dtype=np.uint64)[None, :]
    item = l * np.uint64(n) + q
    ctr = make_counter(0, item[None], pairs[:, None, None], circuit)
    x = philox4x32_10(ctr, key_from_seed(seed))
    top = np.uint64(0xFFFFFFFF)
    x0, x1 = x[..., 0].astype(np.uint64), x[..., 1].astype(np.uint64)
    axis = np.where(x0 < top, x0 % np.uint64(3), np.where(x1 < top, x1 % np.uint64(3), np.uint64(0)))
    theta = 2.0 * np.pi * u53(x[..., 2], x[..., 3])
    return theta, axis.astype(np.int64)


def _store(a, precision_is_fp32):
    if precision_is_fp32:
        return a.astype(np.complex64).astype(np.complex128) if np.iscomplexobj(a) \
            else a.astype(np.float32).astype(np.float64)
    return a


def sample_pairs(ansatz, n, depth, seed, first_pair, num_pairs, fp32=False):
    """Sample num_pairs (U, V) pairs; returns a list of circuit pairs.

    Each circuit is a dict with 'ansatz', 'n' and either
      'gates': list of (bond, 4x4 complex128) in time order, or
      'theta', 'phi': (layers, n) float64 arrays (HEA), or
      'theta' (float64), 'axis' (int): (layers, n) arrays (Pauli-rotation HEA).
    With fp32=True, stored values are rounded to float32 exactly as the
    library stores them and then widened back to float64 exactly.
    """
    pairs = np.arange(first_pair, first_pair + num_pairs, dtype=np.uint64)
    out = []
    if ansatz in PAULI_HEA:
        par = [pauli_params(seed, n, depth, pairs, c) for c in (0, 1)]
        for i in range(num_pairs):
            out.append(tuple({"ansatz": ansatz, "n": n, "theta": _store(par[c][0][i], fp32),
                              "axis": par[c][1][i].copy()} for c in (0, 1)))
        return out
    if ansatz == HEA:
        ang = [hea_angles(seed, n, depth, pairs, c) for c in (0, 1)]
        for i in range(num_pairs):
            pr = []
            for c in (0, 1):
                pr.append({"ansatz": HEA, "n": n,
                           "theta": _store(ang[c][0][i], fp32),
                           "phi": _store(ang[c][1][i], fp32)})
            out.append(tuple(pr))
        return out
    if ansatz == BRICKWORK:
        bonds = np.broadcast_to(brickwork_layout(n, depth), (num_pairs, len(brickwork_layout(n, depth))))
        bonds = [bonds, bonds]
    elif ansatz == LOCAL_RANDOM:
        bonds = [local_random_bonds(seed, n, depth, pairs, c) for c in (0, 1)]
    else:
        raise ValueError("unknown ansatz")
    ngates = bonds[0].shape[1]
    mats = []
    for c in (0, 1):
        z = gaussian_entries(seed, pairs[:, None], c, np.arange(ngates, dtype=np.uint64)[None, :])
        mats.append(_store(haar_from_gaussian(z), fp32))
    for i in range(num_pairs):
        pr = []
        for c in (0, 1):
            pr.append({"ansatz": ansatz, "n": n,
                       "gates": [(int(bonds[c][i, g]), mats[c][i, g]) for g in range(ngates)]})
        out.append(tuple(pr))
    return out


def hea_gate_list(circ):
    """HEA circuit as a time-ordered list of ('1q', q, 2x2) and ('cz', bond)."""
    n = circ["n"]
    theta, phi = circ["theta"], circ["phi"]
    ops = []
    for l in range(theta.shape[0]):
        for q in range(n):
            ops.append(("1q", q, rz(phi[l, q]) @ ry(theta[l, q])))
        for b in range(n - 1):
            ops.append(("cz", b))
    return ops


def ry(t):
    c, s = np.cos(t / 2.0), np.sin(t / 2.0)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def rz(p):
    return np.array([[np.exp(-0.5j * p), 0.0], [0.0, np.exp(0.5j * p)]], dtype=np.complex128)


CZ = np.diag([1.0, 1.0, 1.0, -1.0]).astype(np.complex128)


def pauli_rotation(axis, theta):
    """R_P(theta) = exp(-i theta P / 2) = cos(theta/2) I - i sin(theta/2) P."""
    c, s_ = np.cos(theta / 2.0), np.sin(theta / 2.0)
    p = (PAULI_X, PAULI_Y, PAULI_Z)[int(axis)]
    return c * np.eye(2, dtype=np.complex128) - 1j * s_ * p


PAULI_X = np.array([[0.0, 1.0], [1.0, 0.0]], dtype=np.complex128)
PAULI_Y = np.array([[0.0, -1.0j], [1.0j, 0.0]], dtype=np.complex128)
PAULI_Z = np.array([[1.0, 0.0], [0.0, -1.0]], dtype=np.complex128)
# control = qubit b (the more significant bit of the composite index), target b + 1
CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.complex128)


def pauli_gate_list(circ, wall=True):
    """Pauli-rotation HEA as a time-ordered list of ('1q', q, 2x2) and
    ('2q', bond, 4x4): the RY(pi/4) wall (omitted with wall=False), then per
    layer the rotations, the entangling wall on even bonds, then on odd bonds."""
    n = circ["n"]
    theta, axis = circ["theta"], circ["axis"]
    ent = CNOT if circ["ansatz"] == PAULI_CNOT else CZ
    ops = []
    if wall:
        for q in range(n):
            ops.append(("1q", q, ry(np.pi / 4.0)))
    for l in range(theta.shape[0]):
        for q in range(n):
            ops.append(("1q", q, pauli_rotation(axis[l, q], theta[l, q])))
        for first in (0, 1):
            for b in range(first, n - 1, 2):
                ops.append(("2q", b, ent))
    return ops
