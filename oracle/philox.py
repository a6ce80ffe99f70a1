"""Philox4x32-10 counter-based generator, written from its published definition.

TEST INFRASTRUCTURE: this package is the CPU oracle.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the HIP path.

Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11): a 128-bit counter (c0..c3) and a 64-bit
key (k0, k1).  One round computes the two 32x32->64 products
M0*c0 and M1*c2 and forms
    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0)),
and the key is bumped by the Weyl constants between rounds.

The paper draws its gate parameters with PyTorch (Methods, "Sampling U(d^2)");
it fixes no generator, so this counter-based one is the reading used here.
"""

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Vectorised Philox4x32-10.

    ctr: uint array of shape (..., 4); key: uint array broadcastable to (..., 2).
    Returns uint32 array of shape (..., 4).
    """
    c = np.asarray(ctr, dtype=np.uint64) & MASK
    k = np.asarray(key, dtype=np.uint64) & MASK
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0 = np.broadcast_to(k[..., 0], c0.shape).copy()
    k1 = np.broadcast_to(k[..., 1], c0.shape).copy()
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0          # < 2^64, exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def key_from_seed(seed):
    """64-bit seed -> (k0, k1) = (low word, high word)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint64)


def make_counter(word, item, pair, circuit):
    """Counter layout shared by every draw of the sampler:
    (word, item, pair low 32 bits, pair bits 32..62 | circuit << 31)."""
    word = np.asarray(word, dtype=np.uint64)
    item = np.asarray(item, dtype=np.uint64)
    pair = np.asarray(pair, dtype=np.uint64)
    circuit = np.asarray(circuit, dtype=np.uint64)
    shape = np.broadcast_shapes(word.shape, item.shape, pair.shape, circuit.shape)
    out = np.empty(shape + (4,), dtype=np.uint64)
    out[..., 0] = word
    out[..., 1] = item
    out[..., 2] = pair & MASK
    out[..., 3] = ((pair >> np.uint64(32)) & np.uint64(0x7FFFFFFF)) | (circuit << np.uint64(31))
    return out
