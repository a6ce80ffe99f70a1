"""Per-pair tolerance of a trace against the oracle.

|dTr| <= TOL * max(|Tr|, FLOOR * rms), rms over the oracle's traces of the
compared set.

complex128: TOL 1e-12, FLOOR 1e-3.

complex64: TOL 1e-5, FLOOR 1.  A float32 contraction's error is absolute on
the scale of the traces: every operation rounds at the level of the
register's entries, and a trace that nearly cancels keeps that error while
its own size shrinks.  Measured absolute errors reach 1.4e-6 x rms at n = 20,
depth 6 (about 23 float32 ulps of the typical trace; a CPU emulation of the
same programs in complex64 gives the same sizes, and complex128 meets 1e-12
on the same pairs), so a pair with |Tr| = 0.1 x rms already shows 1.4e-5.
Pairs at or above the rms trace are held to 1e-5 relative, the others to
1e-5 x rms absolute; every F^(k) of a compared batch is held to 1e-5
relative separately.
"""

import math

import numpy as np

TOL = {0: 1e-12, 1: 1e-5}
FLOOR = {0: 1e-3, 1: 1.0}


def floored(got, want, prec):
    """Per-pair floored relative errors (array)."""
    got = np.asarray(got, dtype=np.complex128)
    want = np.asarray(want, dtype=np.complex128)
    rms = math.sqrt(float(np.mean(np.abs(want) ** 2))) if want.size else 1.0
    return np.abs(got - want) / np.maximum(np.abs(want), FLOOR[prec] * rms)


def max_err(got, want, prec):
    e = floored(got, want, prec)
    return float(e.max()) if e.size else 0.0
