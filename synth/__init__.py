"""Seeded synthetic inputs shared by the tests, the bench and the oracle.

This module holds none of the method's arithmetic: it only draws raw numbers
(numpy's PCG64 stream, seeded) and names the workload recipes.  Random
quantities that the method itself draws (gate matrices, bonds, angles) are
produced by each side's own implementation of the counter-based generator;
the arrays here feed paths that take arbitrary tensors (contraction of
non-unitary gate arrays, reductions of arbitrary trace vectors, surrogate
network batches).
"""

import numpy as np

BRICKWORK, LOCAL_RANDOM, HEA, PAULI_CNOT, PAULI_CZ, BRICKWORK_QUDIT = 0, 1, 2, 3, 4, 5
C128, C64, BF16X3 = 0, 1, 2


def workload_seed(config_id, index):
    """Seed of one (configuration, depth-or-step) workload."""
    return ((0xF9000000 + int(config_id)) & 0xFFFFFFFF) | (int(index) << 32)


# Workload recipes: (name, ansatz, n, depth values, pairs per depth, k_max, precision).
WORKLOADS = {
    "brickwork_n6": dict(config_id=1, ansatz=BRICKWORK, n=6, depths=list(range(1, 7)),
                         pairs=2000, k_max=2, precision=C128),
    "brickwork_n20": dict(config_id=2, ansatz=BRICKWORK, n=20, depths=list(range(2, 11)),
                          pairs=100000, k_max=3, precision=C64),
    "hea_n30_mixed": dict(config_id=3, ansatz=HEA, n=30, depths=list(range(1, 9)),
                          pairs=100000, k_max=2, precision=C64),
    "local_random_n50": dict(config_id=4, ansatz=LOCAL_RANDOM, n=50,
                             depths=list(range(50, 801, 50)), pairs=10000, k_max=3,
                             precision=C64),
    "hea_n40_cv": dict(config_id=5, ansatz=HEA, n=40, depths=[6], pairs=10000, k_max=2,
                       precision=C64),
}


def rng(seed):
    return np.random.default_rng(np.uint64(seed & 0xFFFFFFFFFFFFFFFF))


def complex_gaussian(seed, shape):
    """Complex Gaussian array (unit variance per component), complex128."""
    g = rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def heavy_tailed_traces(seed, num, scale=1.0):
    """Complex values whose |.|^2 is exponential with occasional large outliers."""
    g = rng(seed)
    z = (g.standard_normal(num) + 1j * g.standard_normal(num)) * np.sqrt(0.5) * scale
    big = g.random(num) < 0.001
    z[big] *= 30.0
    return z


def uniform(seed, shape, lo=0.0, hi=1.0):
    return rng(seed).uniform(lo, hi, size=shape)


def normal(seed, shape, std=1.0):
    return rng(seed).standard_normal(shape) * std
