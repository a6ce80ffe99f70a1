"""BF16x3 precision (float32 storage, every real product of the contraction as
three bf16 products with float32 accumulation) against the float64 oracle on
the same float32 gates.  Its error is a property of the arithmetic, about
2^-16 per product; the bounds below are loose enough for that and tight
enough to fail for an arithmetic slip (a dropped term or a wrong split gives
errors of order one, a silent fall-back to float32 gives results equal to
FP_C64)."""

import math

import numpy as np
import pytest
import torch

import synth
from oracle import dense, estimator, sampler

pytestmark = pytest.mark.gpu

BF16X3 = 2


@pytest.fixture(scope="module")
def fp():
    import paper_2205_09900_amd as m
    assert torch.cuda.is_available()
    return m


def traces(fp, ens, n, seed, prec):
    g = fp.sample(ens, n, seed, 0, prec)
    tr = fp.contract(ens, g, n, prec)
    torch.cuda.synchronize()
    return tr.cpu().numpy()


def rel_errors(got, want):
    rms = math.sqrt(float(np.mean(np.abs(want) ** 2)))
    floor = np.maximum(np.abs(want), 1e-3 * rms)
    return np.abs(got - want) / floor


@pytest.mark.parametrize("ens,n", [((0, 6, 4), 64), ((0, 8, 6), 32), ((1, 8, 24), 64), ((1, 10, 40), 24),
                                   ((2, 6, 3), 64), ((2, 5, 6), 32)])
def test_bf16x3_vs_dense(fp, ens, n):
    seed = synth.workload_seed(7, ens[2]) + ens[1]
    got = traces(fp, ens, n, seed, BF16X3)
    c64 = traces(fp, ens, n, seed, fp.C64)
    want = dense.traces(sampler.sample_pairs(ens[0], ens[1], ens[2], seed, 0, n, fp32=True))
    r = rel_errors(got, want)
    assert np.median(r) <= 2e-4 and r.max() <= 5e-3, (float(np.median(r)), float(r.max()))
    assert not np.array_equal(got, c64)  # the three-product arithmetic is what ran
    fg, _ = estimator.frame_potential(got, 2)
    fw, _ = estimator.frame_potential(want, 2)
    for k in range(2):
        assert abs(fg[k] - fw[k]) <= 2e-3 * fw[k], (k, fg[k], fw[k])


def test_bf16x3_local_random_n50(fp):
    """Wide circuits (every sweep class of the local random path) against FP_C64 on
    the same float32 gates: the float32 result is within about 1e-6 of float64
    here, far below the BF16x3 error."""
    ens = (1, 50, 120)
    n = 300
    seed = synth.workload_seed(4, 120)
    g = fp.sample(ens, n, seed, 0, fp.C64)
    got = fp.contract(ens, g, n, BF16X3).cpu().numpy()
    ref = fp.contract(ens, g, n, fp.C64).cpu().numpy()
    r = rel_errors(got, ref)
    assert np.isfinite(got).all()
    assert np.median(r) <= 5e-4 and r.max() <= 3e-2, (float(np.median(r)), float(r.max()))


def test_bf16x3_shared_wide_ops_vs_dense(fp):
    """96 pairs of 8 qubits at 40 steps (the batch of the two-slot-size test):
    the widest pairs run their ops on registers from 2^18 entries as chunks
    shared among workgroups, here with the BF16x3 products."""
    ens, n, seed = (1, 8, 40), 96, 4343
    got = traces(fp, ens, n, seed, BF16X3)
    want = dense.traces(sampler.sample_pairs(1, 8, 40, seed, 0, n, fp32=True))
    r = rel_errors(got, want)
    assert np.median(r) <= 2e-4 and r.max() <= 5e-3, (float(np.median(r)), float(r.max()))


@pytest.mark.parametrize("depth", [6, 7, 8])
def test_bf16x3_brickwork_n20_matrix_cores_vs_mpo(fp, depth):
    """Brickwork n = 20 at registers of 2^10, 2^12 and 2^14 entries, where
    consecutive GATEs on disjoint bits run as one 16x16 block on the bf16
    matrix cores: sampled pairs of a 4000-pair batch against MPO-zip on the
    same float32 gates, with the bounds of the vector BF16x3 path."""
    import oracle_pool

    ens, npairs = (0, 20, depth), 4000
    assert fp.fp_plan_info(ens)["peak_bits"] == 2 * depth - 2
    seed = synth.workload_seed(2, depth) + 5
    g = fp.sample(ens, npairs, seed, 0, fp.C64)
    got = fp.contract(ens, g, npairs, BF16X3).cpu().numpy()
    c64 = fp.contract(ens, g, npairs, fp.C64).cpu().numpy()
    assert np.isfinite(got).all()
    pairs = sorted(int(x) for x in synth.rng(300 + depth).choice(npairs, 24, replace=False))
    want = np.array(oracle_pool.traces(0, 20, depth, seed, pairs, fp32=True))
    r = rel_errors(got[pairs], want)
    print(f"brickwork n=20 D={depth} BF16x3: median {np.median(r):.3e}, max {r.max():.3e}")
    assert np.median(r) <= 2e-4 and r.max() <= 5e-3, (depth, float(np.median(r)), float(r.max()))
    # the whole batch against complex64 on the same gates
    rc = rel_errors(got, c64)
    assert np.median(rc) <= 2e-4 and rc.max() <= 3e-2, (depth, float(np.median(rc)), float(rc.max()))
    assert not np.array_equal(got, c64)
    fg, _ = estimator.frame_potential(got, 3)
    fw, _ = estimator.frame_potential(c64, 3)
    for k in range(3):
        assert abs(fg[k] - fw[k]) <= 2e-3 * fw[k], (k, fg[k], fw[k])


def test_bf16x3_brickwork_hbm_tiles_vs_dense(fp):
    """Depth 9 on 10 qubits: 16-bit registers in HBM slots, every run of
    GATEs applied tile by tile through LDS with the matrix-core blocks,
    against the dense oracle on the same float32 gates."""
    ens, n, seed = (0, 10, 9), 12, 4411
    assert fp.fp_plan_info(ens)["peak_bits"] == 16
    got = traces(fp, ens, n, seed, BF16X3)
    want = dense.traces(sampler.sample_pairs(0, 10, 9, seed, 0, n, fp32=True))
    r = rel_errors(got, want)
    print(f"brickwork n=10 D=9 BF16x3 (HBM tiles): median {np.median(r):.3e}, max {r.max():.3e}")
    assert np.median(r) <= 2e-4 and r.max() <= 5e-3, (float(np.median(r)), float(r.max()))
