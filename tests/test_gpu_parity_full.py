"""GPU parity at the workloads' full sizes, in the launch configuration the
bench times, on sampled pairs the oracle contracts one by one.

The oracle draws each sampled pair itself (its own Philox sampler, from the
seed and the global pair index) and contracts it with the MPO-zip or dense
oracle; the device buffer is only used to choose which pairs to check.
Tolerances (per pair, floored relative error of the trace, tests/tolerance.py):
1e-12 for complex128 (floor 1e-3 x rms), 1e-5 for complex64 (floor 1 x rms).
Statistical checks (Haar validation, first moment) use the library's
standard error with a 5 sigma bound on fixed seeds.
"""

import math

import numpy as np
import pytest
import torch

import synth
from oracle import closed_forms, dense, mpo, sampler
from oracle.haar_moments import haar_frame_potential
import oracle_pool

pytestmark = pytest.mark.gpu

from tolerance import TOL, floored


@pytest.fixture(scope="module")
def fp():
    import paper_2205_09900_amd as m
    assert torch.cuda.is_available()
    yield m
    m.fp_set_launch_mode(m.LAUNCH_AUTO)


def as_complex(tr):
    if not tr.is_complex():
        tr = torch.view_as_complex(tr.view(-1, 2))
    return tr.cpu().numpy()


def device_bonds(fp, ens, buf, prec, pairs):
    """Bond lists of chosen pairs of a local random device buffer (selection only)."""
    nb = fp.fp_gate_bytes_per_pair(ens, prec)
    s = ens[2]
    rb = 8 if prec == 0 else 4
    off = 2 * s * 32 * rb
    a = buf.view(-1, nb)[pairs, off: off + 8 * s].cpu().numpy()
    return [np.frombuffer(a[i].tobytes(), np.int32).reshape(2, s) for i in range(len(pairs))]


# ---- local random, n = 50, S = 100: the headline batch ----------------------

BENCH_SEED = synth.workload_seed(4, 0)


def _chosen_pairs(fp, ens, buf, prec, n_pairs, n_random, n_widest, rng_seed):
    rng = synth.rng(rng_seed)
    rand = sorted(int(x) for x in rng.choice(n_pairs, n_random, replace=False))
    # widest pairs of a strided scan (they run in the HBM-slot class)
    scan = list(range(0, n_pairs, 7))
    peaks = []
    for i, b in zip(scan, device_bonds(fp, ens, buf, prec, scan)):
        peaks.append((fp.fp_plan_local_random_host(ens[1], b[0], b[1])["peak_bits"], i))
    peaks.sort(reverse=True)
    wide = [i for _, i in peaks[:n_widest]]
    return sorted(set(rand + wide)), peaks[0][0]


@pytest.mark.parametrize("prec", [1, 0])
def test_local_random_n50_S100_batch_vs_mpo(fp, prec):
    """The headline batch (10^4 pairs, n = 50, S = 100) contracted once
    waiting for its plans and once without: identical traces bit for bit,
    and sampled pairs (random ones and the widest) equal to MPO-zip."""
    ens, npairs = fp.Ensemble(fp.LOCAL_RANDOM, 50, 100), 10000
    seed = BENCH_SEED | (100 << 32)
    g = fp.sample(ens, npairs, seed, 0, prec)
    ws = fp.workspace(ens, npairs, prec)
    out = {}
    for mode in (fp.LAUNCH_WAIT, fp.LAUNCH_WAIT_FREE):
        fp.fp_set_launch_mode(mode)
        out[mode] = fp.contract(ens, g, npairs, prec, ws)
        torch.cuda.synchronize()
    fp.fp_set_launch_mode(fp.LAUNCH_AUTO)
    assert torch.equal(out[fp.LAUNCH_WAIT], out[fp.LAUNCH_WAIT_FREE])
    got = as_complex(out[fp.LAUNCH_WAIT])
    assert np.isfinite(got).all()
    pairs, widest = _chosen_pairs(fp, (1, 50, 100), g, prec, npairs, 8 if prec else 3, 3 if prec else 1, 100 + prec)
    assert widest > 12  # the HBM-slot class is among the checked pairs
    want = np.array(oracle_pool.traces(1, 50, 100, seed, pairs, fp32=(prec != 0)))
    err = floored(got[pairs], want, prec)
    print(f"local random n=50 S=100 prec={prec}: pairs {pairs}, max floored err {err.max():.3e}")
    assert err.max() <= TOL[prec], list(zip(pairs, err))


def _one_gate_buffer(fp, ens, prec, npairs, seed, k_of):
    """U = V except gate k_of(p) of pair p, in a local random buffer."""
    s = ens[2]
    rb = 8 if prec == 0 else 4
    gb = 32 * rb
    half = s * gb
    g = fp.sample(ens, npairs, seed, 0, prec).view(npairs, -1)
    h = g.clone()
    h[:, half:2 * half] = g[:, :half]                 # V's gates := U's gates
    boff = 2 * half
    h[:, boff + 4 * s: boff + 8 * s] = g[:, boff: boff + 4 * s]  # V's bonds := U's bonds
    for p in range(npairs):
        k = k_of(p)
        h[p, half + k * gb: half + (k + 1) * gb] = g[p, half + k * gb: half + (k + 1) * gb]
    return h


@pytest.mark.parametrize("prec", [1, 0])
def test_one_gate_difference_n50_S100(fp, prec):
    """U and V equal except one gate G vs G': Tr = 2^(n-2) Tr(G^dag G')
    (closed form from the same stored gates), at the headline size."""
    ens, npairs = (1, 50, 100), 16
    ks = [(7 * p + 3) % 100 for p in range(npairs)]
    h = _one_gate_buffer(fp, ens, prec, npairs, 0xD1FF, lambda p: ks[p])
    tr = as_complex(fp.contract(ens, h.reshape(-1), npairs, prec))
    real = np.float64 if prec == 0 else np.float32
    a = h.cpu().numpy()
    gb, half = 32 * np.dtype(real).itemsize, 100 * 32 * np.dtype(real).itemsize
    for p in range(npairs):
        k = ks[p]
        gu = np.frombuffer(a[p, k * gb:(k + 1) * gb].tobytes(), real).astype(np.float64).reshape(4, 4, 2)
        gv = np.frombuffer(a[p, half + k * gb: half + (k + 1) * gb].tobytes(), real).astype(np.float64).reshape(4, 4, 2)
        want = closed_forms.one_gate_difference(50, gu[..., 0] + 1j * gu[..., 1], gv[..., 0] + 1j * gv[..., 1])
        assert abs(tr[p] - want) <= TOL[prec] * abs(want), (p, k, tr[p], want)


# ---- brickwork, n = 20, depths 4..8 (complex64) ------------------------------

@pytest.mark.parametrize("depth", [4, 5, 6, 7, 8])
def test_brickwork_n20_c64_vs_mpo(fp, depth):
    """A 20000-pair chunk of the n = 20 workload (the chunk size the bench
    contracts), 64 sampled pairs against MPO-zip on the same float32 gates."""
    ens, npairs = (0, 20, depth), 20000
    seed = synth.workload_seed(2, depth)
    got = as_complex(fp.contract(ens, fp.sample(ens, npairs, seed, 0, fp.C64), npairs, fp.C64))
    assert np.isfinite(got).all()
    pairs = sorted(int(x) for x in synth.rng(200 + depth).choice(npairs, 64, replace=False))
    want = np.array(oracle_pool.traces(0, 20, depth, seed, pairs, fp32=True))
    err = floored(got[pairs], want, 1)
    rms = np.sqrt(np.mean(np.abs(want) ** 2))
    print(f"brickwork n=20 D={depth} c64: max floored err {err.max():.3e}, median {np.median(err):.3e}, "
          f"max |dTr|/rms {np.max(np.abs(got[pairs] - want)) / rms:.3e}")
    assert err.max() <= 1e-5, (depth, err.max())


@pytest.mark.parametrize("prec", [1, 0])
def test_brickwork_hbm_path_vs_dense_both_precisions(fp, prec):
    """Depth 9 on 10 qubits (16-bit boundary, beyond LDS: HBM slots, with the
    matrices staged from their factors) against the dense oracle."""
    ens = (0, 10, 9)
    assert fp.fp_plan_info(ens)["peak_bits"] == 16
    seed, npairs = 78, 12
    got = as_complex(fp.contract(ens, fp.sample(ens, npairs, seed, 0, prec), npairs, prec))
    want = dense.traces(sampler.sample_pairs(0, 10, 9, seed, 0, npairs, fp32=(prec != 0)))
    assert floored(got, want, prec).max() <= TOL[prec]


# ---- HEA n = 30, L = 1..8 in one persistent launch ----------------------------

def test_hea_n30_mixed_launch_vs_mpo(fp):
    """The uneven-depth workload: L = 1..8 groups in one
    fp_contract_trace_groups launch; sampled pairs of every group against
    MPO-zip (float32 angles)."""
    Ls = list(range(1, 9))
    ens = [(2, 30, L) for L in Ls]
    n = 2000
    bufs = [fp.sample(e, n, synth.workload_seed(3, e[2]), 0, fp.C64) for e in ens]
    groups = [(i, fp.C64, 0, n) for i in range(len(ens))]
    tr = torch.empty(2 * n * len(ens), dtype=torch.float64, device="cuda")
    ws = torch.empty(max(256, fp.fp_workspace_bytes_groups(ens, groups)), dtype=torch.uint8, device="cuda")
    fp.fp_contract_trace_groups(ens, groups, bufs, tr, ws)
    got = as_complex(tr)
    assert np.isfinite(got).all()
    for i, L in enumerate(Ls):
        pairs = sorted(int(x) for x in synth.rng(300 + L).choice(n, 6 if L < 8 else 3, replace=False))
        want = np.array(oracle_pool.traces(2, 30, L, synth.workload_seed(3, L), pairs, fp32=True))
        err = floored(got[i * n + np.array(pairs)], want, 1)
        assert err.max() <= 1e-5, (L, err.max())


# ---- statistical checks -------------------------------------------------------

def test_haar_two_qubit_validation(fp):
    """The paper's check of its Haar sampler (Supplementary: validation of
    sampling Haar random two-qubit unitaries): n = 2, one layer, so Tr is
    Tr(G_U^dag G_V) of two Haar U(4) gates and F^(k) must equal the number
    of permutations of k with no increasing subsequence longer than 4:
    1, 2, 6, 24, 119, 694 for k = 1..6."""
    ens, total, chunk = (0, 2, 1), 8_000_000, 2_000_000
    seed = synth.workload_seed(6, 1)
    tr = torch.empty(2 * total, dtype=torch.float64, device="cuda")
    g = fp.alloc_gates(ens, chunk, fp.C128)
    ws = fp.workspace(ens, chunk, fp.C128)
    for o in range(0, total, chunk):
        fp.fp_sample_gates(ens, chunk, seed, o, fp.C128, g)
        fp.fp_contract_trace_batch(ens, chunk, fp.C128, g, tr[2 * o: 2 * (o + chunk)], ws)
    f, se = fp.fp_frame_potential(tr, total, 6)
    # the paper's uncertainty analysis: 300 bootstrap resamples (99.9 % interval)
    med, lo, hi = fp.fp_bootstrap(tr, total, 6, 300, seed, coverage=0.999)
    want = [haar_frame_potential(k, 4) for k in range(1, 7)]
    assert want == [1, 2, 6, 24, 119, 694]
    for k in range(6):
        print(f"k={k + 1}: F={f[k]:.5g} +- {se[k]:.2g}, bootstrap [{lo[k]:.5g}, {hi[k]:.5g}] (exact {want[k]})")
        assert abs(f[k] - want[k]) <= 5 * se[k], (k + 1, f[k], se[k], want[k])
        assert lo[k] <= want[k] <= hi[k], (k + 1, lo[k], hi[k], want[k])
        assert se[k] <= 0.02 * want[k]


@pytest.mark.parametrize("depth", [2, 4, 6, 8])
def test_brickwork_n20_first_moment_is_one(fp, depth):
    """F^(1) = 1 for a brickwork in which every qubit meets a Haar gate (the
    first-moment twirl depolarises), at n = 20 where no dense oracle exists."""
    ens, npairs = (0, 20, depth), 100000
    seed = synth.workload_seed(2, depth)
    tr = torch.empty(2 * npairs, dtype=torch.float64, device="cuda")
    chunk = 20000
    g = fp.alloc_gates(ens, chunk, fp.C64)
    ws = fp.workspace(ens, chunk, fp.C64)
    for o in range(0, npairs, chunk):
        fp.fp_sample_gates(ens, chunk, seed, o, fp.C64, g)
        fp.fp_contract_trace_batch(ens, chunk, fp.C64, g, tr[2 * o: 2 * (o + chunk)], ws)
    f, se = fp.fp_frame_potential(tr, npairs, 1)
    assert abs(f[0] - 1.0) <= 5 * se[0], (depth, f[0], se[0])
    med, lo, hi = fp.fp_bootstrap(tr, npairs, 1, 300, seed, coverage=0.999)
    assert lo[0] <= 1.0 <= hi[0], (depth, lo[0], hi[0])
