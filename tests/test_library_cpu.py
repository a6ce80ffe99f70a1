"""Host-side checks of libfp.so: exports, argument validation, planner sizes.

No call here touches a GPU: only validation failures and host-only planner
entry points are exercised.
"""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fp.h")


@pytest.fixture(scope="module")
def fp():
    import paper_2205_09900_amd as m
    return m


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fp_[a-z0-9_]+)\s*\(", text)))


def test_exports_match_header(fp):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(fp.lib, n), n
    assert sorted(fp.EXPORTS) == names


def test_gate_bytes(fp):
    # brickwork n=6, D=3: (3 + 2 + 3) gates per circuit, 16 complex128 each, two circuits
    assert fp.fp_gate_bytes_per_pair((0, 6, 3), fp.C128) == 2 * 8 * 256
    assert fp.fp_gate_bytes_per_pair((0, 6, 3), fp.C64) == 2 * 8 * 128
    # local random n=50, S=100: matrices + bonds, padded to 64
    assert fp.fp_gate_bytes_per_pair((1, 50, 100), fp.C64) == (2 * 100 * 128 + 2 * 100 * 4 + 63) // 64 * 64
    # HEA n=40, L=6 float32 angles
    assert fp.fp_gate_bytes_per_pair((2, 40, 6), fp.C64) == 2 * 6 * 40 * 2 * 4
    assert fp.fp_gate_bytes_per_pair((7, 6, 3), fp.C64) == 0
    assert fp.fp_gate_bytes_per_pair((0, 1, 3), fp.C64) == 0


def test_validation_errors(fp):
    with pytest.raises(fp.FPError) as e:
        fp.fp_workspace_bytes((0, 65, 3), 10, fp.C64)
    assert e.value.code == fp.FP_EINVAL
    with pytest.raises(fp.FPError) as e:
        fp.fp_workspace_bytes((0, 6, 0), 10, fp.C64)
    assert e.value.code == fp.FP_EINVAL
    with pytest.raises(fp.FPError) as e:
        fp.fp_workspace_bytes((0, 6, 3), -1, fp.C64)
    assert e.value.code == fp.FP_EINVAL
    with pytest.raises(fp.FPError):
        fp.fp_workspace_bytes((0, 6, 3), 10, 9)
    ens = fp.Ensemble(0, 6, 3)
    rc = fp.lib.fp_sample_gates(ctypes.byref(ens), 0, 1, 0, fp.C64, None, 0, None)
    assert rc == fp.FP_OK               # zero pairs: no-op
    rc = fp.lib.fp_sample_gates(ctypes.byref(ens), -1, 1, 0, fp.C64, None, 0, None)
    assert rc == fp.FP_EINVAL
    rc = fp.lib.fp_sample_gates(ctypes.byref(ens), 5, 1, 0, fp.C64, None, 0, None)
    assert rc == fp.FP_EINVAL           # NULL buffer
    rc = fp.lib.fp_contract_trace_batch(ctypes.byref(ens), 0, fp.C64, None, None, None, 0, None)
    assert rc == fp.FP_OK
    f = (ctypes.c_double * 9)()
    rc = fp.lib.fp_frame_potential(ctypes.c_void_p(16), 10, 9, f, None, None)
    assert rc == fp.FP_EINVAL and "k_max" in fp.last_error()
    rc = fp.lib.fp_frame_potential(ctypes.c_void_p(16), 0, 2, f, None, None)
    assert rc == fp.FP_EINVAL
    rc = fp.lib.fp_frame_potential_cv(ctypes.c_void_p(16), ctypes.c_void_p(16), 10, None, 0, 2,
                                      0.5, f, None, None)
    assert rc == fp.FP_EINVAL           # c != 0 without surrogate values


def test_qudit_ensemble_checks(fp):
    """Qudit brickworks: q in 3..5 in local_dim, 0 there for qubit ensembles;
    q^4 complex entries per gate; the register (q^(2(D-1)) entries at depth
    D, the qubit brickwork's program with digits) must fit LDS."""
    d2 = 9 * 9
    G = 3 + 2 + 3  # n = 6, D = 3
    assert fp.fp_gate_bytes_per_pair((5, 6, 3, 3), fp.C128) == -(-2 * G * d2 * 16 // 64) * 64
    assert fp.fp_gate_bytes_per_pair((5, 6, 3, 5), fp.C64) == -(-2 * G * 625 * 8 // 64) * 64
    for bad in [(5, 6, 3, 2), (5, 6, 3, 6), (5, 6, 3, 0), (0, 6, 3, 3)]:
        with pytest.raises(fp.FPError) as e:
            fp.fp_workspace_bytes(bad, 10, fp.C64)
        assert e.value.code == fp.FP_EINVAL, bad
        assert fp.fp_gate_bytes_per_pair(bad, fp.C64) == 0
    assert fp.fp_workspace_bytes((5, 6, 5, 3), 10, fp.C128) == 0   # 3^8 entries
    assert fp.fp_workspace_bytes((5, 6, 4, 5), 10, fp.C64) == 0    # 5^6 entries, complex64
    for ens, prec in [((5, 6, 6, 3), fp.C64), ((5, 6, 5, 4), fp.C64), ((5, 6, 4, 5), fp.C128)]:
        with pytest.raises(fp.FPError) as e:
            fp.fp_workspace_bytes(ens, 10, prec)
        assert e.value.code == fp.FP_ETOOBIG, (ens, prec)
    info = fp.fp_plan_info((5, 8, 4, 3))
    assert info["peak_bits"] == 6 and info["bits"] == fp.fp_plan_info((0, 8, 4))["bits"]
    # GATE ops on b digits cost q^(b+2) multiply-adds: the qubit count at q = 2
    # is the plan's own, so the digit count is checked against it
    assert info["macs"] > fp.fp_plan_info((0, 8, 4))["macs"] * 1.5 ** 6


def test_brickwork_plan_sizes(fp):
    for n in (4, 6, 7, 20):
        for d in range(2, 8):
            info = fp.fp_plan_info((0, n, d))
            assert info["peak_bits"] == 2 * (d - 1)
            assert info["bits"][: n - 2] == [2 * (d - 1)] * (n - 2)
            assert info["bits"][n - 2] == 0
    info = fp.fp_plan_info((0, 6, 1))
    assert info["bits"] == [0] * 5 and info["peak_bits"] == 2


def test_brickwork_mac_count_interior(fp):
    # every interior column applies D-1 gates of 4 complex MACs per entry of a 4^(D-1) boundary
    n, d = 12, 5
    info = fp.fp_plan_info((0, n, d))
    chi = 4 ** (d - 1)
    interior = (n - 3) * (d - 1) * 4 * chi
    assert interior < info["macs"] < interior + 2 * (d - 1) * 4 * chi + 1


def test_hea_plan_sizes(fp):
    for L in range(1, 9):
        info = fp.fp_plan_info((2, 30, L))
        assert info["peak_bits"] == (0 if L == 1 else 2 * L - 2)


def _alternation_bits(n, bu, bv):
    """Independent count: boundary bits after column c = number of wire segments of qubit
    c+1 that join a bond-c gate to a bond-(c+1) gate, around the loop of W = U^dagger V."""
    w = list(bv) + list(reversed(bu))
    out = []
    for c in range(n - 1):
        seq = [b for b in w if b in (c, c + 1)]       # gates touching qubit c+1
        if not seq or all(b == c for b in seq) or all(b == c + 1 for b in seq):
            out.append(0)
            continue
        alt = sum(1 for i in range(len(seq)) if seq[i] != seq[i - 1])
        out.append(alt)
    return out


def test_local_random_plan_matches_alternation_count(fp):
    rng = np.random.default_rng(5)
    for trial in range(60):
        n = int(rng.integers(2, 12))
        s = int(rng.integers(1, 40))
        bu = rng.integers(0, n - 1, s)
        bv = rng.integers(0, n - 1, s)
        info = fp.fp_plan_local_random_host(n, bu, bv)
        want = _alternation_bits(n, bu, bv)
        assert info["bits"][: n - 1] == want, (n, list(bu), list(bv))
        assert info["peak_bits"] >= max(want)
        assert info["peak_bits"] <= max(want) + 4


def test_local_random_plan_edge_cases(fp):
    # everything on one bond of two qubits: all gates merge into one
    info = fp.fp_plan_local_random_host(2, [0, 0, 0], [0, 0, 0])
    assert info["bits"] == [0] and info["peak_bits"] == 2 and info["ops"] == 4
    # a qubit no gate touches
    info = fp.fp_plan_local_random_host(5, [0, 0], [3, 3])
    assert info["bits"] == [0, 0, 0, 0]
    # wide chain of a single repeated bond
    info = fp.fp_plan_local_random_host(50, [20] * 10, [20] * 10)
    assert max(info["bits"]) == 0
    with pytest.raises(fp.FPError):
        fp.fp_plan_local_random_host(5, [0, 4], [1, 1])   # bond 4 does not exist for n = 5
    with pytest.raises(ValueError):
        fp.fp_plan_local_random_host(5, [0, 1], [1])      # both circuits need the same step count


def test_haar_frame_potential_matches_the_oracle_count():
    import paper_2205_09900_amd as fp
    from oracle.haar_moments import haar_frame_potential
    for k in range(1, 9):
        for d in range(1, 10):
            assert fp.fp_haar_frame_potential(k, d) == haar_frame_potential(k, d), (k, d)


def test_sample_size_decision_matches_the_oracle_rule():
    import itertools
    import paper_2205_09900_amd as fp
    from oracle import statistics as st
    cases = itertools.product([1.5, 2.0, 2.2, 2.6, 3.5], [0.01, 0.1, 0.4], [None, 2.4, 4.0], [100, 1000],
                              [1.0, 20.0])
    for f, se, lower, n_done, secs in cases:
        want = st.adaptive_decision(f, se, 2.0, lower, 3.0, n_done, 1000, secs, 10.0)
        got = fp.fp_sample_size_decision(f, se, 2.0, -1.0 if lower is None else lower, 3.0, n_done, 1000, secs, 10.0)
        assert got == want, (f, se, lower, n_done, secs)
