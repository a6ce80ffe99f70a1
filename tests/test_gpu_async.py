"""Local random contraction without host waits: the launches after planning
are derived on the device, so a pair that cannot be contracted is reported
through its trace (NaN, then FP_ENUMERIC from the reduction) rather than by
the call, and the sample -> contract sequence can be captured as a graph."""

import math

import numpy as np
import pytest
import torch

from oracle import dense, estimator, sampler
from tolerance import floored

pytestmark = pytest.mark.gpu

C64 = 1


@pytest.fixture(scope="module")
def fp():
    import paper_2205_09900_amd as m
    assert torch.cuda.is_available()
    return m


def peaks_of(fp, n, s, seed, npairs):
    out = []
    for u, v in sampler.sample_pairs(1, n, s, seed, 0, npairs):
        bu = np.array([b for b, _ in u["gates"]], np.int32)
        bv = np.array([b for b, _ in v["gates"]], np.int32)
        out.append(fp.fp_plan_local_random_host(n, bu, bv)["peak_bits"])
    return np.array(out)


def test_no_room_for_wide_pairs_gives_nan(fp):
    # 96 pairs of 8 qubits at 40 steps, 51 of them beyond the 2^14 entries of
    # LDS: with a workspace that holds the plans but no HBM slot, exactly those
    # get NaN, the others their traces, and the reduction flags the batch
    ens, n, seed = (1, 8, 40), 96, 4343
    peaks = peaks_of(fp, 8, 40, seed, n)
    wide = peaks > 14
    assert 0 < wide.sum() < n
    g = fp.sample(ens, n, seed, 0, C64)
    full = fp.fp_workspace_bytes(ens, n, C64)
    ws = torch.empty(full, dtype=torch.uint8, device="cuda")
    tr = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    lo, hi = 1, full  # smallest workspace the call accepts: the plans, nothing more
    while lo < hi:
        mid = (lo + hi) // 2
        try:
            fp.fp_contract_trace_batch(ens, n, C64, g, tr, ws[:mid])
            hi = mid
        except fp.FPError as e:
            assert e.code == fp.FP_ETOOBIG, e
            lo = mid + 1
    torch.cuda.synchronize()
    tr.fill_(0.0)
    fp.fp_contract_trace_batch(ens, n, C64, g, tr, ws[:lo])
    torch.cuda.synchronize()
    got = torch.view_as_complex(tr.view(-1, 2)).cpu().numpy()
    assert np.isnan(got[wide]).all()
    assert np.isfinite(got[~wide]).all()
    want = dense.traces(sampler.sample_pairs(1, 8, 40, seed, 0, n, fp32=True))
    w = want[~wide]
    err = floored(got[~wide], w, 1)
    assert err.max() <= 1e-5, err.max()
    with pytest.raises(fp.FPError) as ei:
        fp.fp_frame_potential(tr, n, 2)
    assert ei.value.code == fp.FP_ENUMERIC


def capture_and_replay(fp, ens, n, seed, eager_first):
    """Captures sample -> contract of one batch on a side stream and replays it
    three times, with eager work on the same buffers in between; returns the
    traces of the first replay after checking that every replay and every
    eager run agree bit for bit."""
    g = fp.alloc_gates(ens, n, C64)
    ws = fp.workspace(ens, n, C64)
    tr = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    ref = None
    if eager_first:
        with torch.cuda.stream(s):
            fp.fp_sample_gates(ens, n, seed, 0, C64, g, s)
            fp.fp_contract_trace_batch(ens, n, C64, g, tr, ws, s)
        s.synchronize()
        ref = tr.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        fp.fp_sample_gates(ens, n, seed, 0, C64, g, s)
        fp.fp_contract_trace_batch(ens, n, C64, g, tr, ws, s)
    torch.cuda.synchronize()
    first = None
    for rep in range(3):
        tr.fill_(float("nan"))
        g.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        if first is None:
            first = tr.clone()
        assert torch.equal(tr, first), rep
        if ref is not None:
            assert torch.equal(tr, ref), rep
        fp.fp_contract_trace_batch(ens, n, C64, g, tr, ws, s)  # eager, between replays
        s.synchronize()
        assert torch.equal(tr, first), rep
    return torch.view_as_complex(first.view(-1, 2)).cpu().numpy()


@pytest.mark.parametrize("eager_first", [True, False])
def test_graph_replay_wide_pairs_vs_dense(fp, eager_first):
    # 8 qubits, 40 steps: most pairs need HBM slots (up to 2^22 entries) and
    # the widest share their ops; captured with or without an earlier eager
    # batch of the ensemble (launch sizes from it, or as many workgroups as
    # stay resident), the replays must give the oracle's traces
    ens, n, seed = (1, 8, 40 if eager_first else 36), 96, 4343
    peaks = peaks_of(fp, ens[1], ens[2], seed, n)
    assert (peaks > 14).sum() > n // 5 and (peaks >= 18).any()
    got = capture_and_replay(fp, ens, n, seed, eager_first)
    want = dense.traces(sampler.sample_pairs(1, ens[1], ens[2], seed, 0, n, fp32=True))
    err = floored(got, want, 1)
    worst = int(np.argmax(err))
    assert err.max() <= 1e-5, (worst, err.max(), got[worst], want[worst])
    fg, _ = estimator.frame_potential(got, 3)
    fw, _ = estimator.frame_potential(want, 3)
    for k in range(3):
        assert abs(fg[k] - fw[k]) <= 1e-5 * fw[k], (k, fg[k], fw[k])


def test_local_random_graph_replay(fp):
    # every class of the local random path (n = 50, 120 steps, 300 pairs) in
    # one captured graph with its sampling
    got = capture_and_replay(fp, fp.Ensemble(fp.LOCAL_RANDOM, 50, 120), 300, 777, True)
    assert np.isfinite(got).all()


SLOT_TOP = 37  # slot arrays are indexed by register width 0..36, plus one entry for the totals


def read_setup(buf):
    """The launch set-up the device wrote into a chunk header (layout of LrDev)."""
    import ctypes

    class Slot(ctypes.Structure):
        _fields_ = [("base", ctypes.c_uint64), ("alt", ctypes.c_uint64), ("owners", ctypes.c_int32),
                    ("ge", ctypes.c_int32 * (SLOT_TOP + 1)), ("off", ctypes.c_int64 * (SLOT_TOP + 1)),
                    ("alt_off", ctypes.c_int64 * (SLOT_TOP + 1))]

    class Help(ctypes.Structure):
        _fields_ = [("recs", ctypes.c_uint64), ("finished", ctypes.c_uint64), ("wide", ctypes.c_int64),
                    ("help_bits", ctypes.c_int32)]

    class Dev(ctypes.Structure):
        _fields_ = [("first", ctypes.c_int32 * 64), ("range", ctypes.c_int64 * 10), ("claim", ctypes.c_uint64 * 5),
                    ("sl", Slot), ("help", Help), ("wgs", ctypes.c_int32), ("max_bits", ctypes.c_int32),
                    ("status", ctypes.c_int32)]

    d = Dev.from_buffer_copy(bytes(buf[: ctypes.sizeof(Dev)]))
    return dict(first=list(d.first), range=[(d.range[2 * k], d.range[2 * k + 1]) for k in range(5)],
                base=d.sl.base, alt=d.sl.alt, owners=d.sl.owners, ge=list(d.sl.ge), off=list(d.sl.off),
                alt_off=list(d.sl.alt_off), recs=d.help.recs, wide=d.help.wide, help_bits=d.help.help_bits,
                wgs=d.wgs, max_bits=d.max_bits, status=d.status)


def test_device_setup_matches_host_plans(fp):
    # the set-up the device derives from its plans (class ranges, ordering
    # offsets, graded HBM slots, work sharing) against the host planner's
    # widths of the same pairs
    ens, n, seed = (1, 8, 40), 96, 4343
    peaks = peaks_of(fp, 8, 40, seed, n)
    g = fp.sample(ens, n, seed, 0, C64)
    ws = fp.workspace(ens, n, C64)
    fp.contract(ens, g, n, C64, ws)
    torch.cuda.synchronize()
    d = read_setup(ws[1024:1024 + 2048].cpu().numpy().tobytes())
    for b in range(64):
        assert d["first"][b] == int((peaks > b).sum()), b
    bounds = [(-1, -1), (-1, 10), (10, 12), (12, 12), (12, 63)]
    for k, (lo, hi) in enumerate(bounds):
        cnt = int(((peaks > lo) & (peaks <= hi)).sum()) if hi > lo else 0
        assert d["range"][k][1] == cnt, (k, d["range"][k], cnt)
        if cnt:
            assert d["range"][k][0] == int((peaks > hi).sum()), k
    hbm = np.sort(peaks[peaks > 12])[::-1]  # the class in launch order
    owners = d["owners"]
    assert 1 <= owners <= min(len(hbm), 512)
    ge = d["ge"]

    assert d["max_bits"] == int(peaks.max())

    def width(j):
        b = SLOT_TOP - 1
        while b > 0 and ge[b] <= j:
            b -= 1
        return b

    regions = []
    for j in range(owners):
        w = width(j)
        assert w >= (hbm[j] if hbm[j] > 14 else 0), (j, w, hbm[j])  # 0: stays in LDS
        if w > 0:
            regions.append((d["off"][w] + ((j - ge[w + 1]) << w), 1 << w))
    regions.sort()
    for (a0, n0), (a1, _) in zip(regions, regions[1:]):
        assert a0 + n0 <= a1
    ws_end = ws.data_ptr() + ws.numel()
    if regions:
        assert d["base"] + 8 * (regions[-1][0] + regions[-1][1]) <= ws_end
    assert d["wide"] == int((peaks >= d["help_bits"]).sum())
    assert d["status"] == 0 and d["wgs"] >= owners
