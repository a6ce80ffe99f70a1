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

    class Phase(ctypes.Structure):
        _fields_ = [("sl", Slot), ("help", Help), ("first", ctypes.c_int64), ("count", ctypes.c_int64),
                    ("workgroups", ctypes.c_int32), ("max_bits", ctypes.c_int32)]

    class Dev(ctypes.Structure):
        _fields_ = [("first", ctypes.c_int32 * 64), ("range", ctypes.c_int64 * 10), ("claim", ctypes.c_uint64 * 5),
                    ("ph", Phase * 2), ("wgs", ctypes.c_int32), ("max_bits", ctypes.c_int32),
                    ("status", ctypes.c_int32)]

    assert ctypes.sizeof(Dev) <= len(buf)
    d = Dev.from_buffer_copy(bytes(buf[: ctypes.sizeof(Dev)]))

    def phase(p):
        return dict(base=p.sl.base, alt=p.sl.alt, owners=p.sl.owners, ge=list(p.sl.ge), off=list(p.sl.off),
                    alt_off=list(p.sl.alt_off), recs=p.help.recs, wide=p.help.wide, help_bits=p.help.help_bits,
                    first=p.first, count=p.count, wgs=p.workgroups, max_bits=p.max_bits)

    out = dict(first=list(d.first), range=[(d.range[2 * k], d.range[2 * k + 1]) for k in range(5)],
               phases=[phase(d.ph[0]), phase(d.ph[1])], wgs=d.wgs, max_bits=d.max_bits, status=d.status)
    out.update({k: v for k, v in out["phases"][0].items() if k not in ("first", "wgs", "max_bits")})
    return out


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
    d = read_setup(ws[1024:4096].cpu().numpy().tobytes())
    # one launch of the HBM class: no pair is wider than a compute unit's share of the pool
    assert d["phases"][1]["count"] == 0 and d["phases"][1]["wgs"] == 0
    assert d["phases"][0]["first"] == 0 and d["phases"][0]["count"] == int((peaks > 12).sum())
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


def test_device_setup_splits_the_widest_pairs(fp):
    # n = 50, 250 steps, 2000 pairs in a 48 GiB pool: pairs wider than a
    # compute unit's share of the pool (2^24 entries on 256 compute units)
    # form the first launch of the HBM class, the others the second; each
    # launch's slots fit the pool, and every pair is contracted
    ens, n, seed = (1, 50, 250), 2000, 4545
    g = fp.sample(ens, n, seed, 0, C64)
    # widths from the host planner on the sampled bonds (they follow the
    # complex64 gates of U and V)
    S, off = ens[2], 2 * ens[2] * 32 * 4
    a = g.view(n, -1)[:, off: off + 8 * S].cpu().numpy()
    peaks = np.array([fp.fp_plan_local_random_host(50, *np.frombuffer(a[i].tobytes(), np.int32).reshape(2, S))
                      ["peak_bits"] for i in range(n)])
    ws = fp.workspace(ens, n, C64)
    tr = fp.contract(ens, g, n, C64, ws).cpu().numpy()
    torch.cuda.synchronize()
    assert np.isfinite(tr).all()
    d = read_setup(ws[1024:4096].cpu().numpy().tobytes())
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    pool_entries = d["phases"][0]["base"] and (ws.data_ptr() + ws.numel() - d["phases"][0]["base"]) // 8
    split = int(np.floor(np.log2(pool_entries // cus)))
    wide, rest = int((peaks > split).sum()), int(((peaks > 12) & (peaks <= split)).sum())
    assert wide > 0 and rest > 0, (split, wide, rest)
    p0, p1 = d["phases"]
    assert (p0["first"], p0["count"], p1["first"], p1["count"]) == (0, wide, wide, rest)
    assert p0["max_bits"] == int(peaks.max()) and p1["max_bits"] == int(peaks[peaks <= split].max())
    assert p1["owners"] > p0["owners"]
    for p in (p0, p1):
        assert p["wgs"] >= p["owners"] >= 1
        total = p["off"][SLOT_TOP] + (p["alt_off"][SLOT_TOP] if p["alt"] else 0)
        assert total <= pool_entries, (total, pool_entries)
    assert d["status"] == 0
