"""Local random circuits on 50 qubits at 300 steps: registers beyond 2^31
entries (64-bit entry indices, slots of up to 32 GiB in a pool of most of
the device's memory).  Identities with known answers on pairs whose widest
register exceeds 2^31 entries, and the full 10^4-pair batch of the bench
with every pair contracted."""

import gc

import numpy as np
import pytest
import torch

import synth
from oracle import closed_forms
from tolerance import TOL

pytestmark = pytest.mark.gpu

N, S = 50, 300


@pytest.fixture(scope="module")
def fp():
    import paper_2205_09900_amd as m
    assert torch.cuda.is_available()
    yield m
    m.fp_set_launch_mode(m.LAUNCH_AUTO)
    gc.collect()
    torch.cuda.empty_cache()


def _bonds(fp, ens, buf, prec, npairs):
    nb = fp.fp_gate_bytes_per_pair(ens, prec)
    off = 2 * S * 32 * (8 if prec == 0 else 4)
    a = buf.view(npairs, nb)[:, off: off + 8 * S].cpu().numpy()
    return [np.frombuffer(a[i].tobytes(), np.int32).reshape(2, S) for i in range(npairs)]


def _selected_identity_buffer(fp, prec, seed, k_of=None):
    """Pairs with V's circuit := U's (except gate k_of(p) when given), chosen
    so that the widest W = U^dag V register has 2^32 entries (c64) or 2^30
    (c128), plus three narrower ones."""
    ens, cand = (1, N, S), 400
    g = fp.sample(ens, cand, seed, 0, prec).view(cand, -1)
    peaks = [fp.fp_plan_local_random_host(N, b[0], b[0])["peak_bits"] for b in _bonds(fp, ens, g, prec, cand)]
    top = 32 if prec == 1 else 30
    wide = [i for i, p in enumerate(peaks) if p == top][:1]
    rest = [i for i, p in enumerate(peaks) if 20 <= p <= 28][:3]
    assert wide, sorted(peaks)[-8:]
    pick = wide + rest
    rb = 8 if prec == 0 else 4
    gb, half = 32 * rb, S * 32 * rb
    h = g[pick].clone()
    h[:, half:2 * half] = h[:, :half]
    h[:, 2 * half + 4 * S: 2 * half + 8 * S] = h[:, 2 * half: 2 * half + 4 * S]
    ks = []
    for p in range(len(pick)):
        if k_of is not None:
            k = k_of(p)
            h[p, half + k * gb: half + (k + 1) * gb] = g[pick[p], half + k * gb: half + (k + 1) * gb]
            ks.append(k)
    return h, [peaks[i] for i in pick], ks


@pytest.mark.parametrize("prec", [1, 0])
def test_identity_beyond_2_31_entries(fp, prec):
    h, peaks, _ = _selected_identity_buffer(fp, prec, synth.workload_seed(80, prec))
    print(f"register widths 2^{peaks}")
    tr = fp.contract((1, N, S), h.reshape(-1), h.shape[0], prec).cpu().numpy()
    assert np.max(np.abs(tr - 2.0 ** N)) <= TOL[prec] * 2.0 ** N, tr
    del h
    torch.cuda.empty_cache()


def test_one_gate_difference_beyond_2_31_entries(fp):
    prec = 1
    h, peaks, ks = _selected_identity_buffer(fp, prec, synth.workload_seed(81, 0), k_of=lambda p: (37 * p + 11) % S)
    tr = fp.contract((1, N, S), h.reshape(-1), h.shape[0], prec).cpu().numpy()
    a = h.cpu().numpy()
    gb, half = 128, S * 128
    for p, k in enumerate(ks):
        gu = np.frombuffer(a[p, k * gb:(k + 1) * gb].tobytes(), np.float32).astype(np.float64).reshape(4, 4, 2)
        gv = np.frombuffer(a[p, half + k * gb: half + (k + 1) * gb].tobytes(), np.float32).astype(np.float64).reshape(4, 4, 2)
        want = closed_forms.one_gate_difference(N, gu[..., 0] + 1j * gu[..., 1], gv[..., 0] + 1j * gv[..., 1])
        assert abs(tr[p] - want) <= 1e-5 * abs(want), (p, peaks[p], tr[p], want)
    del h
    torch.cuda.empty_cache()


def test_full_batch_at_300_steps(fp):
    """The bench's batch at 300 steps (10^4 pairs, complex64): every pair is
    contracted (its widest register has 2^32 entries), both launch modes give
    the same traces bit for bit."""
    ens, npairs, prec = (1, N, S), 10000, 1
    seed = synth.workload_seed(4, 0) | (S << 32)
    g = fp.sample(ens, npairs, seed, 0, prec)
    ws = fp.workspace(ens, npairs, prec)
    out = {}
    for mode in (fp.LAUNCH_WAIT, fp.LAUNCH_WAIT_FREE):
        fp.fp_set_launch_mode(mode)
        out[mode] = fp.contract(ens, g, npairs, prec, ws)
        torch.cuda.synchronize()
    fp.fp_set_launch_mode(fp.LAUNCH_AUTO)
    a = out[fp.LAUNCH_WAIT].cpu().numpy()
    assert np.isfinite(a).all(), int((~np.isfinite(a)).sum())
    assert torch.equal(out[fp.LAUNCH_WAIT], out[fp.LAUNCH_WAIT_FREE])
    f, se = fp.frame_potential(out[fp.LAUNCH_WAIT], 3)
    print(f"S=300: F = {f}, SE = {se}")
    del g, ws, out
    torch.cuda.empty_cache()


def test_shared_trace_in_place(fp):
    """A pair alone in a workspace with room for one slot of its width: no
    second slot fits, so its shared TRACEs run in place, in rounds of outputs,
    with helpers on every free compute unit (its register reaches 2^30
    entries).  U = V gives 2^n; V differing from U in one gate gives the
    closed form."""
    prec = 1
    ens = (1, N, S)
    cand = 400
    g = fp.sample(ens, cand, synth.workload_seed(82, 1), 0, prec).view(cand, -1)
    pk = [fp.fp_plan_local_random_host(N, b[0], b[0])["peak_bits"] for b in _bonds(fp, ens, g, prec, cand)]
    pick = [i for i, p in enumerate(pk) if p == 30][:1]
    assert pick, sorted(pk)[-8:]
    rb, k = 4, 101
    gb, half = 32 * rb, S * 32 * rb
    u = g[pick].clone()
    u[:, half:2 * half] = u[:, :half]
    u[:, 2 * half + 4 * S: 2 * half + 8 * S] = u[:, 2 * half: 2 * half + 4 * S]
    d = u.clone()
    d[:, half + k * gb: half + (k + 1) * gb] = g[pick, half + k * gb: half + (k + 1) * gb]
    ws = fp.workspace(ens, 1, prec)
    both = torch.cat([u, d])
    tr = [fp.contract(ens, both[i].reshape(-1), 1, prec, ws).cpu().numpy()[0] for i in range(2)]
    assert abs(tr[0] - 2.0 ** N) <= TOL[prec] * 2.0 ** N, tr[0]
    a = d.cpu().numpy()
    gu = np.frombuffer(a[0, k * gb:(k + 1) * gb].tobytes(), np.float32).astype(np.float64).reshape(4, 4, 2)
    gv = np.frombuffer(a[0, half + k * gb: half + (k + 1) * gb].tobytes(), np.float32).astype(np.float64).reshape(4, 4, 2)
    want = closed_forms.one_gate_difference(N, gu[..., 0] + 1j * gu[..., 1], gv[..., 0] + 1j * gv[..., 1])
    assert abs(tr[1] - want) <= 1e-5 * abs(want), (tr[1], want)
    del g, u, d, both, ws
    torch.cuda.empty_cache()
