"""GPU parity of the statistics pipeline against the oracle: the bootstrap
(resample by resample), its quantiles, the layers-to-epsilon fit, and the
adaptive estimator's stopping against the oracle's rule."""

import math

import numpy as np
import pytest
import torch

import synth
from oracle import dense, estimator, sampler
from oracle import statistics as st
from oracle.weingarten import brickwork_frame_potential

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fp():
    import paper_2205_09900_amd as m
    assert torch.cuda.is_available()
    return m


def _dev(z):
    return torch.from_numpy(np.stack([z.real, z.imag], 1).reshape(-1).copy()).cuda()


@pytest.mark.parametrize("n", [1, 2, 7, 4999, 200000])
def test_bootstrap_matches_oracle(fp, n):
    z = synth.heavy_tailed_traces(60 + n, n, scale=2.0)
    kmax, R, seed = 3, 300, 0xB007 + n
    samples = torch.empty(kmax * R, dtype=torch.float64, device="cuda")
    med, lo, hi = fp.fp_bootstrap(_dev(z), n, kmax, R, seed, samples, coverage=0.9)
    got = samples.cpu().numpy().reshape(kmax, R)
    want = st.bootstrap_philox(z, kmax, R, seed)
    assert np.max(np.abs(got - want) / np.abs(want)) <= 1e-12
    for k in range(kmax):
        v = np.sort(want[k])
        for q, g in ((0.5, med[k]), (0.05, lo[k]), (0.95, hi[k])):
            assert abs(g - st.quantile(v, q)) <= 1e-12 * abs(st.quantile(v, q))


def test_bootstrap_flags_nonfinite(fp):
    d = torch.ones(40, dtype=torch.float64, device="cuda")
    d[13] = float("nan")
    with pytest.raises(fp.FPError) as e:
        fp.fp_bootstrap(d, 20, 2, 50, 1)
    assert e.value.code == fp.FP_ENUMERIC


def test_layers_to_epsilon_matches_oracle(fp):
    # noisy exponential decays, one per bootstrap sample, plus samples whose
    # fit must fail (one qualifying depth, or no decay)
    layers = list(range(1, 10))
    R, fh = 300, 2.0
    g = synth.rng(77)
    F = np.empty((len(layers), R))
    for r in range(R):
        A, C = 1.5 + g.random(), 1.0 + g.random()
        F[:, r] = fh + A * A * np.exp(-2.0 * np.array(layers) / C) * np.exp(0.05 * g.standard_normal(len(layers)))
    F[:, 0] = fh * 20.0                 # nothing in the fit region
    F[:, 1] = fh + fh * np.linspace(0.1, 4.0, len(layers))  # rising: no decay
    d_out = torch.empty(R, dtype=torch.float64, device="cuda")
    med, failed = fp.fp_layers_to_epsilon(torch.from_numpy(F.reshape(-1).copy()).cuda(), layers, R, fh, 0.1, 6, 2, 2,
                                          5.0, d_out)
    got = d_out.cpu().numpy()
    want = []
    for r in range(R):
        res = st.layers_to_epsilon(layers, F[:, r], fh, 0.1, 6, 2, 2)
        want.append(np.nan if res is None else res[0])
    want = np.array(want)
    assert np.array_equal(np.isnan(got), np.isnan(want)) and failed == int(np.isnan(want).sum()) == 2
    ok = ~np.isnan(want)
    assert np.max(np.abs(got[ok] - want[ok]) / np.abs(want[ok])) <= 1e-9
    assert abs(med - st.quantile(np.sort(want[ok]), 0.5)) <= 1e-9 * abs(med)


def test_layers_to_epsilon_on_exact_brickwork_values(fp):
    # exact F^(2) of the n = 6 brickwork at depths 1..6 (Weingarten transfer)
    layers = list(range(1, 7))
    F = np.array([brickwork_frame_potential(6, d, 2) for d in layers])
    med, failed = fp.fp_layers_to_epsilon(torch.from_numpy(F).cuda(), layers, 1, 2.0, 0.1, 6, 2, 2)
    want = st.layers_to_epsilon(layers, F, 2.0, 0.1, 6, 2, 2)
    assert failed == 0 and abs(med - want[0]) <= 1e-9 * want[0]
    print(f"n=6 brickwork, k=2: {med:.3f} layers to epsilon = 0.1 (A = {want[1]:.3f}, C = {want[2]:.3f})")


def test_adaptive_estimator_stops_by_the_rule(fp):
    # brickwork n = 6, depth 3 (F^(2) = 2.524 exactly): stops once F^(2)
    # exceeds the Haar value 2 by 3 standard errors
    ens, batch, cap = (0, 6, 3), 500, 200000
    seed = synth.workload_seed(1, 3)
    f, se, used, reason, tr = fp.fp_frame_potential_adaptive(ens, fp.C128, 3, 2, seed, batch, cap, 60.0, 3.0, 2.0)
    assert reason == fp.STOP_RESOLVED and used % batch == 0 and used < cap
    got = torch.view_as_complex(tr[: 2 * used].view(-1, 2)).cpu().numpy()
    # the traces are the oracle's for pairs 0 .. used-1
    want = dense.traces(sampler.sample_pairs(0, 6, 3, seed, 0, used))
    assert np.max(np.abs(got - want)) <= 1e-12 * 64
    wf, wse = estimator.frame_potential(want, 3)
    assert np.allclose(f, wf, rtol=1e-12) and np.allclose(se, wse, rtol=1e-9)
    assert st.adaptive_decision(wf[1], wse[1], 2.0, None, 3.0, used, cap, 0.0, 60.0) == st.STOP_RESOLVED
    if used > batch:
        pf, pse = estimator.frame_potential(want[: used - batch], 3)
        assert st.adaptive_decision(pf[1], pse[1], 2.0, None, 3.0, used - batch, cap, 0.0, 60.0) == st.CONTINUE
    # a budget of one batch stops there
    _, _, used2, reason2, _ = fp.fp_frame_potential_adaptive(ens, fp.C128, 3, 2, seed, batch, batch, 60.0, 1e9, 2.0)
    assert used2 == batch and reason2 == fp.STOP_BUDGET
