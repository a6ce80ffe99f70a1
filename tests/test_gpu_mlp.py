"""GPU parity of the surrogate network and the control-variate combiner."""

import numpy as np
import pytest
import torch

import synth
from oracle import estimator, mlp, sampler

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fp():
    import paper_2205_09900_amd as m
    assert torch.cuda.is_available()
    return m


def cu(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_vs_numpy(fp, ta, tb):
    for (m, n, k) in [(64, 64, 16), (100, 70, 33), (1, 256, 1920), (300, 256, 256), (1920, 256, 129)]:
        a = synth.normal(m * 7 + k, (k, m) if ta else (m, k)).astype(np.float32)
        b = synth.normal(n * 5 + k, (n, k) if tb else (k, n)).astype(np.float32)
        c = torch.zeros(m, n, dtype=torch.float32, device="cuda")
        fp.fp_mlp_gemm(m, n, k, cu(a), a.shape[1], ta, cu(b), b.shape[1], tb, c, n)
        want = (a.T if ta else a).astype(np.float64) @ (b.T if tb else b).astype(np.float64)
        err = np.max(np.abs(c.cpu().numpy() - want)) / max(1.0, np.max(np.abs(want)))
        assert err < 2e-5, (m, n, k, err)


def _setup(n_in=24, h=64, b=50):
    p = synth.normal(11, mlp.param_count(n_in, h), std=0.2).astype(np.float32)
    x = synth.normal(12, (b, n_in)).astype(np.float32)
    t = synth.normal(13, b).astype(np.float32)
    return n_in, h, b, p, x, t


def test_forward_backward_vs_oracle(fp):
    n_in, h, b, p, x, t = _setup()
    dp, dx, dt = cu(p), cu(x), cu(t)
    y = torch.empty(b, dtype=torch.float32, device="cuda")
    act = torch.empty(fp.fp_mlp_act_floats(b, h), dtype=torch.float32, device="cuda")
    fp.fp_mlp_forward(n_in, h, b, dp, dx, y, act)
    yo, _ = mlp.forward(p.astype(np.float64), x.astype(np.float64), n_in, h)
    assert np.max(np.abs(y.cpu().numpy() - yo)) <= 1e-4 * max(1.0, np.max(np.abs(yo)))
    g = torch.empty(fp.fp_mlp_param_count(n_in, h), dtype=torch.float32, device="cuda")
    loss = fp.fp_mlp_backward(n_in, h, b, dp, dx, act, dt, g)
    lo, go = mlp.loss_and_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64), n_in, h)
    assert abs(loss - lo) <= 1e-4 * lo
    gg = g.cpu().numpy()
    rel = np.linalg.norm(gg - go) / np.linalg.norm(go)
    assert rel <= 1e-4, rel
    # every parameter block separately
    o = 0
    for size in [n_in * h, h, h * h, h, h * h, h, h, 1]:
        blk = slice(o, o + size)
        assert np.linalg.norm(gg[blk] - go[blk]) <= 1e-4 * max(np.linalg.norm(go[blk]), 1e-6)
        o += size


def test_adam_vs_oracle(fp):
    n = 1000
    p = synth.normal(1, n).astype(np.float32)
    g = synth.normal(2, n).astype(np.float32)
    dp, dg = cu(p), cu(g)
    state = torch.zeros(2 * n, dtype=torch.float32, device="cuda")
    po, m, v = p.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in (1, 2, 3):
        fp.fp_mlp_adam_step(n, dp, dg, state, step, lr=1e-2)
        po, m, v = mlp.adam(po, g.astype(np.float64), m, v, step, 1e-2)
    assert np.max(np.abs(dp.cpu().numpy() - po)) <= 1e-6


def test_features_vs_oracle(fp):
    ens = (2, 6, 3)
    g = fp.sample(ens, 9, 77, 5, fp.C64)
    x = torch.empty(9, 8 * 6 * 3, dtype=torch.float32, device="cuda")
    fp.fp_mlp_features(ens, 9, g, x)
    pairs = sampler.sample_pairs(2, 6, 3, 77, 5, 9, fp32=True)
    th_u = np.array([pr[0]["theta"] for pr in pairs])
    ph_u = np.array([pr[0]["phi"] for pr in pairs])
    th_v = np.array([pr[1]["theta"] for pr in pairs])
    ph_v = np.array([pr[1]["phi"] for pr in pairs])
    want = mlp.features(th_u, ph_u, th_v, ph_v)
    assert np.max(np.abs(x.cpu().numpy() - want)) <= 2e-6


def test_training_reduces_loss(fp):
    n_in, h, b = 16, 64, 256
    x = synth.normal(5, (b, n_in)).astype(np.float32)
    t = (np.sin(x[:, 0]) + 0.5 * x[:, 1] ** 2).astype(np.float32)
    npar = fp.fp_mlp_param_count(n_in, h)
    p = torch.empty(npar, dtype=torch.float32, device="cuda")
    fp.fp_mlp_init(n_in, h, 3, p)
    st = torch.zeros(2 * npar, dtype=torch.float32, device="cuda")
    g = torch.empty(npar, dtype=torch.float32, device="cuda")
    y = torch.empty(b, dtype=torch.float32, device="cuda")
    act = torch.empty(fp.fp_mlp_act_floats(b, h), dtype=torch.float32, device="cuda")
    dx, dt = cu(x), cu(t)
    losses = []
    for step in range(1, 201):
        fp.fp_mlp_forward(n_in, h, b, p, dx, y, act)
        losses.append(fp.fp_mlp_backward(n_in, h, b, p, dx, act, dt, g))
        fp.fp_mlp_adam_step(npar, p, g, st, step, lr=3e-3)
    assert losses[-1] < 0.1 * losses[0], (losses[0], losses[-1])


def test_control_variate_combiner(fp):
    nb, nc = 1000, 5000
    z = synth.heavy_tailed_traces(21, nb)
    f = np.abs(z) ** 4
    gb = (f * 0.8 + synth.normal(22, nb, std=0.3)).astype(np.float32)
    gc = (np.abs(synth.heavy_tailed_traces(23, nc)) ** 4 * 0.8).astype(np.float32)
    dtr = cu(np.stack([z.real, z.imag], 1).reshape(-1), torch.float64)
    for c in (0.0, 0.9):
        est, se = fp.fp_frame_potential_cv(dtr, cu(gb), nb, cu(gc), nc, 2, c)
        want, wse = estimator.control_variate(f, gb.astype(np.float64), gc.astype(np.float64), c)
        assert abs(est - want) <= 1e-12 * abs(want) and abs(se - wse) <= 1e-9 * wse
    # a constant surrogate gives the plain mean exactly (up to float64 rounding)
    est, _ = fp.fp_frame_potential_cv(dtr, cu(np.full(nb, 2.5, np.float32)), nb,
                                      cu(np.full(nc, 2.5, np.float32)), nc, 2, 0.7)
    assert abs(est - f.mean()) <= 1e-12 * f.mean()
