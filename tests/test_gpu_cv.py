"""The control-variate pipeline end to end at a small scale (GPU)."""

import math

import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fp():
    import paper_2205_09900_amd as m
    assert torch.cuda.is_available()
    return m


def test_cv_pipeline_agrees_with_plain(fp):
    from paper_2205_09900_amd import cv
    ens = fp.Ensemble(fp.HEA, 6, 2)
    model = cv.train_surrogate(ens, k=2, hidden=64, n_train=8192, batch=512, epochs=8)
    assert model["holdout_mse"] < model["history"][0] * 1.0001
    res = cv.estimate(ens, model, k=2, n_exact=4000, n_surrogate=40000, seed_exact=11, seed_surr=12)
    # a high-statistics plain estimate on independent pairs
    tr, _ = cv.exact_traces(ens, 200000, 99)
    f, se = fp.fp_frame_potential(tr, 200000, 2)
    comb = math.sqrt(res["SE_cv"] ** 2 + se[1] ** 2)
    assert abs(res["F_cv"] - f[1]) <= 5 * comb, (res["F_cv"], f[1], comb)
    assert abs(res["F_plain"] - f[1]) <= 5 * math.sqrt(res["SE_plain"] ** 2 + se[1] ** 2)
    assert res["SE_cv"] > 0 and res["c"] == res["c"]


# One-layer HEA: log |Tr|^2 is a sum of per-qubit terms in the angle
# differences, which the network can learn from the sines and cosines; at two
# layers and more it is an interaction of every angle and the network finds
# no correlation (the control variate then falls back to the plain mean).
# F^(2) of the one-layer HEA is (C(4,2)^2 / 4^2)^n = 2.25^n exactly.

N1 = 3


@pytest.fixture(scope="module")
def one_layer_model(fp):
    from paper_2205_09900_amd import cv
    ens = fp.Ensemble(fp.HEA, N1, 1)
    return ens, cv.train_surrogate(ens, k=2, hidden=256, n_train=32768, batch=512, epochs=30, seed=5)


def test_cv_gain_where_the_surrogate_learns(fp, one_layer_model):
    """What the trained network gains: on fresh pairs the variance of
    f - c g is well below that of f (variance per exact pair), and the
    control-variate estimate agrees with the exact F^(2).  The gain per unit
    of time is reported: an exact one-layer trace costs less than a network
    evaluation here."""
    from oracle.closed_forms import hea_one_layer_frame_potential
    from paper_2205_09900_amd import cv
    ens, model = one_layer_model
    assert model["rho_holdout"] > 0.4, model["rho_holdout"]
    res = cv.estimate(ens, model, k=2, n_exact=8000, n_surrogate=400000, seed_exact=21, seed_surr=22)
    exact = hea_one_layer_frame_potential(N1, 2)
    st = res["stats_exact_pairs"]
    c = model["c"]
    var_r = st["var_f"] - 2 * c * st["rho"] * math.sqrt(st["var_f"] * st["var_g"]) + c * c * st["var_g"]
    print(f"rho hold-out {model['rho_holdout']:.3f}, exact pairs {st['rho']:.3f}; var(f - c g)/var(f) = "
          f"{var_r / st['var_f']:.3f}; F_cv {res['F_cv']:.4g} +- {res['SE_cv']:.2g}, plain {res['F_plain']:.4g} "
          f"+- {res['SE_plain']:.2g}, exact {exact:.4g}; time to 1 %: plain {res['time_to_1pct_plain_s']:.3g} s, "
          f"cv {res['time_to_1pct_cv_s']:.3g} s (predicted ratio {res['predicted_time_ratio_from_holdout']:.3g})")
    assert var_r <= 0.8 * st["var_f"]
    assert abs(res["F_cv"] - exact) <= 5 * res["SE_cv"]
    assert res["SE_cv"] < res["SE_plain"]


def test_cv_unbiased_over_repeats(fp, one_layer_model):
    """Unbiasedness (c and g fixed before the estimation pairs are drawn): the
    mean of 50 independent control-variate estimates, and of the plain ones,
    lies within 4 standard errors of the exact F^(2)."""
    import numpy as np
    from oracle.closed_forms import hea_one_layer_frame_potential
    from paper_2205_09900_amd import cv
    ens, model = one_layer_model
    exact = hea_one_layer_frame_potential(N1, 2)
    fcv, fpl = [], []
    for r in range(50):
        res = cv.estimate(ens, model, k=2, n_exact=2000, n_surrogate=50000, seed_exact=1000 + r,
                          seed_surr=5000 + r)
        fcv.append(res["F_cv"])
        fpl.append(res["F_plain"])
    for name, v in (("cv", np.array(fcv)), ("plain", np.array(fpl))):
        m, se = v.mean(), v.std(ddof=1) / math.sqrt(len(v))
        print(f"{name}: mean {m:.4g} +- {se:.2g} (exact {exact:.4g})")
        assert abs(m - exact) <= 4 * se, (name, m, se, exact)
