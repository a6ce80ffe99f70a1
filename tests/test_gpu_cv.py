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
