"""Learned control variate for F^(k) of the hardware-efficient ansatz.

A small network g predicts |Tr(U^dagger V)|^{2k} from the sines and cosines
of the circuit angles.  By default it is fitted in log space: it learns the
standardised log |Tr|^2 (close to a sum over qubits, since the trace of a
shallow ansatz is close to a product of per-qubit factors), and
g = exp(k * prediction) is the control variate; target="power" fits
|Tr|^{2k} / F directly.  It is trained on exact traces that the method
computes, the coefficient c = Cov(f, g)/Var(g) is fixed on a hold-out set,
and then
    F_CV = mean_B(f - c g) + c mean_C(g)
over B fresh exact pairs and C fresh surrogate-only draws.  Because c and g
are fixed before B and C are drawn, F_CV is unbiased; the plain mean over B
is computed alongside as the fallback and as the check of F_CV.

Every arithmetic step runs in the library's kernels (sampling, contraction,
features, network, reductions); this module allocates device buffers and
orders the work.
"""

import math
import time

import numpy as np
import torch

from . import (C64, HEA, Ensemble, fp_contract_trace_batch, fp_cv_choose, fp_cv_holdout, fp_cv_time_to_rel_se,
               fp_frame_potential, fp_frame_potential_cv, fp_log_moments, fp_mlp_act_floats, fp_mlp_adam_step,
               fp_mlp_backward, fp_mlp_features, fp_mlp_forward, fp_mlp_init, fp_mlp_link, fp_mlp_log_targets,
               fp_mlp_param_count, fp_mlp_targets, fp_moments_f32, fp_sample_gates, alloc_gates, workspace)

LOG_EPS = 1e-30


def _sync():
    torch.cuda.synchronize()


def exact_traces(ens, n_pairs, seed, first_pair=0, chunk=65536, with_features=False):
    """Sample and contract n_pairs pairs; optionally also build their features."""
    n_in = 8 * ens.n_qubits * ens.depth
    tr = torch.empty(2 * n_pairs, dtype=torch.float64, device="cuda")
    x = torch.empty(n_pairs, n_in, dtype=torch.float32, device="cuda") if with_features else None
    c = min(chunk, n_pairs)
    g = alloc_gates(ens, c, C64)
    ws = workspace(ens, c, C64)
    for o in range(0, n_pairs, c):
        m = min(c, n_pairs - o)
        fp_sample_gates(ens, m, seed, first_pair + o, C64, g)
        fp_contract_trace_batch(ens, m, C64, g, tr[2 * o: 2 * (o + m)], ws)
        if with_features:
            fp_mlp_features(ens, m, g, x[o: o + m])
    return tr, x


def surrogate_values(ens, params, hidden, n_draws, seed, first_pair=0, chunk=65536):
    """g for n_draws fresh angle draws: sample -> features -> network (no contraction)."""
    n_in = 8 * ens.n_qubits * ens.depth
    out = torch.empty(n_draws, dtype=torch.float32, device="cuda")
    c = min(chunk, n_draws)
    g = alloc_gates(ens, c, C64)
    x = torch.empty(c, n_in, dtype=torch.float32, device="cuda")
    for o in range(0, n_draws, c):
        m = min(c, n_draws - o)
        fp_sample_gates(ens, m, seed, first_pair + o, C64, g)
        fp_mlp_features(ens, m, g, x[:m])
        fp_mlp_forward(n_in, hidden, m, params, x[:m], out[o: o + m])
    return out


def predict(n_in, hidden, params, x, chunk=65536):
    n = x.shape[0]
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    for o in range(0, n, chunk):
        m = min(chunk, n - o)
        fp_mlp_forward(n_in, hidden, m, params, x[o: o + m], y[o: o + m])
    return y


def link(model, y):
    """Network output -> control variate g in units of the training F^(k)."""
    if model["target"] == "power":
        return y
    g = torch.empty_like(y)
    fp_mlp_link(y, y.numel(), model["k"], model["log_mean"], model["log_std"], model["log_shift"], g)
    return g


def train_surrogate(ens, k=2, hidden=256, n_train=65536, holdout_frac=0.1, batch=1024, epochs=30, lr=1e-3,
                    seed=0xC0FFEE, patience=4, log=None, target="log"):
    """Train g on exact |Tr|^{2k} of n_train fresh pairs; returns a dict with the
    parameters (best hold-out loss), the target scale, c on the hold-out and timings."""
    t0 = time.perf_counter()
    n_in = 8 * ens.n_qubits * ens.depth
    tr, x = exact_traces(ens, n_train, seed, 0, with_features=True)
    f_mean, _ = fp_frame_potential(tr, n_train, k)
    scale = 1.0 / f_mean[k - 1]
    t = torch.empty(n_train, dtype=torch.float32, device="cuda")
    log_mean = log_std = 0.0
    if target == "log":
        log_mean, log_std = fp_log_moments(tr, n_train, LOG_EPS)
        fp_mlp_log_targets(tr, n_train, LOG_EPS, log_mean, log_std, t)
    else:
        fp_mlp_targets(tr, n_train, k, scale, t)
    n_hold = int(n_train * holdout_frac)
    n_fit = n_train - n_hold
    _sync()
    t_data = time.perf_counter() - t0

    npar = fp_mlp_param_count(n_in, hidden)
    p = torch.empty(npar, dtype=torch.float32, device="cuda")
    fp_mlp_init(n_in, hidden, seed ^ 0x5EED, p)
    adam = torch.zeros(2 * npar, dtype=torch.float32, device="cuda")
    grad = torch.empty(npar, dtype=torch.float32, device="cuda")
    y = torch.empty(batch, dtype=torch.float32, device="cuda")
    act = torch.empty(fp_mlp_act_floats(batch, hidden), dtype=torch.float32, device="cuda")
    hold_act = torch.empty(fp_mlp_act_floats(n_hold, hidden), dtype=torch.float32, device="cuda")
    hold_y = torch.empty(n_hold, dtype=torch.float32, device="cuda")
    hold_grad = torch.empty(npar, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(seed)
    nb = n_fit // batch
    step = 0
    best, best_p, bad = math.inf, p.clone(), 0
    history = []
    t1 = time.perf_counter()
    for ep in range(epochs):
        for bi in rng.permutation(nb):
            o = int(bi) * batch
            fp_mlp_forward(n_in, hidden, batch, p, x[o: o + batch], y, act)
            fp_mlp_backward(n_in, hidden, batch, p, x[o: o + batch], act, t[o: o + batch], grad, want_loss=False)
            step += 1
            fp_mlp_adam_step(npar, p, grad, adam, step, lr=lr)
        fp_mlp_forward(n_in, hidden, n_hold, p, x[n_fit:], hold_y, hold_act)
        hl = fp_mlp_backward(n_in, hidden, n_hold, p, x[n_fit:], hold_act, t[n_fit:], hold_grad)
        history.append(hl)
        if log:
            log(f"epoch {ep}: hold-out mse {hl:.4f}")
        if hl < best:
            best, bad = hl, 0
            best_p.copy_(p)
        else:
            bad += 1
            if bad >= patience:
                break
    _sync()
    t_train = time.perf_counter() - t1
    model = {"target": target, "k": k, "log_mean": log_mean, "log_std": log_std,
             "log_shift": math.log(f_mean[k - 1])}
    # c and the correlation on the hold-out
    g_hold = link(model, predict(n_in, hidden, best_p, x[n_fit:]))
    st = fp_cv_holdout(tr[2 * n_fit:], g_hold, n_hold, k)
    c, rho = st["c"], st["rho"]
    model.update({"params": best_p, "n_in": n_in, "hidden": hidden, "scale": scale, "c": c, "rho_holdout": rho,
            "holdout_mse": best, "epochs_run": len(history), "history": history,
            "t_data_s": t_data, "t_train_s": t_train, "n_train": n_train})
    return model


def estimate(ens, model, k=2, n_exact=10000, n_surrogate=1000000, seed_exact=0xB0B, seed_surr=0xCAFE):
    """F_CV and the plain estimate on fresh pairs, with wall times of both phases."""
    n_in, hidden, params, c = model["n_in"], model["hidden"], model["params"], model["c"]
    _sync()
    t0 = time.perf_counter()
    tr, x = exact_traces(ens, n_exact, seed_exact, 0, with_features=True)
    g_b = link(model, predict(n_in, hidden, params, x))
    _sync()
    t_exact = time.perf_counter() - t0
    t1 = time.perf_counter()
    g_c = link(model, surrogate_values(ens, params, hidden, n_surrogate, seed_surr))
    _sync()
    t_surr = time.perf_counter() - t1
    f_cv, se_cv = fp_frame_potential_cv(tr, g_b, n_exact, g_c, n_surrogate, k, c)
    f_pl, se_pl = fp_frame_potential(tr, n_exact, k)
    f_pl, se_pl = f_pl[k - 1], se_pl[k - 1]
    tau_e, tau_s = t_exact / n_exact, t_surr / n_surrogate
    # The fallback rule, decided from the hold-out's correlation and the unit
    # costs only (it cannot bias the estimate).
    use_cv, predicted_ratio = fp_cv_choose(model["rho_holdout"], tau_e, tau_s)
    f_used, se_used = (f_cv, se_cv) if use_cv else (f_pl, se_pl)
    # time to 1 % relative standard error, from the exact pairs' statistics
    st_b = fp_cv_holdout(tr, g_b, n_exact, k)
    _, var_g = fp_moments_f32(g_c, n_surrogate)
    t_plain_1pct, t_cv_1pct = fp_cv_time_to_rel_se(st_b, c, var_g, 0.01, tau_e, tau_s)
    var_f = st_b["var_f"]
    return {"F": f_used, "SE": se_used, "used_control_variate": use_cv,
            "predicted_time_ratio_from_holdout": predicted_ratio,
            "F_cv": f_cv, "SE_cv": se_cv, "F_plain": f_pl, "SE_plain": se_pl, "c": c,
            "t_exact_s": t_exact, "t_surrogate_s": t_surr, "n_exact": n_exact, "n_surrogate": n_surrogate,
            "sec_per_exact_pair": tau_e, "sec_per_surrogate": tau_s,
            "var_f": var_f, "var_g": var_g, "rho_exact_pairs": st_b["rho"], "stats_exact_pairs": st_b,
            "rel_se_cv": se_cv / f_cv if f_cv else None, "rel_se_plain": se_pl / f_pl if f_pl else None,
            "time_to_1pct_plain_s": t_plain_1pct, "time_to_1pct_cv_s": t_cv_1pct,
            "variance_reduction_per_time": t_plain_1pct / t_cv_1pct if t_cv_1pct > 0 else None,
            "cv_minus_plain_in_plain_se": (f_cv - f_pl) / se_pl if se_pl else None}


def experiment(n=40, layers=6, k=2, hidden=256, n_train=65536, n_exact=10000, n_surrogate=1000000, epochs=30,
               log=None, target="log"):
    ens = Ensemble(HEA, n, layers)
    model = train_surrogate(ens, k=k, hidden=hidden, n_train=n_train, epochs=epochs, log=log, target=target)
    res = estimate(ens, model, k=k, n_exact=n_exact, n_surrogate=n_surrogate)
    res.update({k_: v for k_, v in model.items() if k_ not in ("params",)})
    res["rho_holdout_link"] = model["rho_holdout"]
    res["workload"] = f"hea_n{n}_L{layers}_cv"
    return res
