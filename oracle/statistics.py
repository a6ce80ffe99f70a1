"""Statistics of the frame-potential estimates (oracle side).

TEST INFRASTRUCTURE (CPU oracle; see oracle/__init__.py).

Follows the paper's uncertainty analysis and fitting (Supplementary Methods:
"Bootstrapping for uncertainty quantification", "Choice of curve fitting
region", "Determination of sample sizes"; main text, the exponential-decay
bound and the layers needed for an epsilon-approximate design):

* bootstrap: N traces resampled with replacement, the estimate recomputed
  per resample, 300 resamples;
* quantiles of a bootstrap distribution (median as the estimate);
* fit region: layers with 0 < (F - F_Haar) / F_Haar < 5;
* fit: F - F_Haar = A^2 exp(-2 l / C), i.e. log(F - F_Haar) linear in l
  (least squares), and the layers for epsilon:
      l = C (k n log q + log A + log(1/epsilon));
* adaptive sample size: stop once F exceeds F_Haar by z standard errors or
  the budget is spent; keep sampling while the estimate is unphysical.

Resampling indices come from the counter-based generator (philox.py):
resample r, draw i uses block b = i >> 1 with counter (b low 32 bits, b high
32 bits, r, 0xB0075A3B) and key = seed; draw i takes the 64-bit word
u = x0 + 2^32 x1 (i even) or x2 + 2^32 x3 (i odd) and the index
floor(u N / 2^64).
"""

import math

import numpy as np

from .philox import key_from_seed, philox4x32_10

BOOT_TAG = 0xB0075A3B
CONTINUE, STOP_RESOLVED, STOP_BUDGET = 0, 1, 2


def resample_indices(n, r, seed):
    """The n indices of resample r (int64 array)."""
    i = np.arange(n, dtype=np.uint64)
    b = i >> np.uint64(1)
    ctr = np.empty((n, 4), dtype=np.uint64)
    ctr[:, 0] = b & np.uint64(0xFFFFFFFF)
    ctr[:, 1] = b >> np.uint64(32)
    ctr[:, 2] = np.uint64(r)
    ctr[:, 3] = np.uint64(BOOT_TAG)
    x = philox4x32_10(ctr, key_from_seed(seed)).astype(np.uint64)
    odd = (i & np.uint64(1)) == np.uint64(1)
    lo = np.where(odd, x[:, 2], x[:, 0])
    hi = np.where(odd, x[:, 3], x[:, 1])
    # floor((hi 2^32 + lo) n / 2^64), exactly, in 64-bit pieces
    nn = np.uint64(n)
    h = (lo * nn) >> np.uint64(32)
    return ((hi * nn + h) >> np.uint64(32)).astype(np.int64)


def bootstrap_philox(tr, k_max, resamples, seed):
    """F^(k) of every resample: array (k_max, resamples), float64."""
    a = np.abs(np.asarray(tr, dtype=np.complex128)) ** 2
    out = np.empty((k_max, resamples))
    for r in range(resamples):
        s = a[resample_indices(a.size, r, seed)]
        for k in range(1, k_max + 1):
            out[k - 1, r] = np.mean(s ** k)
    return out


def quantile(sorted_values, q):
    """Quantile with linear interpolation between order statistics at
    position q (R - 1) of R sorted values."""
    v = np.asarray(sorted_values, dtype=np.float64)
    pos = q * (v.size - 1)
    lo = int(math.floor(pos))
    hi = min(lo + 1, v.size - 1)
    return float(v[lo] + (pos - lo) * (v[hi] - v[lo]))


def fit_region(f, f_haar, rel_dev_max=5.0):
    """Mask of the layers whose deviation (F - F_Haar)/F_Haar lies in (0, rel_dev_max)."""
    d = (np.asarray(f, dtype=np.float64) - f_haar) / f_haar
    return (d > 0.0) & (d < rel_dev_max)


def layers_to_epsilon(layers, f, f_haar, epsilon, n, q, k, rel_dev_max=5.0):
    """(l_epsilon, A, C) from the exponential fit over the fit region, or None
    with fewer than two points or a fit that does not decay."""
    layers = np.asarray(layers, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    m = fit_region(f, f_haar, rel_dev_max)
    if m.sum() < 2:
        return None
    x, y = layers[m], np.log(f[m] - f_haar)
    slope, icept = np.polyfit(x, y, 1)
    if not slope < 0.0:
        return None
    c = -2.0 / slope
    log_a = icept / 2.0
    return c * (k * n * math.log(q) + log_a + math.log(1.0 / epsilon)), math.exp(log_a), c


def adaptive_decision(f, se, f_haar, f_lower, z, n_done, n_max, seconds, max_seconds):
    """One evaluation of the sample-size rule: the budget ends sampling; an
    unphysical estimate (below F_Haar, or above the estimate at one layer
    less, f_lower, when given) keeps it going; an estimate z standard errors
    above F_Haar ends it; anything else keeps sampling."""
    if n_done >= n_max or seconds >= max_seconds:
        return STOP_BUDGET
    if f < f_haar or (f_lower is not None and f > f_lower):
        return CONTINUE
    if f - f_haar > z * se:
        return STOP_RESOLVED
    return CONTINUE
