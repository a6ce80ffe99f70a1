"""Monte Carlo frame-potential estimator (oracle side).

TEST INFRASTRUCTURE (CPU oracle; see oracle/__init__.py).

F^(k) is approximated by the sample mean of |Tr(U^dagger V)|^{2k} over
independently sampled pairs (Sec. II.A, Monte Carlo equation); the same trace
values serve every k (Supplementary Figures, "Sample sizes").  The standard
error is the sample standard deviation over sqrt(N); the paper's uncertainty
analysis resamples N values with replacement 300 times (Supplementary
Methods, bootstrapping).
"""

import numpy as np


def frame_potential(tr, k_max):
    a = np.abs(np.asarray(tr, dtype=np.complex128)) ** 2
    n = a.size
    f = np.empty(k_max)
    se = np.empty(k_max)
    for k in range(1, k_max + 1):
        x = a ** k
        f[k - 1] = x.mean()
        se[k - 1] = x.std(ddof=1) / np.sqrt(n) if n > 1 else np.nan
    return f, se


def bootstrap(tr, k, resamples=300, seed=0):
    """Bootstrap distribution of the k-th frame-potential estimate."""
    a = np.abs(np.asarray(tr, dtype=np.complex128)) ** (2 * k)
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, a.size, size=(resamples, a.size))
    return a[idx].mean(axis=1)


def control_variate(f_b, g_b, g_c, c):
    """F_CV = mean_B(f - c g) + c mean_C(g) and its standard error."""
    f_b = np.asarray(f_b, dtype=np.float64)
    g_b = np.asarray(g_b, dtype=np.float64)
    g_c = np.asarray(g_c, dtype=np.float64)
    r = f_b - c * g_b
    est = r.mean() + c * g_c.mean()
    var = r.var(ddof=1) / r.size + (c * c) * g_c.var(ddof=1) / g_c.size
    return est, np.sqrt(var)
