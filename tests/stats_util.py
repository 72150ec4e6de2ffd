"""Goodness-of-fit helpers shared by the statistical tests."""
import numpy as np
from scipy import stats


def chi2_pvalue(samples, probs, min_expected=5.0):
    """Pearson chi-square of integer samples against a pmf dict/array.

    Cells with small expected counts are pooled (ascending order) until each
    pooled cell expects at least ``min_expected``; the remainder of the support
    becomes one tail cell."""
    samples = np.asarray(samples).ravel()
    n = samples.size
    if isinstance(probs, dict):
        keys = sorted(probs)
        p = np.array([probs[k] for k in keys])
    else:
        keys = list(range(len(probs)))
        p = np.asarray(probs, dtype=float)
    counts = {k: 0 for k in keys}
    other = 0
    vals, cnt = np.unique(samples, return_counts=True)
    for v, c in zip(vals, cnt):
        if int(v) in counts:
            counts[int(v)] += int(c)
        else:
            other += int(c)
    obs, exp = [], []
    acc_o, acc_e = 0, 0.0
    for k, pk in zip(keys, p):
        acc_o += counts[k]
        acc_e += n * pk
        if acc_e >= min_expected:
            obs.append(acc_o)
            exp.append(acc_e)
            acc_o, acc_e = 0, 0.0
    tail_e = max(n - sum(exp), 0.0)
    tail_o = n - sum(obs)
    if tail_e >= min_expected or not exp:
        obs.append(tail_o)
        exp.append(tail_e)
    else:
        obs[-1] += tail_o
        exp[-1] += tail_e
    obs = np.asarray(obs, dtype=float)
    exp = np.asarray(exp, dtype=float)
    if len(obs) < 2:
        return 1.0
    stat = float(np.sum((obs - exp) ** 2 / np.maximum(exp, 1e-300)))
    return float(stats.chi2.sf(stat, len(obs) - 1))


def z_mean(samples, mean):
    s = np.asarray(samples, dtype=float)
    se = s.std(ddof=1) / np.sqrt(s.size)
    return abs(s.mean() - mean) / se if se > 0 else (0.0 if s.mean() == mean else np.inf)


def z_var(samples, var):
    """|sample variance - var| in units of its standard error (4th-moment SE)."""
    s = np.asarray(samples, dtype=float)
    n = s.size
    d = s - s.mean()
    m2 = np.mean(d ** 2)
    m4 = np.mean(d ** 4)
    se = np.sqrt(max(m4 - m2 ** 2, 1e-300) / n)
    return abs(s.var(ddof=1) - var) / se


def ensemble_z(a, b):
    """Per-cell z statistics between two independent ensembles.

    ``a`` and ``b`` are [S][N][T] sample arrays (trajectories last).  For every
    (sample, species) cell: z of the difference of means, sqrt(v_a/n_a + v_b/n_b)
    as its standard error, and z of the difference of the unbiased variances,
    each variance's standard error taken from its fourth central moment.
    Returns (z_mean [S][N], z_var [S][N], both_constant [S][N]); cells where both
    ensembles are constant get z = 0 when they agree and inf when not."""
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    na, nb = a.shape[-1], b.shape[-1]
    ma, mb = a.mean(-1), b.mean(-1)
    da, db = a - ma[..., None], b - mb[..., None]
    m2a, m2b = np.mean(da ** 2, -1), np.mean(db ** 2, -1)
    m4a, m4b = np.mean(da ** 4, -1), np.mean(db ** 4, -1)
    va, vb = m2a * na / (na - 1), m2b * nb / (nb - 1)
    const = (m2a == 0) & (m2b == 0)
    se_m = np.sqrt(va / na + vb / nb)
    se_v = np.sqrt(np.maximum(m4a - m2a ** 2, 0) / na + np.maximum(m4b - m2b ** 2, 0) / nb)
    with np.errstate(divide="ignore", invalid="ignore"):
        zm = np.where(se_m > 0, np.abs(ma - mb) / se_m, 0.0)
        zv = np.where(se_v > 0, np.abs(va - vb) / se_v, 0.0)
    zm = np.where(const, np.where(ma == mb, 0.0, np.inf), zm)
    zv = np.where(const, 0.0, zv)
    return zm, zv, const
