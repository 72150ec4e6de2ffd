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
