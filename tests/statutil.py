"""Statistical acceptance rules for Monte Carlo count matrices.

A count matrix has up to millions of binomial entries, so a literal "every entry within 4
standard errors" fails by chance.  The rules applied (each reported):
  (i)   entries with |z| > 4 must not exceed E + 3 sqrt(E) + 1, E = P(|N(0,1)| > 4) * n_entries;
  (ii)  no entry below the Bonferroni level: exact two-sided binomial p-value >= 0.005 / n_entries;
  (iii) per-row chi-square goodness of fit, Bonferroni over rows.
A stated bias b (per entry, probability units) widens the null to [p - b, p + b].
"""
from __future__ import annotations

import numpy as np
from scipy import stats

P_Z4 = 2 * stats.norm.sf(4.0)  # 6.334e-5


def _two_sided_binom_p(k, n, p):
    p = np.clip(p, 0.0, 1.0)
    lo = stats.binom.cdf(k, n, p)
    hi = stats.binom.sf(k - 1, n, p)
    return np.minimum(1.0, 2 * np.minimum(lo, hi))


def vs_probabilities(counts, n, P, bias=0.0, alpha=0.005):
    """Counts (rows of n walks) against exact probabilities P (same shape)."""
    counts = np.asarray(counts, np.float64)
    P = np.asarray(P, np.float64)
    bias = np.broadcast_to(np.asarray(bias, np.float64), P.shape)
    phat = counts / n
    # the closest null inside [P - b, P + b]
    pn = np.clip(np.clip(phat, P - bias, P + bias), 0.0, 1.0)
    se = np.sqrt(np.maximum(pn * (1 - pn), 1.0 / n) / n)
    z = (phat - pn) / se
    n_ent = counts.size
    E = P_Z4 * n_ent
    n_z4 = int(np.sum(np.abs(z) > 4))
    pv = _two_sided_binom_p(counts, n, pn)
    rep = dict(n_entries=n_ent, n_z4=n_z4, z4_limit=E + 3 * np.sqrt(E) + 1,
               min_p=float(pv.min()), bonferroni=alpha / n_ent, max_abs_z=float(np.abs(z).max()))
    rep["ok"] = rep["n_z4"] <= rep["z4_limit"] and rep["min_p"] >= rep["bonferroni"]
    return rep


def two_sample(c1, n1, c2, n2, alpha=0.005):
    """Two independent binomial count matrices with a common p per entry: conditional exact test
    (given t = k1 + k2, k1 ~ Binomial(t, n1 / (n1 + n2))), plus the |z| > 4 tally."""
    c1 = np.asarray(c1, np.float64)
    c2 = np.asarray(c2, np.float64)
    t = c1 + c2
    w = n1 / (n1 + n2)
    pv = np.where(t > 0, _two_sided_binom_p(c1, t, w), 1.0)
    pooled = t / (n1 + n2)
    se = np.sqrt(np.maximum(pooled * (1 - pooled), 1e-300) * (1.0 / n1 + 1.0 / n2))
    z = np.where(t > 0, (c1 / n1 - c2 / n2) / se, 0.0)
    n_ent = c1.size
    E = P_Z4 * n_ent
    rep = dict(n_entries=n_ent, n_z4=int(np.sum(np.abs(z) > 4)), z4_limit=E + 3 * np.sqrt(E) + 1,
               min_p=float(pv.min()), bonferroni=alpha / n_ent, max_abs_z=float(np.abs(z).max()))
    rep["ok"] = rep["n_z4"] <= rep["z4_limit"] and rep["min_p"] >= rep["bonferroni"]
    return rep


def row_chi2(counts, n, P, alpha=0.005, min_expected=5.0):
    """Per-row chi-square goodness of fit against probabilities P; returns the smallest p-value
    and whether it clears the Bonferroni level over rows."""
    counts = np.asarray(counts, np.float64)
    P = np.asarray(P, np.float64)
    pmin = 1.0
    for c, p in zip(counts, P):
        e = n * p
        big = e >= min_expected
        obs = list(c[big])
        exp = list(e[big])
        if (~big).any():
            obs.append(c[~big].sum())
            exp.append(e[~big].sum())
        obs, exp = np.array(obs), np.array(exp)
        keep = exp > 0
        chi = np.sum((obs[keep] - exp[keep]) ** 2 / exp[keep])
        dof = max(int(keep.sum()) - 1, 1)
        pmin = min(pmin, float(stats.chi2.sf(chi, dof)))
    return dict(min_p=pmin, ok=pmin >= alpha / counts.shape[0])
