"""Statistical acceptance helpers shared by the pin and parity tests.

Per film, bins are compared by z-scores; a film passes when
  1. the number of |z| > 3 stays within the 99.9 % point of its binomial
     distribution (per-bin exceedance 0.27 % for normal z, or the Student-t
     tail when the standard errors come from `dof` degrees of freedom),
  2. max |z| is at most the two-sided Bonferroni bound for a 1 % family-wise
     false-alarm rate over M bins,
  3. sum z^2 (t-scores rescaled to unit variance) lies inside the central
     99.9 % interval of chi^2_M.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import stats


def check_z(z, label="", alpha=0.01, dof=None):
    z = np.asarray(z, float).ravel()
    z = z[np.isfinite(z)]
    M = z.size
    if M == 0:
        raise AssertionError(f"{label}: no bins to test")
    dist = stats.norm if dof is None else stats.t(dof)
    p3 = 2 * dist.sf(3.0)
    n3 = int(np.sum(np.abs(z) > 3))
    lim_n3 = int(stats.binom.ppf(0.999, M, p3))
    zmax = float(np.max(np.abs(z)))
    lim_max = float(dist.isf(alpha / (2 * M)))
    zz = z if dof is None or dof <= 2 else z * math.sqrt((dof - 2) / dof)
    chi2 = float(np.sum(zz * zz))
    lo, hi = stats.chi2.ppf([0.0005, 0.9995], M)
    msg = (f"{label}: M={M} n|z|>3={n3} (<= {lim_n3}) max|z|={zmax:.2f} (<= {lim_max:.2f}) "
           f"chi2={chi2:.1f} in [{lo:.1f},{hi:.1f}]")
    assert n3 <= lim_n3 and zmax <= lim_max and lo <= chi2 <= hi, msg
    return msg


def binom_z(count, n, p):
    se = math.sqrt(max(p * (1 - p), 1e-300) / n)
    return (count / n - p) / se


def multinomial_z(frac, n, p, min_expected=10):
    """Per-bin z of observed fractions vs expected probabilities; bins whose
    expected count is below min_expected are pooled into one."""
    frac = np.asarray(frac, float).ravel()
    p = np.asarray(p, float).ravel()
    keep = p * n >= min_expected
    z = list((frac[keep] - p[keep]) / np.sqrt(p[keep] * (1 - p[keep]) / n))
    pr = p[~keep].sum()
    if pr * n >= min_expected:
        z.append((frac[~keep].sum() - pr) / math.sqrt(pr * (1 - pr) / n))
    return np.array(z)


def escape_z(fa, na, fb, nb, min_count=10):
    """Per-bin z of two independent escape-film estimates (fractions of na and
    nb source photons, multinomial); bins with fewer than min_count photons on
    both sides are pooled into one."""
    fa = np.asarray(fa, float).ravel()
    fb = np.asarray(fb, float).ravel()
    keep = (fa * na >= min_count) | (fb * nb >= min_count)
    p = (fa * na + fb * nb) / (na + nb)
    var = p * (1 - p) * (1.0 / na + 1.0 / nb)
    z = list((fa[keep] - fb[keep]) / np.sqrt(var[keep]))
    ra, rb = fa[~keep].sum(), fb[~keep].sum()
    pr = (ra * na + rb * nb) / (na + nb)
    if pr * (na + nb) >= min_count:
        z.append((ra - rb) / math.sqrt(pr * (1 - pr) * (1.0 / na + 1.0 / nb)))
    return np.array(z)


def batch_z(a_batches, b_batches, min_nonzero=10):
    """z-scores (Welch) of two sets of batch-mean films (leading axis = batch).
    Bins where either side has fewer than min_nonzero nonzero batches are
    dropped, and bins where both variances vanish are skipped."""
    a = np.asarray(a_batches, np.float64)
    b = np.asarray(b_batches, np.float64)
    Ba, Bb = a.shape[0], b.shape[0]
    ma, mb = a.mean(0), b.mean(0)
    va = a.var(0, ddof=1) / Ba
    vb = b.var(0, ddof=1) / Bb
    nza = (a != 0).sum(0)
    nzb = (b != 0).sum(0)
    ok = (nza >= min_nonzero) & (nzb >= min_nonzero) & ((va + vb) > 0)
    z = (ma[ok] - mb[ok]) / np.sqrt(va[ok] + vb[ok])
    return z
