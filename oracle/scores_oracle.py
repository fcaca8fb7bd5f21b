"""Scores of a pose posterior against a Monte-Carlo ground truth, written
from the paper's description of its quality measures (Sec. V-A): the
Kullback-Leibler divergence and the overlapping coefficient between the
distribution a method obtains and the ground-truth samples.

TEST INFRASTRUCTURE ONLY: imported by the test suite and the benchmark's
reporting of the Monte-Carlo workload's oracle check; the product path never
imports it. Plain NumPy / SciPy in FP64.

Readings (the paper names the measures and their sources, not formulas):
 - The KL divergence is taken between normal fits of the two sample sets (the
   paper notes that its KL is computed from the samples' covariance), for the
   translations and the rotations separately (its figures report the two
   separately), in the direction KL(estimate || ground truth).
 - Sample covariance with the n - 1 denominator.
 - OVL is the integral of min(f, g) of the normal fits of one coordinate (the
   cited measure is defined for univariate normal densities); here by
   adaptive quadrature of that integral.
 - Angles are first taken within pi of the ground truth's circular mean, so
   that a set straddling +-pi is not split.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate, optimize


def wrap(a):
    return np.arctan2(np.sin(a), np.cos(a))


def circular_mean(angles):
    """Per-column circular mean of an (n, d) array of angles."""
    return np.arctan2(np.sin(angles).sum(axis=0), np.cos(angles).sum(axis=0))


def fit(x, centre=None):
    """Sample mean and covariance (n - 1) of the rows of x; with ``centre``
    each value v becomes centre + wrap(v - centre) first."""
    x = np.asarray(x, dtype=np.float64)
    if centre is not None:
        x = centre + wrap(x - centre)
    return x.mean(axis=0), np.cov(x.T, ddof=1)


def kl_gauss(ma, Sa, mb, Sb):
    """KL(N(ma, Sa) || N(mb, Sb)), the closed form of the expectation under
    N(ma, Sa) of log N(ma, Sa) - log N(mb, Sb)."""
    k = len(ma)
    iSb = np.linalg.inv(Sb)
    d = np.asarray(mb) - np.asarray(ma)
    _, lda = np.linalg.slogdet(Sa)
    _, ldb = np.linalg.slogdet(Sb)
    return 0.5 * (np.trace(iSb @ Sa) + d @ iSb @ d - k + ldb - lda)


def normal_logpdf(x, m, s):
    return -0.5 * ((x - m) / s) ** 2 - np.log(s * np.sqrt(2.0 * np.pi))


def normal_pdf(x, m, s):
    return np.exp(normal_logpdf(x, m, s))


def ovl_normal(m1, s1, m2, s2):
    """Integral over the real line of min(f1, f2) for two normal densities,
    by adaptive quadrature over +-14 standard deviations of both (the mass
    outside is below 1e-40), in pieces split where the two densities cross
    (located by a sign scan of log f1 - log f2 and bisection), so that the
    integrand is smooth on each piece."""
    lo = min(m1 - 14 * s1, m2 - 14 * s2)
    hi = max(m1 + 14 * s1, m2 + 14 * s2)
    g = lambda x: normal_logpdf(x, m1, s1) - normal_logpdf(x, m2, s2)  # noqa: E731
    xs = np.linspace(lo, hi, 20001)
    gs = g(xs)
    cuts = [lo]
    for i in np.nonzero(np.sign(gs[:-1]) * np.sign(gs[1:]) < 0)[0]:
        cuts.append(optimize.brentq(g, xs[i], xs[i + 1], xtol=1e-15, rtol=1e-15))
    cuts.append(hi)
    f = lambda x: min(normal_pdf(x, m1, s1), normal_pdf(x, m2, s2))  # noqa: E731
    total = 0.0
    for a, b in zip(cuts[:-1], cuts[1:]):
        pts = [p for p in (m1, m2) if a < p < b]
        val, _ = integrate.quad(f, a, b, points=pts or None, limit=500, epsabs=1e-16, epsrel=1e-13)
        total += val
    return total


def scores(a, b):
    """(kl[2], ovl[6]) of pose samples a against reference samples b (n x 6):
    KL of the translation and rotation normal fits, OVL per coordinate."""
    a = np.asarray(a, dtype=np.float64).reshape(-1, 6)
    b = np.asarray(b, dtype=np.float64).reshape(-1, 6)
    centre = circular_mean(b[:, 3:])
    kl, ovl = np.zeros(2), np.zeros(6)
    for g, sl in enumerate((slice(0, 3), slice(3, 6))):
        c = centre if g else None
        ma, Sa = fit(a[:, sl], c)
        mb, Sb = fit(b[:, sl], c)
        kl[g] = kl_gauss(ma, Sa, mb, Sb)
        for d in range(3):
            ovl[3 * g + d] = ovl_normal(ma[d], np.sqrt(Sa[d, d]), mb[d], np.sqrt(Sb[d, d]))
    return kl, ovl
