"""Pins of the posterior-score oracle (KL of normal fits, overlapping
coefficient) against things other than itself: numerical integration of the
KL integrand, Monte-Carlo estimates with scipy's densities, the equal-width
closed form of the overlap, and invariances of the angle handling."""
import numpy as np
import pytest
from scipy import integrate, stats

from oracle import scores_oracle as SO


def _rand_spd(rng, scale=1.0):
    A = rng.normal(size=(3, 3))
    return scale * (A @ A.T + 0.3 * np.eye(3))


def test_kl_of_a_distribution_with_itself_is_zero():
    rng = np.random.default_rng(0)
    m, S = rng.normal(size=3), _rand_spd(rng)
    assert abs(SO.kl_gauss(m, S, m, S)) < 1e-13


def test_kl_diagonal_case_matches_integrals_of_the_1d_integrand():
    """With diagonal covariances KL is the sum of 1-D KLs, each integrated
    numerically as the integral of p log(p / q)."""
    ma, mb = np.array([0.1, -0.3, 0.7]), np.array([0.5, 0.2, 0.4])
    sa, sb = np.array([0.2, 0.5, 1.1]), np.array([0.3, 0.35, 0.9])
    total = 0.0
    for d in range(3):
        p = stats.norm(ma[d], sa[d])
        q = stats.norm(mb[d], sb[d])
        val, _ = integrate.quad(lambda x: p.pdf(x) * (p.logpdf(x) - q.logpdf(x)), ma[d] - 20 * sa[d],
                                ma[d] + 20 * sa[d], limit=500, epsabs=1e-14)
        total += val
    got = SO.kl_gauss(ma, np.diag(sa ** 2), mb, np.diag(sb ** 2))
    np.testing.assert_allclose(got, total, rtol=1e-9)
    # a textbook value: KL(N(0, 1) || N(1, 1)) = 1/2 per dimension
    np.testing.assert_allclose(SO.kl_gauss(np.zeros(3), np.eye(3), np.ones(3), np.eye(3)), 1.5, rtol=1e-14)


def test_kl_full_covariance_matches_a_monte_carlo_estimate():
    rng = np.random.default_rng(1)
    ma, mb = rng.normal(size=3) * 0.3, rng.normal(size=3) * 0.3
    Sa, Sb = _rand_spd(rng, 0.5), _rand_spd(rng, 0.8)
    x = rng.multivariate_normal(ma, Sa, size=400_000)
    vals = stats.multivariate_normal(ma, Sa).logpdf(x) - stats.multivariate_normal(mb, Sb).logpdf(x)
    est, se = vals.mean(), vals.std() / np.sqrt(len(vals))
    got = SO.kl_gauss(ma, Sa, mb, Sb)
    assert abs(got - est) < 5 * se, (got, est, se)


def test_kl_is_not_symmetric():
    rng = np.random.default_rng(2)
    ma, mb, Sa, Sb = rng.normal(size=3), rng.normal(size=3), _rand_spd(rng, 0.2), _rand_spd(rng, 2.0)
    assert abs(SO.kl_gauss(ma, Sa, mb, Sb) - SO.kl_gauss(mb, Sb, ma, Sa)) > 1e-3


@pytest.mark.parametrize("delta,s", [(0.0, 1.0), (0.3, 0.2), (1.7, 0.9), (5.0, 0.4)])
def test_ovl_equal_widths_matches_the_closed_form(delta, s):
    """Two normals of equal width: OVL = 2 Phi(-|delta| / (2 s))."""
    got = SO.ovl_normal(0.2, s, 0.2 + delta, s)
    np.testing.assert_allclose(got, 2 * stats.norm.cdf(-abs(delta) / (2 * s)), rtol=1e-10, atol=1e-14)


def test_ovl_unequal_widths_matches_a_monte_carlo_estimate():
    """OVL = E_{x ~ f1} min(1, f2(x) / f1(x))."""
    rng = np.random.default_rng(3)
    for m1, s1, m2, s2 in [(0.0, 1.0, 0.5, 2.0), (0.1, 0.05, 0.12, 0.01), (-1.0, 0.3, 0.2, 0.7)]:
        x = rng.normal(m1, s1, 1_000_000)
        r = np.minimum(1.0, stats.norm(m2, s2).pdf(x) / stats.norm(m1, s1).pdf(x))
        est, se = r.mean(), r.std() / np.sqrt(len(r))
        got = SO.ovl_normal(m1, s1, m2, s2)
        assert abs(got - est) < 5 * se + 1e-12, (got, est, se)
        np.testing.assert_allclose(got, SO.ovl_normal(m2, s2, m1, s1), rtol=1e-10)


def test_ovl_bounds():
    assert abs(SO.ovl_normal(0.3, 0.2, 0.3, 0.2) - 1.0) < 1e-10
    assert SO.ovl_normal(0.0, 0.1, 10.0, 0.1) < 1e-12
    assert 0.0 < SO.ovl_normal(0.0, 0.1, 0.0, 3.0) < 1.0


def test_fit_is_affine_equivariant():
    rng = np.random.default_rng(4)
    z = rng.normal(size=(500, 3))
    A, c = rng.normal(size=(3, 3)), rng.normal(size=3)
    mz, Sz = SO.fit(z)
    mx, Sx = SO.fit(z @ A.T + c)
    np.testing.assert_allclose(mx, A @ mz + c, atol=1e-12)
    np.testing.assert_allclose(Sx, A @ Sz @ A.T, atol=1e-12)
    np.testing.assert_allclose(Sz, np.cov(z.T), atol=1e-15)


def test_scores_do_not_depend_on_the_angle_origin():
    """A set straddling +-pi scores as it does after turning every angle by
    the same offset: the angles are taken around the reference's circular
    mean."""
    rng = np.random.default_rng(5)
    b = np.concatenate([rng.normal(0, 0.05, (400, 3)), SO.wrap(rng.normal(np.pi, 0.05, (400, 3)))], axis=1)
    a = np.concatenate([rng.normal(0.01, 0.06, (100, 3)), SO.wrap(rng.normal(np.pi - 0.02, 0.04, (100, 3)))],
                       axis=1)
    assert (b[:, 3:] > 0).any() and (b[:, 3:] < 0).any()     # stored on both sides of +-pi
    kl0, ovl0 = SO.scores(a, b)
    shift = np.array([2.0, -1.5, 0.7])
    a1, b1 = a.copy(), b.copy()
    a1[:, 3:] = SO.wrap(a[:, 3:] + shift)
    b1[:, 3:] = SO.wrap(b[:, 3:] + shift)
    kl1, ovl1 = SO.scores(a1, b1)
    np.testing.assert_allclose(kl1, kl0, rtol=1e-9)
    np.testing.assert_allclose(ovl1, ovl0, rtol=1e-9)
    assert kl0[1] < 0.5     # not split at +-pi
