"""The library's posterior scores (stein_icp_posterior_scores, host code)
against the oracle's on seeded sample sets: KL within 1e-10 relative (the
library takes Cholesky factors, the oracle inverses and determinants), OVL
within 1e-9 (the library in closed form from the densities' crossing points,
the oracle by quadrature). No device needed."""
import numpy as np
import pytest

from oracle import scores_oracle as SO
from paper_2106_03287_amd import stein_icp as S


def _sets(seed, na=100, nb=1000, straddle=False):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(6, 6)) * 0.1
    B = rng.normal(size=(6, 6)) * 0.12
    mb = rng.normal(size=6) * 0.2
    ma = mb + rng.normal(size=6) * 0.05
    if straddle:
        ma[3:] += np.pi
        mb[3:] += np.pi
    a = ma + rng.normal(size=(na, 6)) @ A.T
    b = mb + rng.normal(size=(nb, 6)) @ B.T
    a[:, 3:] = SO.wrap(a[:, 3:])
    b[:, 3:] = SO.wrap(b[:, 3:])
    return a, b


@pytest.mark.parametrize("seed,straddle", [(0, False), (1, False), (2, True), (3, True)])
def test_scores_match_the_oracle(seed, straddle):
    a, b = _sets(seed, straddle=straddle)
    kl, ovl = S.stein_icp_posterior_scores(a, b)
    okl, oovl = SO.scores(a, b)
    np.testing.assert_allclose(kl, okl, rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(ovl, oovl, rtol=0, atol=1e-9)
    assert np.all((ovl > 0) & (ovl <= 1))


def test_scores_of_identical_sets_and_of_disjoint_sets():
    a, b = _sets(4)
    kl, ovl = S.stein_icp_posterior_scores(b, b)
    np.testing.assert_allclose(kl, 0.0, atol=1e-12)
    np.testing.assert_allclose(ovl, 1.0, atol=1e-12)
    far = a.copy()
    far[:, :3] += 50.0
    kl, ovl = S.stein_icp_posterior_scores(far, b)
    assert kl[0] > 1e3 and np.all(ovl[:3] < 1e-12)


def test_equal_and_nearly_equal_widths():
    rng = np.random.default_rng(6)
    z = rng.normal(size=(300, 6))
    a, b = z * 0.1, z * 0.1 + 0.02      # equal sample widths, shifted
    kl, ovl = S.stein_icp_posterior_scores(a, b)
    np.testing.assert_allclose(ovl, SO.scores(a, b)[1], atol=1e-9)
    b2 = b * (1 + 1e-13)
    np.testing.assert_allclose(S.stein_icp_posterior_scores(a, b2)[1], SO.scores(a, b2)[1], atol=1e-9)


def test_invalid_sample_sets_are_rejected():
    a, b = _sets(7)
    with pytest.raises(S.SteinICPError, match="at least 2"):
        S.stein_icp_posterior_scores(a[:1], b)
    bad = a.copy()
    bad[3, 2] = np.nan
    with pytest.raises(S.SteinICPError, match="non-finite"):
        S.stein_icp_posterior_scores(bad, b)
    flat = a.copy()
    flat[:, 1] = 0.25                     # zero variance in y: singular covariance
    with pytest.raises(S.SteinICPError, match="positive definite"):
        S.stein_icp_posterior_scores(flat, b)
