"""The set distance of the time-to-MMD measurement (CPU): the unbiased MMD^2
with dimensions standardised by the reference sample's spread and the
Gaussian kernel exp(-|d|^2 / 2), against the closed form for normal
samples: for x ~ N(0, I_6) against y ~ N(delta, I_6) the population value
is 2 * 3^-3 * (1 - exp(-|delta|^2 / 6)), so MMD = 0.05 is a shift of about
0.45 standard deviations."""
import math

import numpy as np
import pytest
import torch

from paper_2106_03287_amd import train_proposal as TP


def _sets(seed, n, K, shift, scale):
    rng = np.random.default_rng(seed)
    Y = rng.standard_normal((n, K, 6)) * scale
    X = rng.standard_normal((n, K, 6)) * scale
    X[..., 0] += shift * scale[0]
    return torch.from_numpy(X), torch.from_numpy(Y)


SCALE = np.array([0.02, 0.03, 0.01, 0.05, 0.1, 0.02])   # m, rad: a tight posterior


@pytest.mark.parametrize("shift", [0.0, 0.45, 1.0, 3.0])
def test_mmd_matches_the_closed_form_for_shifted_normals(shift):
    X, Y = _sets(1, 8, 400, shift, SCALE)
    got = TP.mmd_u2(X, Y).numpy()
    want = 2 * 3 ** -3 * (1 - math.exp(-shift ** 2 / 6))
    # the sample standard deviations of 400 draws stand in for the true ones
    assert abs(got.mean() - want) < 0.004 + 0.1 * want
    if shift == 0.0:
        assert TP.aggregate_mmd(got) < 0.05


def test_mmd_wraps_angles_and_ignores_particle_order():
    X, Y = _sets(2, 4, 100, 0.5, SCALE)
    base = TP.mmd_u2(X, Y)
    Xw = X.clone()
    Xw[..., 3:] += 2 * math.pi * torch.from_numpy(np.random.default_rng(3).integers(-2, 3, (4, 100, 3)).astype(np.float64))
    torch.testing.assert_close(TP.mmd_u2(Xw, Y), base, rtol=1e-9, atol=1e-12)
    perm = torch.from_numpy(np.random.default_rng(4).permutation(100))
    torch.testing.assert_close(TP.mmd_u2(X[:, perm], Y), base, rtol=1e-12, atol=1e-15)


def test_aggregate_is_the_root_of_the_clipped_mean():
    assert TP.aggregate_mmd([0.0025, 0.0025]) == pytest.approx(0.05)
    assert TP.aggregate_mmd([-0.001, 0.0005]) == 0.0
