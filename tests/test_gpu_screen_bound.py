"""The matrix-core screens' error bounds, measured on the hardware: the raw
screened values |q|^2 + |r|^2 - 2 q.r of both screens (the library's own
fragments and matrix products, stein_icp_screen_values) against the exact
squared distance of the FP32 points, on inputs built to stress the bounds:
queries and references on one line far from the centroid (the cross term
then nearly cancels the norms), LiDAR queries at 80 m, scales from 1 mm to
1 km. The matrix core's order and rounding of its additions are not
specified: the bounds allow each addition to lose up to one FP32 ulp of its
partial sum. A sequential FP32 sum rounded to nearest stays within about a
tenth of the FP16 bound on these inputs (CPU emulation); the hardware's
errors come out several times larger than that, which is why the bounds do
not assume rounding to nearest. The measured ratios are printed and must
stay below 1."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2106_03287_amd import stein_icp as S

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _worst_ratio(q, ref, mode):
    vals, c0, e = S.stein_icp_screen_values(dev(q), dev(ref), mode)
    Sv = vals.cpu().numpy().astype(np.float64)
    q64, r64 = q.astype(np.float64), ref.astype(np.float64)
    F = ((q64[:, None, :] - r64[None, :, :]) ** 2).sum(-1)          # exact, from the FP32 points
    qc = np.sqrt(((q.astype(np.float32) - c0[:3]).astype(np.float64) ** 2).sum(1))
    rc = np.sqrt(((ref.astype(np.float32) - c0[:3]).astype(np.float64) ** 2).sum(1))
    if mode == S.NN_BF16_RERANK:
        bound = 52 * U * (qc[:, None] + float(c0[3])) ** 2 + 6.2 * U * F
    else:
        span = qc[:, None] + rc[None, :]
        s = 2.0 ** -e
        bound = 50 * U * span ** 2 + 2.0 ** -22 * (span + s) * s
    bound = bound + 4 * U * F          # the FP32 distance against the exact one
    ok = np.isfinite(Sv)
    assert ok.any()
    return float((np.abs(Sv - F)[ok] / bound[ok]).max()), int((~ok).sum())


def _collinear(seed, far):
    rng = np.random.default_rng(seed)
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    cluster = rng.normal(0, 0.01, (1500, 3))
    line_r = np.linspace(far / 6, far, 500)[:, None] * u + rng.normal(0, 1e-4, (500, 3))
    line_q = np.linspace(far / 3, 1.3 * far, 700)[:, None] * u
    ref = np.concatenate([cluster, line_r])
    q = np.concatenate([line_q, line_r[::5] + rng.normal(0, 1e-5, (100, 3))])
    return q, ref


@pytest.mark.parametrize("mode", [S.NN_BF16_RERANK, S.NN_F16_RERANK])
def test_screened_values_stay_within_the_bound(mode):
    worst = {}
    for far in (1.0, 10.0, 60.0):
        worst[f"collinear {far} m"] = _worst_ratio(*_collinear(int(far), far), mode)
    prob = synth.make_problem("lidar", 0, K=1, T=1)
    rng = np.random.default_rng(12)
    sel = rng.choice(len(prob.pair.src), 600, replace=False)
    q = oracle.transform(prob.theta0[0], prob.pair.src[sel])
    ref = prob.pair.ref[rng.choice(len(prob.pair.ref), 3000, replace=False)]
    worst["lidar"] = _worst_ratio(q, ref, mode)
    for sc in (1e-3, 1.0, 1e3):
        r = np.random.default_rng(int(sc * 1000) + 5)
        ref = r.uniform(-sc, sc, (2000, 3)) + sc * 3
        q = np.concatenate([ref[:300] + r.normal(0, sc * 1e-3, (300, 3)), r.uniform(-2 * sc, 2 * sc, (300, 3))])
        worst[f"uniform {sc} m"] = _worst_ratio(q, ref, mode)
    print(f"mode {mode}: measured error / bound " + ", ".join(f"{k} {v[0]:.3f}" for k, v in worst.items()),
          flush=True)
    for k, (ratio, unscreened) in worst.items():
        assert ratio <= 1.0, k
        if mode == S.NN_BF16_RERANK:
            assert unscreened == 0
