"""GPU parity of the learned-proposal kernels against the FP64 oracle, through
the C ABI: the BF16 matrix-core product (bit-exact where FP32 accumulation
is exact, within the FP32 accumulation bound otherwise), the network input
resampling, the forward pass, the set loss and its gradient, Adam, the
per-pair finiteness flags and the fallback signal."""
import os

import numpy as np
import pytest
import torch

from oracle import proposal_oracle as PO
from paper_2106_03287_amd import proposal as PR

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _cuda(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def _gemm_case(ta, tb, M, N, K, rng, integer):
    if integer:
        A = rng.integers(-4, 5, (K, M) if ta else (M, K)).astype(np.float32)
        B = rng.integers(-4, 5, (N, K) if tb else (K, N)).astype(np.float32)
        bias = rng.integers(-8, 9, N).astype(np.float32)
        C0 = rng.integers(-8, 9, (M, N)).astype(np.float32)
    else:
        A = rng.standard_normal((K, M) if ta else (M, K)).astype(np.float32)
        B = rng.standard_normal((N, K) if tb else (K, N)).astype(np.float32)
        bias = rng.standard_normal(N).astype(np.float32)
        C0 = rng.standard_normal((M, N)).astype(np.float32)
    return A, B, bias, C0


def _run_gemm(A, B, bias, C0, ta, tb, relu, acc, splits):
    M, N = C0.shape
    Cd = _cuda(C0)
    ws = torch.empty(max(splits, 1) * M * N, dtype=torch.float32, device="cuda") if splits > 1 else None
    PR.stein_icp_gemm_bf16(_cuda(A), _cuda(B), Cd, ta=ta, tb=tb, bias=None if bias is None else _cuda(bias),
                           relu=relu, accumulate=acc, splits=splits, workspace=ws)
    torch.cuda.synchronize()
    return Cd.cpu().numpy().astype(np.float64)


def _oracle_gemm(A, B, bias, C0, ta, tb, relu, acc):
    opA = A.T if ta else A
    opB = B.T if tb else B
    out = PO.matmul(opA.astype(np.float64), opB.astype(np.float64))
    if bias is not None:
        out = out + bias
    if relu:
        out = np.maximum(out, 0)
    return out + C0 if acc else out


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("M,N,K,splits", [(1, 1, 1, 1), (65, 70, 33, 1), (130, 64, 96, 1), (3, 64, 1000, 7),
                                          (64, 200, 0, 1), (257, 129, 300, 3)])
def test_gemm_is_exact_when_fp32_accumulation_is(ta, tb, M, N, K, splits):
    rng = np.random.default_rng(M * 7919 + N * 31 + K + 2 * ta + tb)
    A, B, bias, C0 = _gemm_case(ta, tb, M, N, K, rng, integer=True)
    for relu, acc, use_bias in [(0, 0, False), (1, 0, True), (0, 1, True), (1, 1, False)]:
        b = bias if use_bias else None
        got = _run_gemm(A, B, b, C0, ta, tb, relu, acc, splits)
        want = _oracle_gemm(A, B, b, C0, ta, tb, relu, acc)
        assert np.array_equal(got, want), (relu, acc, use_bias)


@pytest.mark.parametrize("ta,tb,M,N,K,splits", [(0, 0, 300, 200, 512, 1), (1, 0, 128, 256, 4000, 16),
                                                (0, 1, 96, 64, 256, 1), (1, 1, 70, 33, 129, 2)])
def test_gemm_rounds_operands_to_bf16_and_accumulates_in_fp32(ta, tb, M, N, K, splits):
    rng = np.random.default_rng(K + M)
    A, B, bias, C0 = _gemm_case(ta, tb, M, N, K, rng, integer=False)
    got = _run_gemm(A, B, None, C0, ta, tb, 0, 0, splits)
    opA = PO.bf16_round(A.T if ta else A)
    opB = PO.bf16_round(B.T if tb else B)
    want = opA @ opB
    # FP32 summation of K exact products: |error| <= (K + 1) u sum |a b|
    bound = (K + 1) * U32 * (np.abs(opA) @ np.abs(opB)) + 1e-30
    assert np.all(np.abs(got - want) <= bound)
    # the BF16 rounding is really applied: the unrounded product is farther
    # away than the accumulation bound allows
    plain = (A.T if ta else A).astype(np.float64) @ (B.T if tb else B).astype(np.float64)
    assert np.any(np.abs(got - plain) > bound)


def _model(K, P, Bmax, params):
    cfg = PR.stein_icp_proposal_default_config(num_particles=K, points=P, max_batch=Bmax)
    return PR.Proposal(cfg, params)


def _params(K, seed):
    rng = np.random.default_rng(seed)
    p = PR.init_params(K, seed=seed, head_scale=1.0).astype(np.float64)
    blocks = PO.unpack(p, K)
    for k in ("b1", "b2", "b3", "b4", "b5"):
        blocks[k] = rng.standard_normal(blocks[k].shape) * 0.1
    return PO.pack(blocks, K).astype(np.float32)


def _clouds(B, P, seed):
    rng = np.random.default_rng(seed)
    c = rng.uniform(-0.5, 0.5, (B, 2, P, 3))
    c[:, :, :, 2] *= 0.3
    return c.astype(np.float32)


def test_prepare_matches_the_oracle_resampling():
    m = _model(4, 1000, 1, _params(4, 1))
    rng = np.random.default_rng(2)
    for n in (1, 7, 999, 1000, 1001, 20000):
        xyz = rng.standard_normal((n, 3)).astype(np.float32)
        out = m.prepare(_cuda(xyz))
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), PO.subsample(xyz, 1000)), n
    m.close()


@pytest.mark.parametrize("K,P,B", [(100, 300, 3), (7, 64, 1), (100, 4096, 2)])
def test_forward_matches_the_oracle(K, P, B):
    params = _params(K, 3)
    clouds = _clouds(B, P, 4)
    m = _model(K, P, B, params)
    y, bad = m.forward(_cuda(clouds))
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    want = PO.forward(params, clouds, K)["Y"]
    assert not bad.cpu().numpy().any()
    scale = np.abs(want).max()
    err = np.abs(y - want).max() / scale
    print(f"forward K={K} P={P} B={B}: max |err| / max |y| = {err:.3e}")
    # FP32 accumulation against FP64 (each product within (K + 1) 2^-24 of
    # its sum of |terms|, K <= 512), and rare BF16 rounding flips of
    # activations that sit within that error of a rounding boundary
    assert err < 1e-4
    assert np.linalg.norm(y - want) <= 1e-5 * np.linalg.norm(want)
    m.close()


@pytest.mark.parametrize("P,reps,cloud_seed", [(8, 1, 4), (1, 1, 0), (8, 8, 4), (1, 64, 0)])
def test_loss_and_gradient_match_the_oracle(P, reps, cloud_seed):
    K, B = 8, 2
    params = _params(K, 5)
    # a case whose max-pool decisions all clear the tie by 1e-3, ten times
    # what an FP32-versus-FP64 difference can move a BF16 operand's product
    # (one BF16 ulp, 2^-7 relative, of terms of size 0.1 or less). Repeating
    # the P points `reps` times gives exact ties between copies, which both
    # sides break towards the first copy; P reps = 64 takes the path that
    # pools inside the last per-point product.
    base = np.random.default_rng(cloud_seed).uniform(-1, 1, (B, 2, P, 3)).astype(np.float32)
    assert PO.pool_margin(PO.forward(params, base, K)) > 1e-3
    clouds = np.tile(base, (1, 1, reps, 1))
    P = P * reps
    rng = np.random.default_rng(7)
    targets = rng.standard_normal((B, K, 6)) * 0.3
    sigma = np.array([[0.1] * 3 + [0.2] * 3, [0.4] * 3 + [0.8] * 3])
    cfg = PR.stein_icp_proposal_default_config(num_particles=K, points=P, max_batch=B, loss_sigma=sigma)
    m = PR.Proposal(cfg, params)
    loss, grad = m.loss(_cuda(clouds), _cuda(targets, torch.float64), grad=True)
    torch.cuda.synchronize()
    loss, grad = loss.cpu().numpy(), grad.cpu().numpy().astype(np.float64)
    want_loss, want_grad, cache = PO.loss_and_grad(params, clouds, targets, K, sigma)
    assert np.allclose(loss, want_loss, rtol=1e-5, atol=0)
    rels = {}
    for name, (o, s) in PO.layout(K).items():
        n = int(np.prod(s))
        g, w = grad[o:o + n], want_grad[o:o + n]
        rels[name] = np.linalg.norm(g - w) / np.linalg.norm(w)
    print("grad rel err " + " ".join(f"{k} {v:.1e}" for k, v in rels.items()))
    # both sides take the dense chain rule with BF16 operands in every matrix
    # product, so they differ by the device's FP32 sums: (n + 1) 2^-24 of the
    # summed magnitudes for n terms (n <= 1024 here, 6e-5 at worst, about
    # sqrt(n) 2^-24 = 2e-6 norm-wise for terms of mixed sign). An operand
    # whose FP32 and FP64 values straddle a BF16 rounding boundary would move
    # one term by 2^-8; these seeded cases (deterministic on the device) have
    # none, and every block lies within 1e-7
    for name, rel in rels.items():
        assert rel < 1e-5, name
    m.close()


def test_adam_step_matches_the_oracle():
    K, P, B = 4, 32, 2
    params = _params(K, 8)
    clouds = _clouds(B, P, 9)
    targets = np.random.default_rng(10).standard_normal((B, K, 6)) * 0.3
    m = _model(K, P, B, params)
    w = params.astype(np.float64)
    mom = np.zeros_like(w)
    vel = np.zeros_like(w)
    for t in (1, 2, 3):
        _, g = m.loss(_cuda(clouds), _cuda(targets, torch.float64), grad=True)
        m.adam(1e-3)
        torch.cuda.synchronize()
        g = g.cpu().numpy().astype(np.float64)
        w, mom, vel = PO.adam(w, g, mom, vel, t, lr=1e-3)
        mom, vel = mom.astype(np.float32).astype(np.float64), vel.astype(np.float32).astype(np.float64)
        w = w.astype(np.float32).astype(np.float64)
        got = m.params().cpu().numpy().astype(np.float64)
        assert np.allclose(got, w, rtol=0, atol=1e-6), t
        w = got     # continue from the device state
    m.close()


def test_set_distance_matches_the_oracle():
    rng = np.random.default_rng(11)
    B, K = 4, 100
    X = rng.standard_normal((B, K, 6)) * 0.2
    Y = rng.standard_normal((B, K, 6)) * 0.2
    Y[0] = X[0]
    Y[1, :, 3:] = X[1, :, 3:] + 2 * np.pi
    Y[1, :, :3] = X[1, :, :3]
    sigma = np.array([[0.05] * 3 + [0.1] * 3, [0.2] * 3 + [0.4] * 3, [1.0] * 6])
    got = PR.stein_icp_proposal_mmd(_cuda(X, torch.float64), _cuda(Y, torch.float64), sigma).cpu().numpy()
    want = np.array([PO.mmd2(X[b], Y[b], sigma) for b in range(B)])
    assert np.allclose(got, want, rtol=1e-12, atol=1e-15)
    assert abs(got[0]) < 1e-15 and abs(got[1]) < 1e-12


def test_nonfinite_outputs_are_flagged_per_pair_and_trigger_the_fallback():
    K, P, B = 10, 128, 3
    # all weights positive and clouds in the positive octant: a pair whose
    # coordinates overflow FP32 in the first product stays +inf to the end
    params = np.abs(_params(K, 12))
    clouds = np.abs(_clouds(B, P, 13))
    clouds[1, 1, 5, :] = 3.0e38
    m = _model(K, P, B, params)
    y, bad = m.forward(_cuda(clouds))
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    assert list(bad.cpu().numpy()) == [0, 1, 0]
    assert np.isfinite(y[0]).all() and np.isfinite(y[2]).all() and not np.isfinite(y[1]).all()
    src = _cuda(clouds[0, 0])
    ref = _cuda(clouds[0, 1])
    parts, fb = m.propose(src, ref)
    torch.cuda.synchronize()
    assert not fb
    assert np.array_equal(parts.cpu().numpy(), y[0])
    bad_params = params.copy()
    bad_params[-1] = np.nan        # a bias of the last layer
    m.set_params(bad_params)
    _, fb = m.propose(src, ref)
    assert fb
    m.close()


def test_training_steps_reduce_the_loss():
    K, P, B = 16, 256, 4
    params = PR.init_params(K, seed=14)
    clouds = _clouds(B, P, 15)
    rng = np.random.default_rng(16)
    centres = rng.uniform(-0.1, 0.1, (B, 1, 6))
    targets = centres + rng.standard_normal((B, K, 6)) * 0.01
    cfg = PR.stein_icp_proposal_default_config(num_particles=K, points=P, max_batch=B)
    m = PR.Proposal(cfg, params)
    c, t = _cuda(clouds), _cuda(targets, torch.float64)
    first = float(m.loss(c, t).mean())
    for _ in range(150):
        m.loss(c, t)
        m.adam(1e-3)
    last = float(m.loss(c, t).mean())
    print(f"training loss {first:.4f} -> {last:.4f}")
    assert last < 0.5 * first
    m.close()


def test_trained_proposal_reaches_plain_300_iteration_quality_in_30_iterations():
    """The committed weights on the first 8 pairs of the held-out split (4
    cuboid, 4 Kinect-shaped): after the network and 30 Stein iterations the
    particle sets are as close to a 300-iteration reference as plain Stein
    ICP after 100 or more iterations, and far closer than plain Stein ICP
    after 30 (the same schedules; only the initial particles differ)."""
    import os
    from paper_2106_03287_amd import train_proposal as TP
    path = os.path.join(os.path.dirname(PR.__file__), "weights", "proposal_k100_p4096.npy")
    cfg = PR.stein_icp_proposal_default_config(num_particles=100, points=4096, max_batch=32)
    m = PR.Proposal(cfg, np.load(path, allow_pickle=False))
    ds, X, _ = TP.build_dataset(m, "test", 8, None, label=False)
    res = TP.evaluate(m, ds, X)
    for kind in ("cuboid", "kinect"):
        r = res[kind]
        prop30 = r["proposal_mmd"][30]["mean"]
        print(kind, "proposal+30", prop30, "plain", {t: v["mean"] for t, v in r["plain_mmd"].items()})
        assert r["fallbacks"] == 0
        assert prop30 < r["plain_mmd"][100]["mean"]
        assert prop30 < r["plain_mmd"][30]["mean"] / 3
    m.close()


@pytest.mark.parametrize("P,B", [(64, 2), (4096, 1)])
def test_fused_per_point_kernel_matches_the_gemm_chain(P, B):
    """With P a multiple of 64 the three per-point layers and the max-pool
    run in one kernel; its result equals the same layers done with the GEMM
    primitive and a max over points, up to the FP32 reassociation the head's
    split-K reduction may apply (a different rounding point anywhere in the
    per-point layers would show as BF16-sized, ~1e-3, differences)."""
    K = 16
    params = _params(K, 21)
    clouds = _clouds(B, P, 22)
    m = _model(K, P, B, params)
    y, _ = m.forward(_cuda(clouds))
    torch.cuda.synchronize()
    blocks = {k: _cuda(v.astype(np.float32)) for k, v in PO.unpack(params, K).items()}
    X = _cuda(clouds.reshape(-1, 3))
    rows = X.shape[0]

    def layer(A, name, n, relu):
        out = torch.empty(A.shape[0], n, dtype=torch.float32, device="cuda")
        PR.stein_icp_gemm_bf16(A, blocks["W" + name].reshape(A.shape[1], n).contiguous(), out,
                               bias=blocks["b" + name], relu=relu)
        return out

    H3 = layer(layer(layer(X, "1", 64, 1), "2", 128, 1), "3", 256, 1)
    F = H3.reshape(B * 2, P, 256).amax(dim=1).reshape(B, 512).contiguous()
    Y = layer(layer(F, "4", 256, 1), "5", 6 * K, 0)
    torch.cuda.synchronize()
    got, want = y.cpu().numpy(), Y.cpu().numpy().astype(np.float64).reshape(B, K, 6)
    assert np.abs(got - want).max() <= 1e-5 * np.abs(want).max()
    assert rows == 2 * B * P
    m.close()


@pytest.mark.parametrize("M,N,K", [(256, 64, 3), (192, 128, 64), (128, 256, 128)])
def test_matrix_core_product_is_bitwise_symmetric_in_its_operands(M, N, K):
    """(x W)^T and W^T x^T from the BF16 matrix-core product have the same
    bits: the fused per-point kernel takes the transposed form and the
    backward recomputes the untransposed one at the winning points."""
    rng = np.random.default_rng(M + N + K)
    X = rng.standard_normal((M, K)).astype(np.float32)
    W = rng.standard_normal((K, N)).astype(np.float32)
    Xd, Wd = _cuda(X), _cuda(W)
    C = torch.empty(M, N, dtype=torch.float32, device="cuda")
    Ct = torch.empty(N, M, dtype=torch.float32, device="cuda")
    PR.stein_icp_gemm_bf16(Xd, Wd, C)
    PR.stein_icp_gemm_bf16(Wd, Xd, Ct, ta=1, tb=1)
    torch.cuda.synchronize()
    assert torch.equal(C, Ct.t())


def test_model_loaded_by_the_library_from_the_weight_file_equals_the_uploaded_one():
    """stein_icp_proposal_load reads the committed weight file itself; its
    forward equals that of a model given the same parameters from NumPy."""
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2106_03287_amd", "weights", "proposal_k100_p4096.npy")
    loaded = PR.Proposal.load(path)
    assert loaded.K == 100
    ref = PR.Proposal(PR.stein_icp_proposal_default_config(), np.load(path, allow_pickle=False))
    assert torch.equal(loaded.params(), ref.params())
    clouds = torch.from_numpy(np.random.default_rng(3).uniform(-0.3, 0.3, (2, 2, 4096, 3)).astype(np.float32)).cuda()
    a, _ = loaded.forward(clouds)
    b, _ = ref.forward(clouds)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    loaded.close()
    ref.close()
