"""Pins of the FP64 oracle against things other than itself: scipy's rotations
and KD-tree, finite differences, closed forms of the median-heuristic kernel,
torch's Adam, the Kabsch least-squares solution, and SVGD invariants."""
import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.distance import pdist
from scipy.spatial.transform import Rotation
from scipy import stats

import synth


def _rand_theta(rng, k=1, t=0.3, r=1.0):
    return np.concatenate([rng.uniform(-t, t, (k, 3)), rng.uniform(-r, r, (k, 3))], axis=1)


# ---------------------------------------------------------------- rotation

def test_rotation_matches_scipy_zyx(orc):
    rng = np.random.default_rng(1)
    for th in _rand_theta(rng, 20, r=3.0):
        R, _ = orc.rotation(th)
        ref = Rotation.from_euler("ZYX", [th[5], th[4], th[3]]).as_matrix()
        np.testing.assert_allclose(R, ref, atol=2e-15)


def test_rotation_derivatives_central_differences(orc):
    rng = np.random.default_rng(2)
    h = 1e-6
    for th in _rand_theta(rng, 10, r=3.0):
        _, dR = orc.rotation(th)
        for d in range(3):
            tp, tm = th.copy(), th.copy()
            tp[3 + d] += h
            tm[3 + d] -= h
            fd = (orc.rotation(tp)[0] - orc.rotation(tm)[0]) / (2 * h)
            np.testing.assert_allclose(dR[d], fd, atol=1e-9)


def test_transform_matches_scipy_apply(orc):
    rng = np.random.default_rng(3)
    th = _rand_theta(rng)[0]
    s = rng.uniform(-2, 2, (50, 3)).astype(np.float32)
    q = orc.transform(th, s)
    ref = Rotation.from_euler("ZYX", [th[5], th[4], th[3]]).apply(s.astype(np.float64)) + th[:3]
    np.testing.assert_allclose(q, ref, atol=1e-14)


# ---------------------------------------------------------------- nearest neighbour

def test_dist2_f32_exact_on_integers_and_fp32_bound(orc):
    assert orc.dist2_f32([1, 2, 3], [0, 0, 0]) == 14.0
    assert orc.dist2_f32([0.5, -0.25, 2.0], [0.5, -0.25, 2.0]) == 0.0
    rng = np.random.default_rng(4)
    q = rng.uniform(-1, 1, (200, 3)).astype(np.float32)
    r = rng.uniform(-1, 1, (200, 3)).astype(np.float32)
    for a, b in zip(q, r):
        exact = float(np.sum((a.astype(np.float64) - b.astype(np.float64)) ** 2))
        assert abs(orc.dist2_f32(a, b) - exact) <= 4 * 2.0 ** -24 * exact + 1e-45


def test_nn_matches_kdtree_away_from_ties(orc):
    rng = np.random.default_rng(5)
    ref = rng.uniform(-1, 1, (3000, 3)).astype(np.float32)
    q = rng.uniform(-1.1, 1.1, (2000, 3)).astype(np.float32)
    idx, d2 = orc.nn_f32(q, ref)
    dist, kd = cKDTree(ref.astype(np.float64)).query(q.astype(np.float64), k=2)
    clear = dist[:, 1] ** 2 > dist[:, 0] ** 2 * (1 + 1e-5)
    assert clear.mean() > 0.99
    np.testing.assert_array_equal(idx[clear], kd[clear, 0])
    np.testing.assert_allclose(d2, dist[:, 0] ** 2, rtol=1e-6, atol=1e-12)


def test_nn_ties_go_to_lowest_index(orc):
    ref = np.array([[1, 0, 0], [0, 0, 0], [0, 0, 0], [-1, 0, 0], [0, 0, 0]], np.float32)
    idx, d2 = orc.nn_f32(np.array([[0, 0, 0]], np.float32), ref)
    assert idx[0] == 1 and d2[0] == 0.0
    # equidistant from indices 0 and 3
    idx, _ = orc.nn_f32(np.array([[0, 0.5, 0]], np.float32), ref[[0, 3]])
    assert idx[0] == 0


def test_nn_brute_force_python_tiny(orc):
    rng = np.random.default_rng(6)
    ref = rng.integers(-3, 4, (40, 3)).astype(np.float32)   # many exact ties
    q = rng.integers(-3, 4, (60, 3)).astype(np.float32)
    idx, _ = orc.nn_f32(q, ref)
    for i in range(len(q)):
        best, bi = None, None
        for j in range(len(ref)):
            d = int(np.sum((q[i].astype(int) - ref[j].astype(int)) ** 2))
            if best is None or d < best:
                best, bi = d, j
        assert idx[i] == bi


# ---------------------------------------------------------------- gradient

def _small_problem(seed=7, N=300, M=800):
    rng = np.random.default_rng(seed)
    ref = rng.uniform(-0.3, 0.3, (M, 3)).astype(np.float32)
    src = rng.uniform(-0.3, 0.3, (N, 3)).astype(np.float32)
    return rng, src, ref


def test_gradient_matches_central_differences_frozen_matches(orc):
    rng, src, ref = _small_problem()
    batch = rng.choice(len(src), 64, replace=False).astype(np.int32)
    th = _rand_theta(rng)[0]
    q = orc.transform(th, src[batch]).astype(np.float32)
    match, _ = orc.nn_f32(q, ref)
    g = orc.icp_gradient(th, src, ref, batch, match)
    h = 1e-6
    fd = np.zeros(6)
    for d in range(6):
        tp, tm = th.copy(), th.copy()
        tp[d] += h
        tm[d] -= h
        fd[d] = (orc.icp_cost(tp, src, ref, batch, match) - orc.icp_cost(tm, src, ref, batch, match)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-7, atol=1e-10)


def test_gradient_equals_rematched_differences_away_from_ties(orc):
    """Danskin: with the matches recomputed at every evaluation, the cost has
    the same derivative where no match changes."""
    rng, src, ref = _small_problem(8)
    batch = rng.choice(len(src), 32, replace=False).astype(np.int32)
    th = _rand_theta(rng)[0]

    def cost_rematched(t):
        q = orc.transform(t, src[batch]).astype(np.float32)
        mt, _ = orc.nn_f32(q, ref)
        return orc.icp_cost(t, src, ref, batch, mt), mt

    _, match = cost_rematched(th)
    g = orc.icp_gradient(th, src, ref, batch, match)
    h = 1e-7
    for d in range(6):
        tp, tm = th.copy(), th.copy()
        tp[d] += h
        tm[d] -= h
        cp, mp = cost_rematched(tp)
        cm, mm = cost_rematched(tm)
        if np.array_equal(mp, match) and np.array_equal(mm, match):
            assert abs((cp - cm) / (2 * h) - g[d]) <= 1e-6 * max(1.0, abs(g[d]))


def test_identity_gives_zero_cost_and_gradient(orc):
    pair = synth.cuboid_pair(11)
    S = pair.ref.copy()
    batch = np.arange(len(S), dtype=np.int32)
    th = np.zeros(6)
    q = orc.transform(th, S[batch]).astype(np.float32)
    match, d2 = orc.nn_f32(q, S)
    assert np.all(d2 == 0.0)
    assert orc.icp_cost(th, S, S, batch, match) == 0.0
    assert np.all(orc.icp_gradient(th, S, S, batch, match) == 0.0)
    # and through a whole iteration with K = 1 (kernel 1, no repulsion)
    cfg = orc.make_config(1, len(S), len(S), len(S), optimizer=orc.SGD, lr=0.1)
    st = orc.State(th[None, :])
    diag = orc.step(cfg, S, S, batch, st)
    assert np.all(diag["gbar"] == 0.0) and np.all(diag["phi"] == 0.0)
    assert np.all(st.theta == 0.0)


# ---------------------------------------------------------------- SVGD direction

def _kernel_matrix(orc, cfg, theta):
    """Read k(theta_l, theta_k) off the oracle through the linearity of phi in G."""
    K = len(theta)
    base, h = orc.svgd_phi(cfg, theta, np.zeros((K, 6)))
    kt = np.zeros((K, K))
    kr = np.zeros((K, K))
    for l in range(K):
        G = np.zeros((K, 6))
        G[l, 0] = 1.0
        G[l, 3] = 1.0
        phi, _ = orc.svgd_phi(cfg, theta, G)
        kt[l] = (phi[:, 0] - base[:, 0]) * K
        kr[l] = (phi[:, 3] - base[:, 3]) * K
    return kt, kr, h, base


def _wrapped_dists(theta):
    K = len(theta)
    Dr = np.zeros((K, K))
    for k in range(K):
        d = np.angle(np.exp(1j * (theta[k, 3:] - theta[:, 3:])))
        Dr[k] = np.sqrt(np.sum(d ** 2, axis=1))
    return Dr


def test_svgd_single_particle_is_plain_gradient(orc):
    rng = np.random.default_rng(12)
    th = _rand_theta(rng)
    G = rng.normal(size=(1, 6))
    cfg = orc.make_config(1, 1, 1, 1)
    phi, h = orc.svgd_phi(cfg, th, G)
    np.testing.assert_array_equal(phi, G)
    assert list(h) == [1.0, 1.0]


def test_svgd_two_particles_kernel_is_one_half(orc):
    rng = np.random.default_rng(13)
    th = _rand_theta(rng, 2)
    cfg = orc.make_config(2, 1, 1, 1)
    kt, kr, _, _ = _kernel_matrix(orc, cfg, th)
    np.testing.assert_allclose(kt, [[1, 0.5], [0.5, 1]], rtol=1e-14)
    np.testing.assert_allclose(kr, [[1, 0.5], [0.5, 1]], rtol=1e-14)


@pytest.mark.parametrize("K", [3, 7, 10])
def test_svgd_median_pair_kernel_is_one_over_K(orc, K):
    """Odd pair count: the median-distance pair has kernel exp(-ln K) = 1/K."""
    rng = np.random.default_rng(14 + K)
    th = _rand_theta(rng, K, r=2.5)
    cfg = orc.make_config(K, 1, 1, 1)
    kt, kr, h, _ = _kernel_matrix(orc, cfg, th)
    Dt = pdist(th[:, :3])
    med_t = np.median(Dt)
    iu = np.triu_indices(K, 1)
    sel = np.argmin(np.abs(Dt - med_t))
    assert kt[iu][sel] == pytest.approx(1.0 / K, rel=1e-12)
    assert h[0] == pytest.approx(med_t ** 2 / np.log(K), rel=1e-14)
    Dr = _wrapped_dists(th)[iu]
    med_r = np.median(Dr)
    sel = np.argmin(np.abs(Dr - med_r))
    assert kr[iu][sel] == pytest.approx(1.0 / K, rel=1e-12)
    assert h[1] == pytest.approx(med_r ** 2 / np.log(K), rel=1e-13)


def test_svgd_even_pair_count_median_is_mean_of_middle_pair(orc):
    K = 4   # 6 pairs
    rng = np.random.default_rng(20)
    th = _rand_theta(rng, K)
    cfg = orc.make_config(K, 1, 1, 1)
    _, h = orc.svgd_phi(cfg, th, np.zeros((K, 6)))
    assert h[0] == pytest.approx(np.median(pdist(th[:, :3])) ** 2 / np.log(K), rel=1e-14)


def test_svgd_repulsion_sums_to_zero_and_pushes_apart(orc):
    rng = np.random.default_rng(21)
    K = 9
    th = _rand_theta(rng, K, r=1.0)
    cfg = orc.make_config(K, 1, 1, 1)
    phi, _ = orc.svgd_phi(cfg, th, np.zeros((K, 6)))
    np.testing.assert_allclose(phi.sum(axis=0), 0.0, atol=1e-12)
    two = _rand_theta(rng, 2, r=0.5)
    phi2, _ = orc.svgd_phi(orc.make_config(2, 1, 1, 1), two, np.zeros((2, 6)))
    assert np.dot(two[0, :3] - two[1, :3], phi2[0, :3]) > 0
    assert np.dot(two[0, 3:] - two[1, 3:], phi2[0, 3:]) > 0


def test_svgd_two_particle_repulsion_closed_form_with_wrapping(orc):
    """K = 2, G = 0: h = |d|^2 / ln 2 and k = 1/2, so
    phi_1 = (1/2) (2/h) d (1/2) = d ln2 / (2 |d|^2), with d the (wrapped)
    difference theta_1 - theta_2. Angles straddle +-pi so the wrap matters."""
    cfg = orc.make_config(2, 1, 1, 1)
    th = np.array([[0.1, -0.2, 0.3, 3.0, -2.9, 0.4],
                   [-0.2, 0.1, 0.2, -3.0, 3.1, -0.3]])
    phi, _ = orc.svgd_phi(cfg, th, np.zeros((2, 6)))
    dt = th[0, :3] - th[1, :3]
    dr = np.angle(np.exp(1j * (th[0, 3:] - th[1, 3:])))
    np.testing.assert_allclose(phi[0, :3], dt * np.log(2) / (2 * dt @ dt), rtol=1e-13)
    np.testing.assert_allclose(phi[0, 3:], dr * np.log(2) / (2 * dr @ dr), rtol=1e-13)
    np.testing.assert_allclose(phi[1], -phi[0], rtol=1e-13)


def test_svgd_permutation_equivariance(orc):
    rng = np.random.default_rng(22)
    K = 12
    th = _rand_theta(rng, K)
    G = rng.normal(size=(K, 6))
    cfg = orc.make_config(K, 1, 1, 1)
    phi, h = orc.svgd_phi(cfg, th, G)
    perm = rng.permutation(K)
    phi_p, h_p = orc.svgd_phi(cfg, th[perm], G[perm])
    np.testing.assert_allclose(phi_p, phi[perm], rtol=1e-12, atol=1e-14)
    np.testing.assert_array_equal(h, h_p)


def test_svgd_tiny_fixed_bandwidth_decouples_particles(orc):
    rng = np.random.default_rng(23)
    K = 6
    th = _rand_theta(rng, K)
    G = rng.normal(size=(K, 6))
    cfg = orc.make_config(K, 1, 1, 1, bandwidth=orc.BW_FIXED, h_fixed=(1e-6, 1e-6))
    phi, _ = orc.svgd_phi(cfg, th, G)
    np.testing.assert_allclose(phi, G / K, rtol=1e-15)


def test_median_matches_numpy(orc):
    rng = np.random.default_rng(24)
    for n in (1, 2, 5, 6, 101, 1000):
        v = rng.normal(size=n)
        assert orc.median(v) == np.median(v)


# ---------------------------------------------------------------- priors

def test_prior_gradients_match_scipy_log_densities(orc):
    mu = [0.1, -0.2, 0.3, 0.4, -0.5, 1.0]
    var = [0.04, 0.09, 0.25]
    kappa = [2.0, 5.0, 0.5]
    cfg = orc.make_config(1, 1, 1, 1, prior={"mu": mu, "var_trans": var, "kappa_rot": kappa})
    th = np.array([0.3, 0.1, -0.2, 1.2, 0.3, -2.0])
    g = orc.prior_grad(cfg, th)
    h = 1e-6
    for d in range(6):
        def lp(x):
            if d < 3:
                return stats.norm.logpdf(x, mu[d], np.sqrt(var[d]))
            return stats.vonmises.logpdf(x, kappa[d - 3], loc=mu[d])
        fd = (lp(th[d] + h) - lp(th[d] - h)) / (2 * h)
        assert g[d] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    assert np.all(orc.prior_grad(orc.make_config(1, 1, 1, 1), th) == 0.0)


# ---------------------------------------------------------------- optimiser

def test_adam_matches_torch_adam(orc):
    import torch
    rng = np.random.default_rng(25)
    K = 5
    cfg = orc.make_config(K, 1, 1, 1, lr=0.03)
    th = _rand_theta(rng, K)
    mom = np.zeros_like(th)
    vel = np.zeros_like(th)
    p = torch.tensor(th.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.03, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 21):
        phi = rng.normal(size=(K, 6)) * 10 ** rng.uniform(-3, 3)
        th, mom, vel = orc.update(cfg, t, th, mom, vel, phi)
        opt.zero_grad()
        p.grad = torch.tensor(-phi, dtype=torch.float64)
        opt.step()
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_sgd_mode_is_the_literal_step(orc):
    rng = np.random.default_rng(26)
    cfg = orc.make_config(3, 1, 1, 1, lr=0.2, optimizer=orc.SGD)
    th = _rand_theta(rng, 3)
    phi = rng.normal(size=(3, 6))
    th2, _, _ = orc.update(cfg, 1, th, np.zeros_like(th), np.zeros_like(th), phi)
    np.testing.assert_array_equal(th2, th + 0.2 * phi)


# ---------------------------------------------------------------- whole iteration

def _kabsch(src, ref):
    """Least-squares rigid fit ref ~ R src + t with known correspondences."""
    a = src.astype(np.float64)
    b = ref.astype(np.float64)
    ca, cb = a.mean(0), b.mean(0)
    H = (a - ca).T @ (b - cb)
    U, _, Vt = np.linalg.svd(H)
    D = np.diag([1, 1, np.sign(np.linalg.det(Vt.T @ U.T))])
    R = Vt.T @ D @ U.T
    return R, cb - R @ ca


def test_exact_recovery_of_a_rigid_transform(orc):
    """K = 1, full batch, literal step: converges to the least-squares pose."""
    rng = np.random.default_rng(27)
    p = rng.uniform(-1, 1, (60, 3))
    rot = Rotation.from_euler("ZYX", [0.3, -0.2, 0.25])
    t = np.array([0.2, -0.1, 0.3])
    ref = p.astype(np.float32)
    src = rot.inv().apply(p - t).astype(np.float32)      # ref = rot src + t
    R_ls, t_ls = _kabsch(src, ref)
    yaw, pitch, roll = Rotation.from_matrix(R_ls).as_euler("ZYX")
    theta_ls = np.array([*t_ls, roll, pitch, yaw])
    N = len(src)
    cfg = orc.make_config(1, N, N, N, optimizer=orc.SGD, lr=0.5 / N)
    st = orc.State((theta_ls + np.array([0.02, -0.02, 0.01, 0.02, -0.01, 0.02]))[None, :])
    sched = np.arange(N, dtype=np.int32)[None, :]
    orc.run(cfg, src, ref, sched, 400, st)
    np.testing.assert_allclose(st.theta[0], theta_ls, atol=1e-9)
    np.testing.assert_allclose(theta_ls, [*t, 0.25, -0.2, 0.3], atol=1e-6)


def test_single_particle_adam_equals_independent_sgd_icp(orc):
    """K = 1: phi = -N gbar, so the run is SGD-ICP with Adam. The reference loop
    below uses scipy's KD-tree for matching, torch autograd for the gradient of
    the minibatch cost, and torch's Adam."""
    import torch
    prob = synth.make_problem("cuboid", 3, K=1, T=40)
    src, ref = prob.pair.src, prob.pair.ref
    N = len(src)
    cfg = orc.make_config(1, prob.m, N, len(ref), lr=prob.lr)
    st = orc.State(prob.theta0)
    orc.run(cfg, src, ref, prob.schedule, prob.T, st)

    tree = cKDTree(ref.astype(np.float64))
    p = torch.tensor(prob.theta0[0].copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=prob.lr, betas=(0.9, 0.999), eps=1e-8)
    S = torch.tensor(src.astype(np.float64))
    Rf = torch.tensor(ref.astype(np.float64))

    def rot(th):
        r, pi, y = th[3], th[4], th[5]
        one, zero = torch.ones((), dtype=th.dtype), torch.zeros((), dtype=th.dtype)
        Rx = torch.stack([torch.stack([one, zero, zero]),
                          torch.stack([zero, torch.cos(r), -torch.sin(r)]),
                          torch.stack([zero, torch.sin(r), torch.cos(r)])])
        Ry = torch.stack([torch.stack([torch.cos(pi), zero, torch.sin(pi)]),
                          torch.stack([zero, one, zero]),
                          torch.stack([-torch.sin(pi), zero, torch.cos(pi)])])
        Rz = torch.stack([torch.stack([torch.cos(y), -torch.sin(y), zero]),
                          torch.stack([torch.sin(y), torch.cos(y), zero]),
                          torch.stack([zero, zero, one])])
        return Rz @ Ry @ Rx

    for t in range(prob.T):
        b = torch.tensor(prob.schedule[t].astype(np.int64))
        with torch.no_grad():
            q = S[b] @ rot(p).T + p[:3]
        _, j = tree.query(q.numpy().astype(np.float32).astype(np.float64))
        opt.zero_grad()
        e = S[b] @ rot(p).T + p[:3] - Rf[torch.tensor(j)]
        cost = 0.5 * (e ** 2).sum() / prob.m
        cost.backward()
        p.grad *= N          # descent direction -phi = N * gbar for one particle
        opt.step()
    np.testing.assert_allclose(st.theta[0], p.detach().numpy(), rtol=1e-9, atol=1e-11)


def test_step_is_the_composition_of_its_parts(orc):
    prob = synth.make_problem("cuboid", 4, K=8, T=3)
    src, ref = prob.pair.src, prob.pair.ref
    cfg = orc.make_config(prob.K, prob.m, len(src), len(ref), lr=prob.lr)
    st = orc.State(prob.theta0)
    batch = prob.schedule[0]
    diag = orc.step(cfg, src, ref, batch, st)
    G = np.zeros((prob.K, 6))
    for k in range(prob.K):
        q = orc.transform(prob.theta0[k], src[batch]).astype(np.float32)
        mt, _ = orc.nn_f32(q, ref)
        np.testing.assert_array_equal(mt, diag["match"][k])
        g = orc.icp_gradient(prob.theta0[k], src, ref, batch, mt)
        np.testing.assert_array_equal(g, diag["gbar"][k])
        G[k] = -len(src) * g
    phi, h = orc.svgd_phi(cfg, prob.theta0, G)
    np.testing.assert_array_equal(phi, diag["phi"])
    th, _, _ = orc.update(cfg, 1, prob.theta0, np.zeros((prob.K, 6)), np.zeros((prob.K, 6)), phi)
    np.testing.assert_array_equal(th, st.theta)


def test_translation_posterior_spread_matches_gaussian(orc):
    """All N source points at the origin and one reference point r: the
    translation posterior is N(r, I/N) (unit-variance residual likelihood of
    the mean minibatch gradient scaled by N). SVGD with the median heuristic
    should reproduce the spread roughly; a wrong N scaling (m instead of N)
    or a missing/doubled repulsion misses it by far."""
    N, m, K = 256, 16, 100
    src = np.zeros((N, 3), np.float32)
    ref = np.array([[0.3, -0.2, 0.1]], np.float32)
    rng = np.random.default_rng(28)
    theta0 = np.concatenate([rng.uniform(0.0, 0.6, (K, 3)) + ref[0] - 0.3,
                             rng.uniform(-0.5, 0.5, (K, 3))], axis=1)
    sched = np.stack([rng.choice(N, m, replace=False) for _ in range(8)]).astype(np.int32)
    cfg = orc.make_config(K, m, N, 1, lr=0.01)
    st = orc.State(theta0)
    orc.run(cfg, src, ref, sched, 1500, st)
    std = st.theta[:, :3].std(axis=0)
    mean = st.theta[:, :3].mean(axis=0)
    np.testing.assert_allclose(mean, ref[0], atol=0.02)
    assert np.all(std > 0.7 / np.sqrt(N)) and np.all(std < 1.3 / np.sqrt(N)), std
