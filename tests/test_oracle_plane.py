"""Pins of the oracle's point-to-plane parts against things other than
itself: scipy's KD-tree and numpy's symmetric eigensolver for the neighbours
and normals, exactly representable planes and lines, finite differences of the
point-to-plane cost, its reduction to the point-to-point gradient, the
invariances of a planar reference, and exact recovery of a rigid transform."""
import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

import synth


def _surface(seed, M=3000, noise=0.002):
    """Noisy smooth surface z = 0.3 sin(3x) cos(2y), FP32."""
    rng = np.random.default_rng(seed)
    xy = rng.uniform(-0.5, 0.5, (M, 2))
    z = 0.3 * np.sin(3 * xy[:, 0]) * np.cos(2 * xy[:, 1]) + rng.normal(0, noise, M)
    return np.column_stack([xy, z]).astype(np.float32)


def _separated(d, k):
    """Rows whose k-th and (k+1)-th neighbour distances differ clearly (FP64)."""
    return (d[:, k] - d[:, k - 1]) > 1e-5 * np.maximum(d[:, k - 1], 1e-12)


# ---------------------------------------------------------------- neighbours

@pytest.mark.parametrize("k", [1, 5, 10, 32])
def test_knn_matches_kdtree_away_from_ties(orc, k):
    ref = _surface(1, 2500)
    rng = np.random.default_rng(2)
    q = (ref[rng.choice(len(ref), 400, replace=False)] + rng.normal(0, 0.01, (400, 3))).astype(np.float32)
    idx, d2 = orc.knn_f32(q, ref, k)
    d, j = cKDTree(ref.astype(np.float64)).query(q.astype(np.float64), k + 1)
    ok = _separated(d, k)
    assert ok.mean() > 0.98
    # order within the k as well: consecutive distances distinct in these rows
    gaps = np.diff(d[:, :k], axis=1) if k > 1 else np.ones((len(q), 1))
    ok &= np.all(gaps > 1e-5 * np.maximum(d[:, :k][:, :max(k - 1, 1)], 1e-12), axis=1)
    np.testing.assert_array_equal(idx[ok], j[ok, :k])
    np.testing.assert_allclose(d2[ok], (d[ok, :k] ** 2), rtol=1e-5)


def test_knn_brute_force_python_with_exact_ties(orc):
    """Integer grid with duplicates: every distance is an exact small integer,
    so a pure-Python sort by (distance, index) is the definition."""
    rng = np.random.default_rng(3)
    ref = rng.integers(-3, 4, (150, 3)).astype(np.float32)
    q = rng.integers(-4, 5, (60, 3)).astype(np.float32)
    k = 7
    idx, d2 = orc.knn_f32(q, ref, k)
    for i in range(len(q)):
        keys = sorted((int(((q[i] - ref[j]) ** 2).sum()), j) for j in range(len(ref)))[:k]
        assert [j for _, j in keys] == list(idx[i])
        assert [float(d) for d, _ in keys] == list(d2[i])


def test_knn_fewer_references_than_k(orc):
    ref = np.array([[0, 0, 0], [1, 0, 0], [0, 2, 0]], np.float32)
    idx, d2 = orc.knn_f32(np.zeros((1, 3), np.float32), ref, 5)
    assert list(idx[0]) == [0, 1, 2, -1, -1]
    assert list(d2[0][:3]) == [0.0, 1.0, 4.0] and np.all(np.isinf(d2[0][3:]))


# ---------------------------------------------------------------- normals

def test_normals_match_numpy_pca(orc):
    k = 10
    for ref in (_surface(4, 3000), synth.make_problem("cuboid", 0).pair.ref):
        n, w = orc.normals(ref, k)
        R64 = ref.astype(np.float64)
        d, nb = cKDTree(R64).query(R64, k + 1)
        ok = _separated(d, k)
        assert ok.mean() > 0.97
        checked = 0
        for i in np.nonzero(ok)[0]:
            P = R64[nb[i, :k]]
            C = np.cov(P.T, bias=True)
            wn, V = np.linalg.eigh(C)
            tr = wn.sum()
            np.testing.assert_allclose(w[i], wn, rtol=0, atol=1e-12 * tr)
            if wn[1] - wn[0] > 1e-6 * tr:       # a well-defined normal
                assert abs(abs(n[i] @ V[:, 0]) - 1.0) < 1e-10
                checked += 1
        assert checked > 0.95 * len(ref)
        np.testing.assert_allclose(np.linalg.norm(n, axis=1), 1.0, atol=1e-14)


def test_normals_of_an_exact_plane(orc):
    """Points of z = 0.25 x + 0.5 y + 0.125 on a 1/64 grid are exact in FP32;
    every normal is +-(-0.25, -0.5, 1) / |.|."""
    g = np.arange(-16, 17) / 64.0
    x, y = np.meshgrid(g, g)
    ref = np.column_stack([x.ravel(), y.ravel(), 0.25 * x.ravel() + 0.5 * y.ravel() + 0.125]).astype(np.float32)
    assert np.array_equal(ref[:, 2].astype(np.float64), 0.25 * ref[:, 0] + 0.5 * ref[:, 1] + 0.125)
    n, _ = orc.normals(ref, 10)
    true = np.array([-0.25, -0.5, 1.0]) / np.sqrt(1.3125)
    np.testing.assert_allclose(np.abs(n @ true), 1.0, atol=1e-12)


def test_normals_of_lines_and_repeated_points_are_zero(orc):
    t = np.arange(40) / 16.0
    line = np.column_stack([t, 2 * t, -t]).astype(np.float32)
    n, w = orc.normals(line, 8)
    assert np.all(n == 0.0)
    same = np.tile(np.array([[0.5, -0.25, 2.0]], np.float32), (20, 1))
    n, w = orc.normals(same, 8)
    assert np.all(n == 0.0) and np.all(w == 0.0)
    # a grid point with its six axis neighbours: isotropic, no unique plane
    star = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.float32)
    n, w = orc.normals(star, 7)
    assert np.all(n[0] == 0.0) and w[0][0] == w[0][2]
    # a plane grid keeps its normals
    g = np.arange(6) / 8.0
    x, y = np.meshgrid(g, g)
    flat = np.column_stack([x.ravel(), y.ravel(), np.zeros(x.size)]).astype(np.float32)
    n, _ = orc.normals(flat, 8)
    assert np.all(np.abs(n[:, 2]) == 1.0)


def test_normals_with_fewer_points_than_k(orc):
    ref = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], np.float32)
    n, _ = orc.normals(ref, 10)
    np.testing.assert_array_equal(np.abs(n), np.tile([0.0, 0.0, 1.0], (4, 1)))


# ---------------------------------------------------------------- cost and gradient

def _plane_problem(orc, seed=7, N=300, M=900):
    rng = np.random.default_rng(seed)
    ref = _surface(seed, M)
    src = (ref[rng.choice(M, N, replace=False)] + rng.normal(0, 0.01, (N, 3))).astype(np.float32)
    nrm, _ = orc.normals(ref, 10)
    return rng, src, ref, nrm


def _theta(rng, t=0.05, r=0.2):
    return np.concatenate([rng.uniform(-t, t, 3), rng.uniform(-r, r, 3)])


def test_plane_gradient_matches_central_differences(orc):
    rng, src, ref, nrm = _plane_problem(orc)
    batch = rng.choice(len(src), 64, replace=False).astype(np.int32)
    for _ in range(3):
        th = _theta(rng)
        q = orc.transform(th, src[batch]).astype(np.float32)
        match, _ = orc.nn_f32(q, ref)
        g = orc.plane_gradient(th, src, ref, nrm, batch, match)
        h = 1e-6
        fd = np.zeros(6)
        for d in range(6):
            tp, tm = th.copy(), th.copy()
            tp[d] += h
            tm[d] -= h
            fd[d] = (orc.plane_cost(tp, src, ref, nrm, batch, match)
                     - orc.plane_cost(tm, src, ref, nrm, batch, match)) / (2 * h)
        np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-11)


def test_plane_gradient_is_point_gradient_when_normals_follow_residuals(orc):
    """With n_j = e_i / |e_i| the projection n n^T e is e itself."""
    rng, src, ref, _ = _plane_problem(orc, seed=8)
    batch = rng.choice(len(src), 50, replace=False).astype(np.int32)
    match = rng.choice(len(ref), 50, replace=False).astype(np.int32)   # distinct references
    th = _theta(rng)
    e = orc.transform(th, src[batch]) - ref[match].astype(np.float64)
    nrm = np.zeros((len(ref), 3))
    nrm[match] = e / np.linalg.norm(e, axis=1, keepdims=True)
    gp = orc.plane_gradient(th, src, ref, nrm, batch, match)
    gi = orc.icp_gradient(th, src, ref, batch, match)
    np.testing.assert_allclose(gp, gi, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(orc.plane_cost(th, src, ref, nrm, batch, match),
                               orc.icp_cost(th, src, ref, batch, match), rtol=1e-12)


def test_planar_reference_leaves_in_plane_motion_free(orc):
    """Reference on z = 0 (normals +-e_z from the oracle's own PCA): sliding in
    x, y and turning about z change no residual, so those three gradient
    components are exactly zero; z, roll and pitch are not."""
    g = np.arange(-16, 17) / 32.0
    x, y = np.meshgrid(g, g)
    ref = np.column_stack([x.ravel(), y.ravel(), np.zeros(x.size)]).astype(np.float32)
    nrm, _ = orc.normals(ref, 10)
    assert np.all(np.abs(nrm[:, 2]) == 1.0) and np.all(nrm[:, :2] == 0.0)
    rng = np.random.default_rng(9)
    src = rng.uniform(-0.4, 0.4, (200, 3)).astype(np.float32)
    batch = np.arange(200, dtype=np.int32)
    th = np.array([0.03, -0.02, 0.05, 0.1, -0.15, 0.3])
    q = orc.transform(th, src).astype(np.float32)
    match, _ = orc.nn_f32(q, ref)
    gp = orc.plane_gradient(th, src, ref, nrm, batch, match)
    assert gp[0] == 0.0 and gp[1] == 0.0 and gp[5] == 0.0
    assert np.all(np.abs(gp[[2, 3, 4]]) > 1e-4)
    gi = orc.icp_gradient(th, src, ref, batch, match)
    assert abs(gi[0]) > 1e-4 or abs(gi[1]) > 1e-4


def _box_surface(rng, M, size=(2.0, 1.5, 1.0)):
    """Points uniform on the surface of an axis-aligned box centred at 0."""
    a, b, c = size
    areas = np.array([b * c, b * c, a * c, a * c, a * b, a * b])
    face = rng.choice(6, M, p=areas / areas.sum())
    u, v = rng.uniform(-0.5, 0.5, M), rng.uniform(-0.5, 0.5, M)
    p = np.empty((M, 3))
    for f in range(6):
        s = face == f
        ax, sign = f // 2, (1 if f % 2 else -1)
        o = [d for d in range(3) if d != ax]
        p[s, ax] = sign * size[ax] / 2
        p[s, o[0]] = u[s] * size[o[0]]
        p[s, o[1]] = v[s] * size[o[1]]
    return p


def test_plane_icp_recovers_a_rigid_transform_exactly(orc):
    """K = 1, full batch, literal step on a noise-free box whose source points
    are moved reference points: the run converges to the true pose."""
    rng = np.random.default_rng(11)
    ref = _box_surface(rng, 1500).astype(np.float32)
    nrm, _ = orc.normals(ref, 10)
    sub = rng.choice(len(ref), 300, replace=False)
    rot = Rotation.from_euler("ZYX", [0.2, -0.15, 0.1])
    t = np.array([0.1, -0.05, 0.08])
    src = rot.inv().apply(ref[sub].astype(np.float64) - t).astype(np.float32)
    yaw, pitch, roll = rot.as_euler("ZYX")
    theta_true = np.array([*t, roll, pitch, yaw])
    N = len(src)
    cfg = orc.make_config(1, N, N, len(ref), optimizer=orc.SGD, lr=1.0 / N, metric=orc.PLANE)
    st = orc.State((theta_true + np.array([0.02, -0.015, 0.01, 0.02, -0.015, 0.02]))[None, :])
    sched = np.arange(N, dtype=np.int32)[None, :]
    orc.run(cfg, src, ref, sched, 300, st, normals=nrm)
    np.testing.assert_allclose(st.theta[0], theta_true, atol=1e-6)


def test_plane_step_is_the_composition_of_its_parts(orc):
    prob = synth.make_problem("cuboid", 4, K=8, T=3)
    src, ref = prob.pair.src, prob.pair.ref
    nrm, _ = orc.normals(ref, 10)
    cfg = orc.make_config(prob.K, prob.m, len(src), len(ref), lr=prob.lr, metric=orc.PLANE)
    st = orc.State(prob.theta0)
    batch = prob.schedule[0]
    diag = orc.step(cfg, src, ref, batch, st, normals=nrm)
    G = np.zeros((prob.K, 6))
    for k in range(prob.K):
        q = orc.transform(prob.theta0[k], src[batch]).astype(np.float32)
        mt, _ = orc.nn_f32(q, ref)
        np.testing.assert_array_equal(mt, diag["match"][k])
        g = orc.plane_gradient(prob.theta0[k], src, ref, nrm, batch, mt)
        np.testing.assert_array_equal(g, diag["gbar"][k])
        G[k] = -len(src) * g
    phi, _ = orc.svgd_phi(cfg, prob.theta0, G)
    np.testing.assert_array_equal(phi, diag["phi"])
    with pytest.raises(ValueError):
        orc.step(cfg, src, ref, batch, orc.State(prob.theta0))
