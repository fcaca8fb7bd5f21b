"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded clouds, initial particles and minibatch schedules.

Bars: nearest-neighbour indices and FP32 distances bit-exact (both sides
decide the argmin in FP32 on the same FP32 queries); particle poses within
1e-4 m / 1e-4 rad after the fixed iteration count (the stated tolerance);
per-iteration quantities (gbar, phi, h, theta) also within tighter relative
bounds derived from FP64 summation-order differences, which is what the
implementations differ by once the matches agree."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2106_03287_amd import stein_icp as S

pytestmark = pytest.mark.gpu

POSE_TOL = 1e-4       # m / rad, after the fixed iteration count
STEP_RTOL = 1e-9      # one iteration from identical state


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def wrapped(d):
    d = np.array(d, dtype=np.float64, copy=True)
    d[..., 3:] = np.angle(np.exp(1j * d[..., 3:]))
    return d


def both_configs(prob, opts=None):
    o = dict(opts or {})
    g = dict(num_particles=prob.K, batch_size=prob.m, schedule_rows=prob.schedule.shape[0],
              lr=prob.lr)
    okw = dict(lr=prob.lr)
    if o.get("sgd"):
        g["optimizer"] = S.OPT_SGD
        okw["optimizer"] = oracle.SGD
    if "h_fixed" in o:
        g.update(bandwidth_mode=S.BW_FIXED, fixed_h_trans=o["h_fixed"][0], fixed_h_rot=o["h_fixed"][1])
        okw.update(bandwidth=oracle.BW_FIXED, h_fixed=tuple(o["h_fixed"]))
    if "prior" in o:
        pr = o["prior"]
        g.update(prior_mode=S.PRIOR_GAUSS_VONMISES, prior_mu=pr["mu"], prior_var_trans=pr["var_trans"],
                 prior_kappa_rot=pr["kappa_rot"])
        okw["prior"] = pr
    for k in ("use_graph", "autotune"):
        if k in o:
            g[k] = o[k]
    gcfg = S.stein_icp_default_config(**g)
    ocfg = oracle.make_config(prob.K, prob.m, len(prob.pair.src), len(prob.pair.ref), **okw)
    return gcfg, ocfg


def gpu_solver(prob, opts=None):
    gcfg, _ = both_configs(prob, opts)
    return S.SteinICP(gcfg, dev(prob.pair.src), dev(prob.pair.ref), dev(prob.theta0),
                      dev(prob.schedule))


def gpu_run(prob, T, opts=None):
    sol = gpu_solver(prob, opts)
    sol.step(T)
    out = sol.particles().cpu().numpy()[0]
    sol.close()
    return out


def oracle_run(prob, T, opts=None):
    _, ocfg = both_configs(prob, opts)
    st = oracle.State(prob.theta0)
    oracle.run(ocfg, prob.pair.src, prob.pair.ref, prob.schedule, T, st)
    return st.theta


def assert_poses_close(gpu, ref, tol=POSE_TOL):
    d = np.abs(wrapped(gpu - ref))
    print(f"max |dtheta| trans {d[:, :3].max():.3e} rot {d[:, 3:].max():.3e}", flush=True)
    assert d.max() <= tol


# ------------------------------------------------------------------ NN

@pytest.mark.parametrize("nq,M", [(1, 1), (100, 17), (4097, 2000), (777, 20011), (0, 5)])
def test_nn_bitwise_against_oracle(nq, M):
    rng = np.random.default_rng(nq * 31 + M)
    ref = rng.uniform(-1, 1, (M, 3)).astype(np.float32)
    q = rng.uniform(-1.2, 1.2, (nq, 3)).astype(np.float32)
    if nq > 10 and M > 10:
        q[:5] = ref[rng.integers(0, M, 5)]           # exact hits (distance 0)
    print(f"nn nq={nq} M={M}", flush=True)
    idx, d2 = S.stein_icp_nn(dev(q).reshape(-1, 3), dev(ref))
    if nq == 0:
        return
    oi, od = oracle.nn_f32(q, ref)
    np.testing.assert_array_equal(idx.cpu().numpy(), oi)
    np.testing.assert_array_equal(d2.cpu().numpy(), od)


def test_nn_exact_ties_take_lowest_index():
    rng = np.random.default_rng(3)
    ref = rng.integers(-4, 5, (3001, 3)).astype(np.float32)     # many duplicates
    q = rng.integers(-5, 6, (2500, 3)).astype(np.float32)
    idx, d2 = S.stein_icp_nn(dev(q), dev(ref))
    oi, od = oracle.nn_f32(q, ref)
    np.testing.assert_array_equal(idx.cpu().numpy(), oi)
    np.testing.assert_array_equal(d2.cpu().numpy(), od)


def test_nn_full_lidar_reference_sampled_queries():
    prob = synth.make_problem("lidar", 0, K=1, T=1)
    rng = np.random.default_rng(4)
    sel = rng.choice(len(prob.pair.src), 3000, replace=False)
    q = oracle.transform(prob.pair.theta_true, prob.pair.src[sel]).astype(np.float32)
    idx, d2 = S.stein_icp_nn(dev(q), dev(prob.pair.ref))
    oi, od = oracle.nn_f32(q, prob.pair.ref)
    np.testing.assert_array_equal(idx.cpu().numpy(), oi)
    np.testing.assert_array_equal(d2.cpu().numpy(), od)


# ------------------------------------------------------------------ one iteration

def _one_step_compare(prob, opts=None):
    sol = gpu_solver(prob, opts)
    sol.step(1)
    diag = {k: v.cpu().numpy()[0] for k, v in sol.diagnostics().items()}
    th_gpu = sol.particles().cpu().numpy()[0]
    _, _, _, t = sol.get_state()
    sol.close()
    _, ocfg = both_configs(prob, opts)
    st = oracle.State(prob.theta0)
    od = oracle.step(ocfg, prob.pair.src, prob.pair.ref, prob.schedule[0], st)
    assert t == 1
    np.testing.assert_array_equal(diag["match"], od["match"])
    np.testing.assert_allclose(diag["gbar"], od["gbar"], rtol=STEP_RTOL, atol=1e-13)
    np.testing.assert_allclose(diag["h"], od["h"], rtol=1e-12)
    scale = np.abs(od["phi"]).max()
    np.testing.assert_allclose(diag["phi"], od["phi"], rtol=STEP_RTOL, atol=1e-12 * scale)
    np.testing.assert_allclose(th_gpu, st.theta, rtol=0, atol=1e-11)


def test_one_iteration_cuboid():
    _one_step_compare(synth.make_problem("cuboid", 0))


def test_one_iteration_kinect():
    _one_step_compare(synth.make_problem("kinect", 0, T=1))


def test_one_iteration_lidar_full_size():
    prob = synth.make_problem("lidar", 0, T=1)
    print("lidar full-size one iteration: K=300 m=1000 M=100000", flush=True)
    _one_step_compare(prob)


# ------------------------------------------------------------------ free running

def test_cuboid_50_iterations_free_running():
    prob = synth.make_problem("cuboid", 0)
    assert_poses_close(gpu_run(prob, prob.T), oracle_run(prob, prob.T))


def test_cuboid_other_seeds_free_running():
    for p in (1, 2):
        prob = synth.make_problem("cuboid", p)
        assert_poses_close(gpu_run(prob, prob.T), oracle_run(prob, prob.T))


def test_kinect_20_iterations_free_running():
    prob = synth.make_problem("kinect", 0, T=20)
    assert_poses_close(gpu_run(prob, prob.T), oracle_run(prob, prob.T))


@pytest.mark.parametrize("opts", [
    {"sgd": True},
    {"h_fixed": (0.01, 0.05)},
    {"prior": {"mu": [0.01, -0.02, 0.0, 0.1, -0.1, 0.05], "var_trans": [0.01, 0.02, 0.03],
               "kappa_rot": [2.0, 4.0, 8.0]}},
    {"use_graph": 0},
])
def test_method_options(opts):
    prob = synth.make_problem("cuboid", 5, T=10)
    if opts.get("sgd"):
        prob.lr = 1e-5
    print(f"options {opts}", flush=True)
    assert_poses_close(gpu_run(prob, prob.T, opts), oracle_run(prob, prob.T, opts))
    _one_step_compare(prob, opts)


@pytest.mark.parametrize("K,m", [(1, 100), (2, 100), (3, 1), (4, 37), (1024, 4)])
def test_particle_and_batch_extremes(K, m):
    prob = synth.make_problem("cuboid", 6, K=K, m=m, T=4)
    print(f"K={K} m={m}", flush=True)
    assert_poses_close(gpu_run(prob, prob.T), oracle_run(prob, prob.T))
    _one_step_compare(prob)


def test_ragged_reference_and_source_sizes():
    base = synth.cuboid_pair(77, n_src=133, n_ref=77)
    prob = synth.make_problem("cuboid", 7, K=9, m=133, T=6, pair=base)
    assert_poses_close(gpu_run(prob, prob.T), oracle_run(prob, prob.T))
    _one_step_compare(prob)


def test_single_reference_point():
    base = synth.cuboid_pair(78, n_src=64, n_ref=1)
    prob = synth.make_problem("cuboid", 8, K=5, m=16, T=5, pair=base)
    assert_poses_close(gpu_run(prob, prob.T), oracle_run(prob, prob.T))


# ------------------------------------------------------------------ engine behaviour

def test_graph_direct_and_autotuned_runs_are_bitwise_identical():
    prob = synth.make_problem("kinect", 1, T=8)
    a = gpu_run(prob, prob.T, {"use_graph": 1})
    b = gpu_run(prob, prob.T, {"use_graph": 0})
    c = gpu_run(prob, prob.T, {"autotune": 1})
    d = gpu_run(prob, prob.T, {"use_graph": 1})
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a, c)
    np.testing.assert_array_equal(a, d)


def test_state_round_trip_continues_bitwise():
    prob = synth.make_problem("cuboid", 9, T=12)
    full = gpu_run(prob, 12)
    sol = gpu_solver(prob)
    sol.step(5)
    th, mo, ve, t = sol.get_state()
    sol.close()
    sol2 = gpu_solver(prob)
    sol2.set_state(th, mo, ve, t)
    sol2.step(7)
    np.testing.assert_array_equal(sol2.particles().cpu().numpy()[0], full)
    sol2.step(0)
    np.testing.assert_array_equal(sol2.particles().cpu().numpy()[0], full)
    sol2.close()


def test_batched_context_matches_single_contexts_and_oracle():
    probs = [synth.make_problem("cuboid", 10 + i, K=16, m=40, T=6,
                                pair=synth.cuboid_pair(900 + i, n_src=n, n_ref=M))
             for i, (n, M) in enumerate([(300, 1000), (500, 2003), (64, 77)])]
    gcfg, _ = both_configs(probs[0])
    batch = S.SteinICP.batch(gcfg, [dev(p.pair.src) for p in probs], [dev(p.pair.ref) for p in probs],
                             dev(np.stack([p.theta0 for p in probs])),
                             [dev(p.schedule) for p in probs])
    batch.step(6)
    got = batch.particles().cpu().numpy()
    batch.close()
    for i, p in enumerate(probs):
        np.testing.assert_array_equal(got[i], gpu_run(p, 6))
        assert_poses_close(got[i], oracle_run(p, 6))


def test_fp32_particle_input_and_output():
    """FP32 K x 6 particles in (widened exactly, a fresh start) and out
    (rounded to nearest): a solve started from FP32 particles equals one
    started from the same values in FP64, and the FP32 output is the FP64
    state rounded once; non-finite input is refused with the state kept."""
    prob = synth.make_problem("cuboid", 15, K=24, T=6)
    th32 = prob.theta0.astype(np.float32)
    a = gpu_solver(prob)
    a.step(3)
    a.set_particles_f32(dev(th32))
    a.step(prob.T)
    b = gpu_solver(prob)
    b.set_state(dev(th32.astype(np.float64)))
    b.step(prob.T)
    np.testing.assert_array_equal(a.particles().cpu().numpy(), b.particles().cpu().numpy())
    assert a.get_state()[3] == prob.T
    f = a.particles_f32().cpu().numpy()
    np.testing.assert_array_equal(f, a.particles().cpu().numpy().astype(np.float32))
    bad = th32.copy()
    bad[2, 4] = np.inf
    before = a.particles().clone()
    with pytest.raises(S.SteinICPError) as e:
        a.set_particles_f32(dev(bad))
    assert e.value.code == S.E_INVALID
    assert torch.equal(a.particles(), before)
    a.close()
    b.close()


def test_library_drawn_particles_and_schedule():
    prob = synth.make_problem("cuboid", 11, T=5)
    cfg = S.stein_icp_default_config(num_particles=prob.K, batch_size=prob.m, schedule_rows=5,
                                     lr=prob.lr, seed=1234)
    sol = S.SteinICP(cfg, dev(prob.pair.src), dev(prob.pair.ref))
    th0 = sol.particles().cpu().numpy()[0]
    np.testing.assert_array_equal(th0, S.stein_icp_make_init(1234, prob.K, 0.2, np.pi / 4))
    sol.step(5)
    got = sol.particles().cpu().numpy()[0]
    sol.close()
    prob.theta0 = th0
    prob.schedule = S.stein_icp_make_schedule(1234, len(prob.pair.src), prob.m, 5)
    assert_poses_close(got, oracle_run(prob, 5))


def test_invalid_device_inputs_are_rejected():
    prob = synth.make_problem("cuboid", 12, K=4, T=2)
    gcfg, _ = both_configs(prob)
    bad = prob.pair.src.copy()
    bad[3, 1] = np.nan
    with pytest.raises(S.SteinICPError) as e:
        S.SteinICP(gcfg, dev(bad), dev(prob.pair.ref), dev(prob.theta0), dev(prob.schedule))
    assert e.value.code == S.E_INVALID and "non-finite" in str(e.value)
    sch = prob.schedule.copy()
    sch[1, 2] = len(prob.pair.src)
    with pytest.raises(S.SteinICPError) as e:
        S.SteinICP(gcfg, dev(prob.pair.src), dev(prob.pair.ref), dev(prob.theta0), dev(sch))
    assert "schedule" in str(e.value)
    th = prob.theta0.copy()
    th[0, 0] = np.inf
    with pytest.raises(S.SteinICPError):
        S.SteinICP(gcfg, dev(prob.pair.src), dev(prob.pair.ref), dev(th), dev(prob.schedule))
    big = prob.pair.ref.copy()
    big[0, 0] = 3e9
    with pytest.raises(S.SteinICPError):
        S.stein_icp_nn(dev(prob.pair.src), dev(big))
    # set_state checks every input before it changes anything
    sol = S.SteinICP(gcfg, dev(prob.pair.src), dev(prob.pair.ref), dev(prob.theta0), dev(prob.schedule))
    sol.step(1)
    before = sol.get_state()
    for which in range(3):
        arrs = [dev(prob.theta0), torch.zeros(prob.K, 6, dtype=torch.float64, device="cuda"),
                torch.zeros(prob.K, 6, dtype=torch.float64, device="cuda")]
        arrs[which][1, 2] = float("nan")
        with pytest.raises(S.SteinICPError) as e:
            sol.set_state(*arrs, 0)
        assert e.value.code == S.E_INVALID and "non-finite" in str(e.value)
    after = sol.get_state()
    for a, b in zip(before[:3], after[:3]):
        assert torch.equal(a, b)
    assert before[3] == after[3] == 1
    sol.close()


# ------------------------------------------------------------------ median selection paths

def _theta_variant(prob, kind, rng):
    K = prob.K
    th = prob.theta0.copy()
    if kind == "identical":
        th[:] = th[0]
    elif kind == "two_clusters":
        th[: K // 2] = th[0]
        th[K // 2:] = th[1]
    elif kind == "near_duplicates":
        th = th[0] + rng.normal(scale=1e-9, size=th.shape)
    elif kind == "few_values":
        th = th[rng.integers(0, 5, K)]
    return th


@pytest.mark.parametrize("kind", ["identical", "two_clusters", "near_duplicates", "few_values"])
def test_bandwidth_selection_degenerate_particle_sets(kind):
    prob = synth.make_problem("cuboid", 13, K=120, T=2)
    prob.theta0 = _theta_variant(prob, kind, np.random.default_rng(5))
    print(f"selection case {kind}", flush=True)
    _one_step_compare(prob)


@pytest.mark.parametrize("K,kind", [(K, kind) for K in (120, 300)
                                    for kind in ("uniform", "identical", "two_clusters", "near_duplicates",
                                                 "few_values")] +
                         [(133, "uniform"), (134, "uniform"), (400, "uniform"), (400, "few_values")])
def test_bandwidths_beside_the_screen_search_equal_the_gradient_launch(kind, K):
    """With a screen and few particles in flight the median bandwidths run
    as extra workgroups of the nearest-neighbour launch, on its workgroup
    size (256, 512 or 1024 threads): h equals the gradient launch's (FP32
    search, 1024 threads) bit for bit and the oracle's, and the iteration's
    particles are the same, on degenerate particle sets too. K = 120 keeps
    the pair keys in LDS there; K = 300 (the LiDAR particle count) keeps
    them in global memory there, while the gradient launch keys them in
    LDS. K = 133 is the largest K whose keys fit the 48 KB there, K = 134
    the smallest that takes global memory; K = 400 has too many pairs for
    16-bit keys, and both launches select over FP64 distances in global
    memory."""
    prob = synth.make_problem("cuboid", 13, K=K, T=2)
    if kind != "uniform":
        prob.theta0 = _theta_variant(prob, kind, np.random.default_rng(5))
    print(f"fused bandwidth case {kind} K={K}", flush=True)
    _one_step_compare(prob)
    sol = gpu_solver(prob)
    sol.step(1)
    want_h = sol.diagnostics()["h"].cpu().numpy()
    want_th = sol.particles().cpu().numpy()
    sol.close()
    gcfg, _ = both_configs(prob)
    for mode in (S.NN_F16_RERANK, S.NN_BF16_RERANK):
        gcfg.nn_mode = mode
        for q, w in ((2, 4), (2, 8), (1, 16)):
            sol = S.SteinICP(gcfg, dev(prob.pair.src), dev(prob.pair.ref), dev(prob.theta0), dev(prob.schedule))
            sol.set_tiling(q, w, 64 * w)
            sol.step(1)
            np.testing.assert_array_equal(sol.diagnostics()["h"].cpu().numpy(), want_h, err_msg=f"{mode} {q},{w}")
            np.testing.assert_array_equal(sol.particles().cpu().numpy(), want_th, err_msg=f"{mode} {q},{w}")
            sol.close()


@pytest.mark.parametrize("K", [346, 347, 400])
def test_bandwidth_keyed_and_global_paths(K):
    prob = synth.make_problem("cuboid", 14, K=K, m=8, T=2)
    print(f"K={K}", flush=True)
    _one_step_compare(prob)
    assert_poses_close(gpu_run(prob, prob.T), oracle_run(prob, prob.T))


def test_every_nn_work_shape_gives_identical_results():
    prob = synth.make_problem("kinect", 2, T=3)
    ref_sol = gpu_solver(prob)
    ref_sol.step(prob.T)
    want = ref_sol.particles().cpu().numpy()
    want_match = ref_sol.diagnostics()["match"].cpu().numpy()
    ref_sol.close()
    for q in (1, 2, 4):
        for w in (4, 8, 16):
            for chunk in (w * 16, 1024, 20000):
                sol = gpu_solver(prob)
                sol.set_tiling(q, w, chunk)
                sol.step(prob.T)
                np.testing.assert_array_equal(sol.particles().cpu().numpy(), want)
                np.testing.assert_array_equal(sol.diagnostics()["match"].cpu().numpy(), want_match)
                sol.close()
    with pytest.raises(S.SteinICPError):
        sol = gpu_solver(prob)
        try:
            sol.set_tiling(3, 4, 64)
        finally:
            sol.close()


def test_batched_uneven_pairs_tuned_and_persistent():
    probs = synth.batched_problems(6, K=16, m=40, T=5, size_scale=0.2)
    gcfg, _ = both_configs(probs[0])
    srcs = [dev(p.pair.src) for p in probs]
    refs = [dev(p.pair.ref) for p in probs]
    th0 = dev(np.stack([p.theta0 for p in probs]))
    scheds = [dev(p.schedule) for p in probs]
    outs = []
    for tiling in (None, "tuned", (2, 8, 512, 2), (1, 16, 64, 1)):
        cfg = S.stein_icp_default_config(num_particles=16, batch_size=40, schedule_rows=5, lr=probs[0].lr,
                                         autotune=1 if tiling == "tuned" else 0)
        b = S.SteinICP.batch(cfg, srcs, refs, th0, scheds)
        if isinstance(tiling, tuple):
            b.set_tiling(*tiling)
        b.step(5)
        outs.append(b.particles().cpu().numpy())
        b.close()
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])
    for i, p in enumerate(probs):
        np.testing.assert_array_equal(outs[0][i], gpu_run(p, 5))
        if i < 2:
            assert_poses_close(outs[0][i], oracle_run(p, 5))


# ------------------------------------------------------------------ BF16 screen + FP32 rerank

SCREENS = [S.NN_BF16_RERANK, S.NN_F16_RERANK]


def _bf16_check(q, ref, mode=S.NN_BF16_RERANK):
    """A certified matrix-core screen (BF16 x 3 or FP16 x 2) returns the FP32
    search's answer: the same index (lowest on ties) and the same FP32
    distance, bit for bit."""
    idx, d2 = S.stein_icp_nn(dev(q), dev(ref), mode=mode)
    idx, d2 = idx.cpu().numpy(), d2.cpu().numpy()
    oi, od = oracle.nn_f32(q, ref)
    np.testing.assert_array_equal(idx, oi)
    np.testing.assert_array_equal(d2.view(np.uint32), od.astype(np.float32).view(np.uint32))


@pytest.mark.parametrize("mode", [S.NN_FP32] + SCREENS)
def test_nn_empty_single_and_ragged_sizes(mode):
    """Edge sizes of the stand-alone search: no queries (an empty answer),
    a single reference, references and queries one either side of the
    32-reference blocks and 64-query work items; answers equal the oracle's
    bit for bit. No references is refused."""
    rng = np.random.default_rng(61)
    idx, d2 = S.stein_icp_nn(dev(np.zeros((0, 3), np.float32)), dev(rng.normal(size=(5, 3)).astype(np.float32)),
                             mode=mode)
    assert idx.numel() == 0 and d2.numel() == 0
    with pytest.raises(S.SteinICPError):
        S.stein_icp_nn(dev(np.zeros((4, 3), np.float32)), dev(np.zeros((0, 3), np.float32)), mode=mode)
    for n_ref in (1, 31, 32, 33, 100):
        for nq in (1, 63, 64, 65, 129):
            ref = rng.normal(size=(n_ref, 3)).astype(np.float32)
            q = rng.normal(size=(nq, 3)).astype(np.float32)
            idx, d2 = S.stein_icp_nn(dev(q), dev(ref), mode=mode)
            oi, od = oracle.nn_f32(q, ref)
            np.testing.assert_array_equal(idx.cpu().numpy(), oi, err_msg=f"n_ref {n_ref} nq {nq}")
            np.testing.assert_array_equal(d2.cpu().numpy().view(np.uint32), od.astype(np.float32).view(np.uint32))


@pytest.mark.parametrize("mode", SCREENS)
def test_bf16_screen_kinect_queries(mode):
    prob = synth.make_problem("kinect", 0, T=1)
    rng = np.random.default_rng(8)
    sel = rng.choice(len(prob.pair.src), 4000, replace=False)
    q = np.concatenate([oracle.transform(prob.theta0[k], prob.pair.src[sel[k::8]]) for k in range(8)])
    _bf16_check(q.astype(np.float32), prob.pair.ref, mode)


@pytest.mark.parametrize("mode", SCREENS)
def test_bf16_screen_lidar_queries(mode):
    # 80 m coordinates: the error bound is wide and many queries take the
    # exact FP32 path; the answers must still be the FP32 search's
    prob = synth.make_problem("lidar", 0, K=1, T=1)
    rng = np.random.default_rng(9)
    sel = rng.choice(len(prob.pair.src), 3000, replace=False)
    q = oracle.transform(prob.theta0[0], prob.pair.src[sel]).astype(np.float32)
    _bf16_check(q, prob.pair.ref, mode)


@pytest.mark.parametrize("mode", SCREENS)
@pytest.mark.parametrize("nq,M", [(1, 1), (100, 17), (4097, 2000), (0, 5)])
def test_bf16_screen_ragged_sizes(nq, M, mode):
    rng = np.random.default_rng(nq + 7 * M)
    ref = rng.uniform(-1, 1, (M, 3)).astype(np.float32)
    q = rng.uniform(-1.2, 1.2, (nq, 3)).astype(np.float32)
    if nq == 0:
        S.stein_icp_nn(dev(q).reshape(-1, 3), dev(ref), mode=mode)
        return
    _bf16_check(q, ref, mode)


@pytest.mark.parametrize("mode", SCREENS)
def test_bf16_screen_exact_ties_go_to_the_lowest_index(mode):
    # points on an integer grid, references repeated: many exact ties,
    # within and across 16-reference blocks and screen lanes
    rng = np.random.default_rng(31)
    base = rng.integers(-6, 7, (700, 3)).astype(np.float32)
    ref = np.concatenate([base, base[::-1], base[rng.permutation(700)]])
    q = (rng.integers(-12, 13, (3000, 3)) / 2.0).astype(np.float32)
    _bf16_check(q, ref, mode)


@pytest.mark.parametrize("mode", SCREENS)
@pytest.mark.parametrize("seed", range(16))
def test_bf16_screen_randomized_scales_offsets_and_near_ties(seed, mode):
    """The certificate's error bound scales with the centred norms, so the
    screen is swept over cloud scales from 0.1 m to 100 m, centres up to
    300 m from the origin, near-duplicate references (jittered copies) and
    queries placed next to references (near-ties across blocks); indices and
    distances equal the oracle's FP32 search bit for bit."""
    rng = np.random.default_rng(900 + seed)
    scale = 10.0 ** rng.uniform(-1, 2)
    centre = rng.uniform(-1, 1, 3) * 10.0 ** rng.uniform(0, 2.5)
    M = int(rng.integers(100, 20000))
    nq = int(rng.integers(100, 4000))
    ref = centre + rng.uniform(-scale, scale, (M, 3))
    dup = rng.choice(M, M // 5, replace=False)
    ref[dup[: len(dup) // 2]] = ref[dup[len(dup) // 2:2 * (len(dup) // 2)]] + rng.normal(0, 1e-6 * scale, (len(dup) // 2, 3))
    near = rng.choice(M, nq, replace=True)
    q = ref[near] + rng.normal(0, 1e-3 * scale, (nq, 3)) * rng.uniform(0, 1, (nq, 1))
    _bf16_check(q.astype(np.float32), ref.astype(np.float32), mode)


@pytest.mark.parametrize("seed", range(8))
def test_screen_two_block_keys_randomized_scales_offsets_and_near_ties(seed):
    """The randomized clouds above (scales 0.1 to 100 m, centres up to 300 m,
    jittered duplicate references, queries next to references), searched
    with keys over two blocks (two queries per lane, a chunk of 192 blocks
    per wavefront): the first iteration's matches of both screens equal the
    FP32 search's bit for bit."""
    rng = np.random.default_rng(1900 + seed)
    scale = 10.0 ** rng.uniform(-1, 2)
    centre = rng.uniform(-1, 1, 3) * 10.0 ** rng.uniform(0, 2.5)
    M = int(rng.integers(2000, 30000))
    ref = centre + rng.uniform(-scale, scale, (M, 3))
    dup = rng.choice(M, M // 5, replace=False)
    half = len(dup) // 2
    ref[dup[:half]] = ref[dup[half:2 * half]] + rng.normal(0, 1e-6 * scale, (half, 3))
    K, m = 8, 400
    src = ref[rng.choice(M, 1000, replace=False)] - centre + rng.normal(0, 1e-3 * scale, (1000, 3))
    theta0 = np.zeros((K, 6))
    theta0[:, :3] = centre + rng.normal(0, 0.01 * scale, (K, 3))
    theta0[:, 3:] = rng.normal(0, 0.02, (K, 3))
    sched = synth.minibatch_schedule(seed, len(src), m, 1)
    src, ref = src.astype(np.float32), ref.astype(np.float32)
    matches = {}
    for mode in (S.NN_FP32, S.NN_F16_RERANK, S.NN_BF16_RERANK):
        cfg = S.stein_icp_default_config(num_particles=K, batch_size=m, schedule_rows=1, autotune=0, nn_mode=mode)
        sol = S.SteinICP(cfg, dev(src), dev(ref), dev(theta0), dev(sched))
        try:
            if mode != S.NN_FP32:
                sol.set_tiling(2, 4, 32 * 4 * TWO_BLOCK_KEY_RANGE)
            sol.step(1)
            matches[mode] = sol.diagnostics()["match"].cpu().numpy()
        finally:
            sol.close()
    for mode in (S.NN_F16_RERANK, S.NN_BF16_RERANK):
        np.testing.assert_array_equal(matches[mode], matches[S.NN_FP32], err_msg=f"mode {mode}")


def _grid_problem():
    """Cloud pair on an integer grid with repeated references: many exact
    ties between and inside the screen's 32-reference blocks."""
    rng = np.random.default_rng(41)
    base = rng.integers(-6, 7, (500, 3)).astype(np.float32)
    ref = np.concatenate([base, base[rng.permutation(500)], base[::-1]])
    src = (rng.integers(-12, 13, (800, 3)) / 2.0).astype(np.float32)
    K, m, rows = 16, 64, 2
    theta0 = np.zeros((K, 6))
    theta0[:, :3] = rng.integers(-2, 3, (K, 3)) / 4.0   # exact translations keep the ties exact
    sched = synth.minibatch_schedule(41, len(src), m, rows)
    return src, ref, theta0, sched, K, m, rows


@pytest.mark.parametrize("mode", SCREENS)
@pytest.mark.parametrize("q", [1, 2])
@pytest.mark.parametrize("w", [4, 8, 16])
def test_bf16_screen_every_block_count_per_wavefront(q, w, mode):
    """Chunks of 1 to 89 blocks of 32 references give the wavefronts of a
    workgroup 0 to 22 blocks each: every trip count of the screen's block
    loops (the two-buffer loop, and the software pipeline with two fragment
    buffers (BF16 x 3) or four (FP16 x 2), with all their tails) and ragged
    last chunks. The first iteration's matches equal the oracle's
    (lowest index on ties), on the cuboid pair and on an all-ties grid."""
    prob = synth.make_problem("cuboid", 0, T=1)
    cases = [(prob.pair.src, prob.pair.ref, prob.theta0, prob.schedule, prob.K, prob.m, prob.schedule.shape[0]),
             _grid_problem()]
    if (q, w) == (2, 16):
        # not built (two queries per lane need more registers than sixteen
        # wavefronts leave): the shape is refused, nothing is launched
        cfg = S.stein_icp_default_config(num_particles=prob.K, batch_size=prob.m, schedule_rows=1,
                                         nn_mode=mode)
        sol = S.SteinICP(cfg, dev(prob.pair.src), dev(prob.pair.ref), dev(prob.theta0), dev(prob.schedule[:1]))
        try:
            with pytest.raises(S.SteinICPError):
                sol.set_tiling(q, w, 64)
        finally:
            sol.close()
        return
    for src, ref, theta0, sched, K, m, rows in cases:
        cfg = S.stein_icp_default_config(num_particles=K, batch_size=m, schedule_rows=rows, autotune=0,
                                         nn_mode=mode)
        ocfg = oracle.make_config(K, m, len(src), len(ref))
        want = oracle.step(ocfg, src, ref, sched[0], oracle.State(theta0))["match"]
        sol = S.SteinICP(cfg, dev(src), dev(ref), dev(theta0), dev(sched))
        for nb in (1, 2, 3, 5, 8, 13, 21, 34, 55, 89):
            sol.set_tiling(q, w, 32 * nb)
            sol.set_state(dev(theta0))
            sol.step(1)
            got = sol.diagnostics()["match"].cpu().numpy()[0]
            assert np.array_equal(got, want), (q, w, nb, int((got != want).sum()))
        sol.close()


# the shortest chunk, in blocks of 32 references per wavefront, from which
# the two-queries-per-lane screen keys two blocks at a time
TWO_BLOCK_KEY_RANGE = 192


@pytest.mark.parametrize("mode", SCREENS)
@pytest.mark.parametrize("w", [4, 8])
def test_screen_two_block_keys_every_block_count_per_wavefront(w, mode):
    """With two queries per lane and chunks of at least 192 blocks per
    wavefront, each key spans two blocks of 32 references. Reference clouds
    of 1 to 89 blocks (ragged last blocks included) give the wavefronts 0 to
    23 blocks each: odd and even counts, every tail of the block loops, a
    last key of one block. The first iteration's matches equal the
    oracle's (lowest index on ties), on the cuboid pair and on an all-ties
    grid, and equal those of the one-block keys (a chunk one block
    shorter)."""
    prob = synth.make_problem("cuboid", 0, T=1)
    gsrc, gref, gtheta, gsched, gK, gm, grows = _grid_problem()
    long_chunk = 32 * w * TWO_BLOCK_KEY_RANGE
    for nb in (1, 2, 3, 4, 5, 7, 8, 9, 13, 21, 34, 47, 55, 89):
        for src, ref, theta0, sched, K, m, rows in (
                (prob.pair.src, prob.pair.ref, prob.theta0, prob.schedule, prob.K, prob.m, prob.schedule.shape[0]),
                (gsrc, gref, gtheta, gsched, gK, gm, grows)):
            ref = ref[: max(1, 32 * nb - (nb % 3) * 7)]
            cfg = S.stein_icp_default_config(num_particles=K, batch_size=m, schedule_rows=rows, autotune=0,
                                             nn_mode=mode)
            ocfg = oracle.make_config(K, m, len(src), len(ref))
            want = oracle.step(ocfg, src, ref, sched[0], oracle.State(theta0))["match"]
            sol = S.SteinICP(cfg, dev(src), dev(ref), dev(theta0), dev(sched))
            try:
                for chunk in (long_chunk, long_chunk - 32):
                    sol.set_tiling(2, w, chunk)
                    sol.set_state(dev(theta0))
                    sol.step(1)
                    got = sol.diagnostics()["match"].cpu().numpy()[0]
                    assert np.array_equal(got, want), (w, nb, len(ref), chunk, int((got != want).sum()))
            finally:
                sol.close()


def test_bf16_solver_equals_the_fp32_solver_bitwise():
    """With the certified screen the matches are the FP32 search's, so the
    whole solve is bit for bit the FP32 solve (and the first iteration's
    matches are the oracle's)."""
    for name in ("kinect", "cuboid"):
        prob = synth.make_problem(name, 0, T=10)
        gcfg, ocfg = both_configs(prob, {})
        runs = {}
        for mode in (S.NN_FP32, S.NN_BF16_RERANK, S.NN_F16_RERANK):
            gcfg.nn_mode = mode
            sol = S.SteinICP(gcfg, dev(prob.pair.src), dev(prob.pair.ref), dev(prob.theta0), dev(prob.schedule))
            sol.step(1)
            match = sol.diagnostics()["match"].cpu().numpy()[0]
            sol.step(prob.T - 1)
            runs[mode] = (match, sol.particles().cpu().numpy()[0])
            sol.close()
        st = oracle.State(prob.theta0)
        od = oracle.step(ocfg, prob.pair.src, prob.pair.ref, prob.schedule[0], st)
        np.testing.assert_array_equal(runs[S.NN_BF16_RERANK][0], od["match"])
        np.testing.assert_array_equal(runs[S.NN_BF16_RERANK][0], runs[S.NN_FP32][0])
        np.testing.assert_array_equal(runs[S.NN_BF16_RERANK][1], runs[S.NN_FP32][1])
        np.testing.assert_array_equal(runs[S.NN_F16_RERANK][0], od["match"])
        np.testing.assert_array_equal(runs[S.NN_F16_RERANK][1], runs[S.NN_FP32][1])


# ------------------------------------------------------------------ the bench's launch shapes

def _pinned(workload, nn):
    import bench
    return tuple(int(x) for x in bench.PINNED_TILING[(workload, nn)].split(","))


def test_kinect_full_solve_at_the_bench_shapes_bf16_equals_fp32_and_oracle():
    """The benched Kinect solve (K 100, m 300, M 20,000, T 200) with the
    pinned NN shape of each search mode: both give the same particles bit
    for bit, within the pose bar of the oracle's solve."""
    prob = synth.make_problem("kinect", 0)
    print(f"kinect full solve at bench shapes: T={prob.T}", flush=True)
    out = {}
    for nn, mode in (("bf16", S.NN_BF16_RERANK), ("f16", S.NN_F16_RERANK), ("fp32", S.NN_FP32)):
        gcfg, _ = both_configs(prob)
        gcfg.nn_mode = mode
        sol = S.SteinICP(gcfg, dev(prob.pair.src), dev(prob.pair.ref), dev(prob.theta0), dev(prob.schedule))
        sol.set_tiling(*_pinned("kinect", nn))
        sol.step(prob.T)
        out[nn] = sol.particles().cpu().numpy()[0]
        sol.close()
    np.testing.assert_array_equal(out["bf16"], out["fp32"])
    np.testing.assert_array_equal(out["f16"], out["fp32"])
    assert_poses_close(out["bf16"], oracle_run(prob, prob.T))


@pytest.mark.parametrize("nn", ["bf16", "f16", "fp32"])
def test_lidar_full_size_iteration_at_the_bench_shape(nn):
    """One LiDAR iteration (K 300, m 1000, M 100,000) with the pinned NN shape
    the bench times, against the oracle (matches bit-exact)."""
    prob = synth.make_problem("lidar", 0, T=1)
    print(f"lidar full-size iteration at the bench shape ({nn})", flush=True)
    gcfg, ocfg = both_configs(prob)
    gcfg.nn_mode = {"bf16": S.NN_BF16_RERANK, "f16": S.NN_F16_RERANK, "fp32": S.NN_FP32}[nn]
    sol = S.SteinICP(gcfg, dev(prob.pair.src), dev(prob.pair.ref), dev(prob.theta0), dev(prob.schedule))
    sol.set_tiling(*_pinned("lidar", nn))
    sol.step(1)
    diag = {k: v.cpu().numpy()[0] for k, v in sol.diagnostics().items()}
    th = sol.particles().cpu().numpy()[0]
    sol.close()
    st = oracle.State(prob.theta0)
    od = oracle.step(ocfg, prob.pair.src, prob.pair.ref, prob.schedule[0], st)
    np.testing.assert_array_equal(diag["match"], od["match"])
    np.testing.assert_allclose(diag["gbar"], od["gbar"], rtol=STEP_RTOL, atol=1e-13)
    np.testing.assert_allclose(th, st.theta, rtol=0, atol=1e-11)


@pytest.mark.parametrize("K", [40, 150, 240])
def test_batched_bandwidths_beside_the_screen_search(K):
    """A few pairs with few particles in flight (pairs x K <= 512) take the
    bandwidth workgroups of every pair into the screen launch: keys in LDS
    (K = 40), keys in global memory (K = 150, 240). Each pair's bandwidths
    and the particles after the solve equal the FP32 batch's bit for bit."""
    probs = synth.batched_problems(2, K=K, m=40, T=6, size_scale=0.3)
    out = {}
    for mode in (S.NN_FP32, S.NN_F16_RERANK, S.NN_BF16_RERANK):
        gcfg, _ = both_configs(probs[0])
        gcfg.nn_mode = mode
        b = S.SteinICP.batch(gcfg, [dev(p.pair.src) for p in probs], [dev(p.pair.ref) for p in probs],
                             dev(np.stack([p.theta0 for p in probs])), [dev(p.schedule) for p in probs])
        try:
            b.step(6)
            out[mode] = (b.diagnostics()["h"].cpu().numpy(), b.particles().cpu().numpy())
        finally:
            b.close()
    for mode in (S.NN_F16_RERANK, S.NN_BF16_RERANK):
        np.testing.assert_array_equal(out[mode][0], out[S.NN_FP32][0], err_msg=f"h, mode {mode}")
        np.testing.assert_array_equal(out[mode][1], out[S.NN_FP32][1], err_msg=f"particles, mode {mode}")


def test_batched_uneven_pairs_bf16_equals_fp32_bitwise():
    """Uneven pairs in one batch: both certified screens give the FP32
    search's particles bit for bit."""
    probs = synth.batched_problems(6, K=16, m=40, T=8, size_scale=0.3)
    out = {}
    for mode in (S.NN_FP32, S.NN_BF16_RERANK, S.NN_F16_RERANK):
        gcfg, _ = both_configs(probs[0])
        gcfg.nn_mode = mode
        b = S.SteinICP.batch(gcfg, [dev(p.pair.src) for p in probs], [dev(p.pair.ref) for p in probs],
                             dev(np.stack([p.theta0 for p in probs])), [dev(p.schedule) for p in probs])
        b.step(8)
        out[mode] = b.particles().cpu().numpy()
        b.close()
    np.testing.assert_array_equal(out[S.NN_BF16_RERANK], out[S.NN_FP32])
    np.testing.assert_array_equal(out[S.NN_F16_RERANK], out[S.NN_FP32])
