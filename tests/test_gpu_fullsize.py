"""Parity at the benched sizes: the LiDAR workload late in its solve and the
batched workload with all 64 pairs at their full sizes, through the C ABI,
against the FP64 oracle on the same clouds, particles and minibatches.

Both follow the whole-iteration protocol of the oracle: the GPU state after
t iterations (particles, Adam moments, step count) is loaded into the
oracle, both sides take the next iteration (minibatch, transform, Eq. 1,
Eqs. 4-5, Eq. 16 with the median bandwidths, Adam), and the results are
compared with the bars of the one-iteration tests: matches bit-exact,
gbar and phi within 1e-9 relative, h within 1e-12, particles within 1e-11.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2106_03287_amd import stein_icp as S

pytestmark = pytest.mark.gpu

STEP_RTOL = 1e-9


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _pinned(workload, nn):
    import bench
    return tuple(int(x) for x in bench.PINNED_TILING[(workload, nn)].split(","))


def _assert_step(diag, th_gpu, od, th_or, tag):
    """One iteration's quantities of one pair against the oracle's."""
    bad = int((diag["match"] != od["match"]).sum())
    assert bad == 0, f"{tag}: {bad} matches differ"
    np.testing.assert_allclose(diag["gbar"], od["gbar"], rtol=STEP_RTOL, atol=1e-13, err_msg=tag)
    np.testing.assert_allclose(diag["h"], od["h"], rtol=1e-12, err_msg=tag)
    scale = np.abs(od["phi"]).max()
    np.testing.assert_allclose(diag["phi"], od["phi"], rtol=STEP_RTOL, atol=1e-12 * scale, err_msg=tag)
    np.testing.assert_allclose(th_gpu, th_or, rtol=0, atol=1e-11, err_msg=tag)


def test_lidar_iterations_late_in_the_solve_at_the_bench_shapes():
    """LiDAR (K 300, m 1000, M 100,000, T 300) solved on the GPU with the
    FP32 search and both matrix-core screens at the NN shapes the bench
    times; at t = 50, 150 and 299 the three GPU states are bitwise equal, and
    the next iteration from that state matches the oracle's. The screens' failed certificates (rescanned in
    FP32) are counted along the way."""
    prob = synth.make_problem("lidar", 0)
    rows = prob.schedule.shape[0]
    cfg = S.stein_icp_default_config(num_particles=prob.K, batch_size=prob.m, schedule_rows=rows, lr=prob.lr)
    ocfg = oracle.make_config(prob.K, prob.m, len(prob.pair.src), len(prob.pair.ref), lr=prob.lr)
    src, ref, th0, sch = dev(prob.pair.src), dev(prob.pair.ref), dev(prob.theta0), dev(prob.schedule)
    sols = {}
    for nn, mode in (("fp32", S.NN_FP32), ("bf16", S.NN_BF16_RERANK), ("f16", S.NN_F16_RERANK)):
        cfg.nn_mode = mode
        sols[nn] = S.SteinICP(cfg, src, ref, th0, sch)
        sols[nn].set_tiling(*_pinned("lidar", nn))
    done = 0
    try:
        for t in (50, 150, 299):
            print(f"lidar: GPU solves to t={t}", flush=True)
            for sol in sols.values():
                sol.step(t - done)
            states = {nn: sol.get_state() for nn, sol in sols.items()}
            for other in ("bf16", "f16"):
                for a, b in zip(states["fp32"][:3], states[other][:3]):
                    assert torch.equal(a, b)
            th, mo, ve, tt = states["fp32"]
            assert tt == t
            st = oracle.State(th.cpu().numpy()[0], mo.cpu().numpy()[0], ve.cpu().numpy()[0], t)
            print(f"lidar: oracle iteration {t} -> {t + 1}", flush=True)
            od = oracle.step(ocfg, prob.pair.src, prob.pair.ref, prob.schedule[t % rows], st)
            for nn, sol in sols.items():
                sol.step(1)
                diag = {k: v.cpu().numpy()[0] for k, v in sol.diagnostics().items()}
                _assert_step(diag, sol.particles().cpu().numpy()[0], od, st.theta, f"lidar {nn} t={t}")
            for other in ("bf16", "f16"):
                r, n = sols[other].nn_rescans()
                print(f"lidar t={t + 1}: {other} certificates {n}, failed and rescanned {r} ({r / n:.2e})",
                      flush=True)
                assert 0 < n and 0 <= r < n
            done = t + 1
        assert sols["fp32"].nn_rescans() == (0, 0)
    finally:
        for sol in sols.values():
            sol.close()


@pytest.fixture(scope="module")
def batched64():
    print("generating the 64 batched pairs", flush=True)
    return synth.batched_problems(64)


@pytest.mark.parametrize("mode", [S.NN_BF16_RERANK, S.NN_F16_RERANK])
def test_batched_64_full_size_pairs_equal_sequential_solves_and_the_oracle(batched64, mode):
    """The batched workload at full size (64 pairs, M 2k-50k, N 1k-20k, K 100,
    m 300, T 150) in one context with a certified matrix-core screen at the
    tuner's shapes equals 64 single-pair FP32 contexts bit for bit after
    the whole solve; the first and the last-plus-one iterations of three
    pairs (the largest reference among them) match the oracle."""
    probs = batched64
    P, K, m = len(probs), probs[0].K, probs[0].m
    T = probs[0].T
    rows = probs[0].schedule.shape[0]
    srcs = [dev(p.pair.src) for p in probs]
    refs = [dev(p.pair.ref) for p in probs]
    scheds = [dev(p.schedule) for p in probs]
    th0 = dev(np.stack([p.theta0 for p in probs]))
    cfg = S.stein_icp_default_config(num_particles=K, batch_size=m, schedule_rows=rows, lr=probs[0].lr,
                                     nn_mode=mode, autotune=1)
    print(f"batched: {P} pairs, M {min(len(p.pair.ref) for p in probs)}-{max(len(p.pair.ref) for p in probs)}",
          flush=True)
    batch = S.SteinICP.batch(cfg, srcs, refs, th0, scheds)
    print(f"batched: tuned shape {batch.tiling()}", flush=True)
    picks = [int(np.argmax([len(p.pair.ref) for p in probs])), 0, 1]
    ocfgs = {i: oracle.make_config(K, m, len(probs[i].pair.src), len(probs[i].pair.ref), lr=probs[i].lr)
             for i in picks}
    try:
        # first iteration from the initial particles
        batch.step(1)
        diag = {k: v.cpu().numpy() for k, v in batch.diagnostics().items()}
        th = batch.particles().cpu().numpy()
        for i in picks:
            st = oracle.State(probs[i].theta0)
            od = oracle.step(ocfgs[i], probs[i].pair.src, probs[i].pair.ref, probs[i].schedule[0], st)
            _assert_step({k: v[i] for k, v in diag.items()}, th[i], od, st.theta, f"pair {i} t=0")
        batch.step(T - 1)
        got = batch.particles().cpu().numpy()
        print("batched: sequential single-pair solves", flush=True)
        cfg1 = S.stein_icp_default_config(num_particles=K, batch_size=m, schedule_rows=rows, lr=probs[0].lr)
        for i, p in enumerate(probs):
            sol = S.SteinICP(cfg1, srcs[i], refs[i], th0[i].contiguous(), scheds[i])
            sol.step(T)
            one = sol.particles().cpu().numpy()[0]
            sol.close()
            assert np.array_equal(got[i], one), f"pair {i} differs from its single-pair solve"
        # the iteration after the whole solve, from the batch's state
        thb, mob, veb, tt = batch.get_state()
        assert tt == T
        batch.step(1)
        diag = {k: v.cpu().numpy() for k, v in batch.diagnostics().items()}
        th = batch.particles().cpu().numpy()
        for i in picks:
            st = oracle.State(thb.cpu().numpy()[i], mob.cpu().numpy()[i], veb.cpu().numpy()[i], T)
            od = oracle.step(ocfgs[i], probs[i].pair.src, probs[i].pair.ref, probs[i].schedule[T % rows], st)
            _assert_step({k: v[i] for k, v in diag.items()}, th[i], od, st.theta, f"pair {i} t={T}")
        r, n = batch.nn_rescans()
        print(f"batched (mode {mode}): certificates {n}, failed and rescanned {r} ({r / n:.2e})", flush=True)
    finally:
        batch.close()
