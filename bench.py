"""Stein-ICP throughput on one MI355X.

One step = one complete solve of the workload: reset the K particles and the
Adam state to the seeded initial set, then run T iterations (minibatch,
transform, brute-force nearest neighbours, mean gradients, Stein direction,
Adam), all on the GPU through the C ABI. Inputs are resident in HBM before
the timed region. Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload kinect]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Stein-ICP iters/s & particle·point NN queries/s; time-to-MMD≤0.05 vs plain"
VALU_PEAK_TFLOPS = 157.3    # MI355X FP32 vector peak: 256 CUs x 2.4 GHz x 256 FP32 flop/clk/CU
MFMA_BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 matrix peak
HBM_PEAK_GBPS = 8000.0      # MI355X HBM3E
NORMAL_K = 10               # neighbours per normal of the point-to-plane metric
# Algorithmic work of one pair evaluation of Eq. 1: the FP32 squared distance,
# 3 subtractions, 1 multiply and 2 fused multiply-adds (2 flops each) = 8 flops.
FLOPS_PER_PAIR = 8
# Issued matrix-core work of the screens per pair: BF16 x 3 takes two
# 32x32x16 BF16 products (2 * 32 * 32 * 16 flops each) per 32 references x
# 32 queries = 64 flops (24 of its 32 K slots carry the three-part split);
# FP16 x 2 takes one 32x32x16 FP16 product = 32 flops (15 of 16 K slots).
MFMA_FLOPS_PER_PAIR_ISSUED = {"bf16": 64, "f16": 32}
SCREENS = ("bf16", "f16")
NN_MODE = {"fp32": 0, "bf16": 1, "f16": 2}     # STEIN_ICP_NN_*
DTYPE = {"fp32": "f32", "bf16": "bf16+f32", "f16": "f16+f32"}
NN_SOURCES = ["paper_2106_03287_amd/csrc/nn.hpp", "paper_2106_03287_amd/csrc/common.hpp"]
NN_BF16_SOURCES = NN_SOURCES + ["paper_2106_03287_amd/csrc/nn_bf16.hpp"]


def host_info(smi=True):
    """Host CPU and the GPU's clocks and power as found (rocm-smi, run as a
    child process). Called before this process touches the GPU: a process
    that has initialised the GPU starts no other program (under a profiler
    that initialises it first, pass --no-smi). Any field that cannot be read
    is None."""
    import subprocess
    info = {"cpu_model": None, "cpu_threads": os.cpu_count(), "rocm_smi": None}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        if not smi:
            raise RuntimeError("rocm-smi not queried")
        r = subprocess.run(["rocm-smi", "--showclocks", "--showpower", "--json"], capture_output=True, text=True,
                           timeout=20)
        card = next(iter(json.loads(r.stdout).values()))
        info["rocm_smi"] = {k: v for k, v in card.items()
                            if any(w in k.lower() for w in ("sclk", "mclk", "fclk", "power"))}
    except Exception:
        pass
    return info


def gpu_info(host):
    """The host record with the device, HIP and torch versions added (no
    child process: the GPU is initialised by now)."""
    import torch
    info = dict(host)
    info["hip"] = getattr(torch.version, "hip", None)
    info["torch"] = torch.__version__
    try:
        info["gpu"] = torch.cuda.get_device_name(0)
    except Exception:
        info["gpu"] = None
    return info


def code_text(path):
    """A source file's code with its comments and blank space taken out, so
    that a fingerprint of it changes with the code and not with the comments
    (the kernel sources hold no string literals)."""
    import re
    t = open(path).read()
    t = re.sub(r"/\*.*?\*/", " ", t, flags=re.S)
    t = re.sub(r"//[^\n]*", " ", t)
    return " ".join(t.split())


def nn_source_sha(nn="fp32"):
    import hashlib
    h = hashlib.sha256()
    for f in (NN_BF16_SOURCES if nn in SCREENS else NN_SOURCES):
        h.update(code_text(os.path.join(ROOT, f)).encode())
    return h.hexdigest()[:16]


def measured_counters(workload, tiling, nn="fp32"):
    """Counter figures of the NN kernel from the committed rocprofv3 runs
    (HBM bytes per launch from FETCH_SIZE / WRITE_SIZE scaled by a plain
    copy, and the matrix-core busy fraction), if they were taken on the
    current kernel source, this workload, search mode and NN shape; else {}."""
    path = os.path.join(ROOT, "profiles", "nn_traffic.json")
    if not os.path.exists(path):
        return {}
    rec = json.load(open(path)).get(workload if nn == "fp32" else f"{workload}:{nn}")
    shape = "%d,%d,%d,%d" % (tiling["queries_per_lane"], tiling["waves"], tiling["chunk"], tiling["persist"])
    if not rec or rec.get("source_sha") != nn_source_sha(nn) or rec.get("tiling") != shape:
        return {}
    return rec


CEILINGS = {}   # the device's own ceilings, measured once per run (paper_2106_03287_amd.peaks)


def measure_ceilings():
    """Streaming copy, unpacked FP32 FMA and 32x32x16 FP16 / BF16 matrix-core
    rates of this device, best of five probes each, before any timed region."""
    from paper_2106_03287_amd import peaks
    CEILINGS.update(peaks.measure())
    return {k: (round(v, 1) if isinstance(v, float) else v) for k, v in CEILINGS.items()}


def nn_roofline(nn, pairs_per_launch, nn_ms, counters):
    """Roofline of the dominant kernel, the nearest-neighbour search: the
    algorithmic 8 flops per pair evaluation over the launch time, against
    the peak of the arithmetic the kernel runs on (BF16 matrix cores for the
    screen, FP32 vector ALUs for the plain search); the screen's issued
    matrix-core work, the counted HBM bytes and their rate beside it."""
    t = nn_ms * 1e-3
    useful = pairs_per_launch * FLOPS_PER_PAIR / t / 1e12
    traffic = counters.get("hbm_bytes_per_launch")
    out = {"achieved": round(useful, 3), "unit": "TFLOP/s", "traffic": traffic,
           "flops_per_pair": FLOPS_PER_PAIR, "avg_launch_ms": round(nn_ms, 5),
           "pair_evals_per_launch": pairs_per_launch,
           "hbm_gbps": None if traffic is None else round(traffic / t / 1e9, 1),
           "hbm_frac": None if traffic is None else round(traffic / t / 1e9 / HBM_PEAK_GBPS, 4)}
    if nn in SCREENS:
        per = MFMA_FLOPS_PER_PAIR_ISSUED[nn]
        issued = pairs_per_launch * per / t / 1e12
        out.update(bound="mfma", peak=MFMA_BF16_PEAK_TFLOPS, frac=round(useful / MFMA_BF16_PEAK_TFLOPS, 4),
                   kernel="nn_bf16_kernel (%s)" % ("BF16 x 3" if nn == "bf16" else "FP16 x 2"),
                   issued_mfma={"flops_per_pair": per, "achieved": round(issued, 3),
                                "frac": round(issued / MFMA_BF16_PEAK_TFLOPS, 4)},
                   mfma_busy=counters.get("mfma_busy"), valu_busy=counters.get("valu_busy"),
                   valu_insts_per_mfma=counters.get("valu_insts_per_mfma"))
    else:
        out.update(bound="alu", peak=VALU_PEAK_TFLOPS, frac=round(useful / VALU_PEAK_TFLOPS, 4),
                   kernel="nn_fp32_kernel")
    if CEILINGS:
        # the same achieved rate against the ceiling this device sustains for
        # the kernel's arithmetic (the build has no packed FP32 instructions,
        # so the FP32 search's ceiling is the unpacked FMA rate)
        key = {"f16": "mfma_f16_tflops", "bf16": "mfma_bf16_tflops"}.get(nn, "fp32_fma_tflops")
        out["measured_peak"] = {"value": round(CEILINGS[key], 1), "unit": "TFLOP/s", "probe": key,
                                "frac": round(useful / CEILINGS[key], 4)}
        if traffic is not None:
            out["hbm_frac_of_measured_copy"] = round(traffic / t / 1e9 / CEILINGS["hbm_copy_gbps"], 4)
    order = ["bound", "achieved", "peak", "unit", "frac", "traffic"]
    return {k: out[k] for k in order + sorted(k for k in out if k not in order)}


def cpu_baseline(prob, budget_s=15.0, plane=False):
    """The FP64 oracle as it stands, on this host's cores, for as many of the
    workload's iterations as fit in about ``budget_s`` seconds (point-to-plane:
    the normals are computed first, outside the timing, as at init)."""
    import oracle
    cfg = oracle.make_config(prob.K, prob.m, len(prob.pair.src), len(prob.pair.ref), lr=prob.lr,
                             metric=oracle.PLANE if plane else oracle.POINT)
    nrm = oracle.normals(prob.pair.ref, NORMAL_K)[0] if plane else None
    st = oracle.State(prob.theta0)
    oracle.run(cfg, prob.pair.src, prob.pair.ref, prob.schedule, 1, st, normals=nrm)  # warm-up / estimate
    t0 = time.perf_counter()
    oracle.run(cfg, prob.pair.src, prob.pair.ref, prob.schedule, 1, st, normals=nrm)
    per = time.perf_counter() - t0
    n = int(max(1, min(prob.T - 2, budget_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    oracle.run(cfg, prob.pair.src, prob.pair.ref, prob.schedule, n, st, normals=nrm)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": (n + 1) / (dt + per), "unit": "iters/s", "cores": cores, "kind": "oracle",
            "sample": f"iterations 2-{n + 2} of the {prob.name} workload (pair 0, K={prob.K}, "
                      f"m={prob.m}, M={len(prob.pair.ref)}{', point-to-plane' if plane else ''}), "
                      f"FP64 oracle with OpenMP NN; the rate of these iterations, extrapolated to "
                      f"the T={prob.T} solve"}


class KDTreeReference:
    """A fast CPU form of the iteration for context beside the oracle (not the
    oracle, and not the product): the nearest neighbours of the FP32 queries
    from a scipy cKDTree over the reference (the oracle's threads, distances in
    FP64, so a near-tie may match differently from the FP32 search), the rest
    vectorised in NumPy FP64 as the method states it: minibatch row t mod
    rows, the pose R = Rz(yaw) Ry(pitch) Rx(roll) and its derivatives, the
    mean gradient of Eqs. 4-5, the Stein direction of Eq. 16 with the
    wrapped-angle kernel of Eq. 17 and median-heuristic bandwidths, Adam on
    the negative direction (Sec. V)."""

    def __init__(self, prob, beta1=0.9, beta2=0.999, eps=1e-8):
        from scipy.spatial import cKDTree
        self.src = np.asarray(prob.pair.src, np.float32)
        self.ref = np.asarray(prob.pair.ref, np.float32).astype(np.float64)
        self.tree = cKDTree(self.ref)
        self.workers = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))   # the oracle's threads
        self.sched = np.asarray(prob.schedule)
        self.K, self.m, self.N, self.lr = prob.K, prob.m, len(prob.pair.src), prob.lr
        self.b1, self.b2, self.eps = beta1, beta2, eps
        self.theta = np.array(prob.theta0, np.float64)
        self.mom = np.zeros_like(self.theta)
        self.vel = np.zeros_like(self.theta)
        self.t = 0

    @staticmethod
    def _wrap(x):
        return x - np.rint(x / (2 * np.pi)) * (2 * np.pi)

    @staticmethod
    def _pose(th):
        cr, sr = np.cos(th[:, 3]), np.sin(th[:, 3])
        cp, sp = np.cos(th[:, 4]), np.sin(th[:, 4])
        cy, sy = np.cos(th[:, 5]), np.sin(th[:, 5])
        z, o = np.zeros_like(cr), np.ones_like(cr)
        Rx = np.stack([o, z, z, z, cr, -sr, z, sr, cr], 1).reshape(-1, 3, 3)
        Ry = np.stack([cp, z, sp, z, o, z, -sp, z, cp], 1).reshape(-1, 3, 3)
        Rz = np.stack([cy, -sy, z, sy, cy, z, z, z, o], 1).reshape(-1, 3, 3)
        dRx = np.stack([z, z, z, z, -sr, -cr, z, cr, -sr], 1).reshape(-1, 3, 3)
        dRy = np.stack([-sp, z, cp, z, z, z, -cp, z, -sp], 1).reshape(-1, 3, 3)
        dRz = np.stack([-sy, -cy, z, cy, -sy, z, z, z, z], 1).reshape(-1, 3, 3)
        R = Rz @ Ry @ Rx
        return R, np.stack([Rz @ Ry @ dRx, Rz @ dRy @ Rx, dRz @ Ry @ Rx], 1)

    def step(self):
        K, m = self.K, self.m
        s = self.src[self.sched[self.t % len(self.sched)]].astype(np.float64)          # m x 3
        R, D = self._pose(self.theta)
        q = np.einsum("kij,mj->kmi", R, s) + self.theta[:, None, :3]                     # K x m x 3
        _, j = self.tree.query(q.astype(np.float32).reshape(-1, 3).astype(np.float64), workers=self.workers)
        e = q - self.ref[j].reshape(K, m, 3)
        g = np.empty((K, 6))
        g[:, :3] = e.mean(1)
        g[:, 3:] = np.einsum("kmi,kdij,mj->kd", e, D, s, optimize=True) / m
        dt = self.theta[:, None, :3] - self.theta[None, :, :3]                            # l, k
        dr = self._wrap(self.theta[:, None, 3:] - self.theta[None, :, 3:])
        d2 = [(dt ** 2).sum(-1), (dr ** 2).sum(-1)]
        iu = np.triu_indices(K, 1)
        G = -self.N * g
        phi = np.zeros((K, 6))
        for b, diff in enumerate((dt, dr)):
            if K > 1:
                v = np.sort(d2[b][iu])
                n = len(v)
                med = np.sqrt(v[(n - 1) // 2]) if n % 2 else 0.5 * (np.sqrt(v[n // 2 - 1]) + np.sqrt(v[n // 2]))
                h = med * med / np.log(K) if med > 0 else 1.0
            else:
                h = 1.0
            kern = np.exp(-d2[b] / h)
            sl = slice(3 * b, 3 * b + 3)
            phi[:, sl] = (kern.T @ G[:, sl] + (-2.0 / h) * np.einsum("lk,lkd->kd", kern, diff)) / K
        self.t += 1
        gr = -phi
        self.mom = self.b1 * self.mom + (1 - self.b1) * gr
        self.vel = self.b2 * self.vel + (1 - self.b2) * gr * gr
        mh = self.mom / (1 - self.b1 ** self.t)
        vh = self.vel / (1 - self.b2 ** self.t)
        self.theta = self.theta - self.lr * mh / (np.sqrt(vh) + self.eps)
        return j


def cpu_kdtree_reference(prob, budget_s=10.0):
    """KDTreeReference timed on this host for about ``budget_s`` seconds."""
    ref = KDTreeReference(prob)
    ref.step()   # warm-up
    t0 = time.perf_counter()
    n = 0
    while n < prob.T - 1 and (n == 0 or time.perf_counter() - t0 < budget_s):
        ref.step()
        n += 1
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "iters/s", "cores": ref.workers,
            "kind": "scipy cKDTree nearest neighbours + NumPy FP64 (a fast CPU form, not the oracle)",
            "sample": f"iterations 2-{n + 1} of the {prob.name} workload (K={prob.K}, m={prob.m}, "
                      f"M={len(prob.pair.ref)}), the tree built outside the timing"}


# Search mode of --nn auto. The certified screens return the FP32 search's
# answers bit for bit. The FP16 x 2 screen (one matrix product per block)
# measured faster than the BF16 x 3 screen (two) on the NN launch: LiDAR
# 1.22 against 1.64 ms, Kinect 36.9 against 44.3 us; both beat the FP32
# search there, and neither does on the small cuboid clouds, where the search
# is latency-bound.
AUTO_NN = {"cuboid": "fp32", "kinect": "f16", "lidar": "f16", "mc": "f16", "batched": "f16"}

# NN shapes (queries per lane, wavefronts per workgroup, chunk, persistent
# workgroups per CU) pinned from sweeps of the NN launch on one MI355X: LiDAR
# FP16 x 2 1.22 ms with one chunk (1.24 with two, 1.44 with four), BF16 x 3
# 1.64 ms with two (1.77 with four); Kinect one chunk of the whole reference.
PINNED_TILING = {
    ("kinect", "fp32"): "4,16,2048,2",
    ("kinect", "bf16"): "2,8,20096,0",
    ("kinect", "f16"): "2,8,20096,0",
    ("lidar", "fp32"): "4,8,4096,0",
    ("lidar", "bf16"): "2,4,50176,0",
    ("lidar", "f16"): "2,4,50016,0",
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="lidar", choices=["cuboid", "kinect", "lidar", "batched", "proposal", "mc"])
    ap.add_argument("--runs", type=int, default=1000, help="independent single-particle runs of the mc workload")
    ap.add_argument("--pairs", type=int, default=64, help="pairs of the batched and proposal workloads")
    ap.add_argument("--workers", type=int, default=16,
                    help="host processes generating the proposal workload's pairs (1: in process)")
    ap.add_argument("--nn", default="auto", choices=["auto", "fp32", "bf16", "f16"],
                    help="nearest-neighbour search: FP32, or a certified matrix-core screen, BF16 x 3 or FP16 x 2 "
                         "(the same answers); auto takes the faster for the workload")
    ap.add_argument("--metric", default="point", choices=["point", "plane"],
                    help="ICP error metric: point-to-point (Eqs. 4-5) or point-to-plane (normals at init)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-smi", action="store_true",
                    help="do not query rocm-smi (a profiler that initialises the GPU before the program starts "
                         "forbids starting another program)")
    ap.add_argument("--autotune", type=int, default=0,
                    help="tune the NN shape at init instead of using the pinned shape of the workload")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this size first (counter calibration)")
    ap.add_argument("--iters", type=int, default=0,
                    help="iterations per solve (default: the workload's T); for short profiled runs")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip measuring the device's own copy / FMA / matrix-core ceilings (skipped anyway "
                         "with --iters, the short profiled runs)")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batched workload: skip the same pairs solved one after another (counter runs, whose "
                         "kernel records should hold the batched launches only)")
    ap.add_argument("--tiling", default="",
                    help="force the NN shape 'queries_per_lane,waves,chunk[,persist]' instead of tuning")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the particle-sharded multi-GPU design is described, not built)", file=sys.stderr)
        sys.exit(2)

    args.host = host_info(not args.no_smi)   # before anything touches the GPU
    import torch
    import synth
    from paper_2106_03287_amd import stein_icp as S

    args.ceilings = None
    if not args.no_ceilings and not args.iters:
        args.ceilings = measure_ceilings()
    if args.nn == "auto":
        args.nn = AUTO_NN.get(args.workload, "fp32")
    if not args.tiling and not args.autotune:
        args.tiling = PINNED_TILING.get((args.workload, args.nn), "")
        if not args.tiling:
            args.autotune = 1
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.workload == "batched":
        return run_batched(args)
    if args.workload == "proposal":
        return run_proposal(args)
    if args.workload == "mc":
        return run_mc(args)

    prob = synth.make_problem(args.workload, 0)
    if args.iters:
        prob.T = args.iters
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    src, ref = dev(prob.pair.src), dev(prob.pair.ref)
    theta0, sched = dev(prob.theta0), dev(prob.schedule)
    cfg = S.stein_icp_default_config(num_particles=prob.K, batch_size=prob.m,
                                     schedule_rows=prob.schedule.shape[0], lr=prob.lr,
                                     autotune=0 if args.tiling else args.autotune,
                                     nn_mode=NN_MODE[args.nn],
                                     metric=S.METRIC_PLANE if args.metric == "plane" else S.METRIC_POINT,
                                     normal_k=NORMAL_K)
    t_init = time.perf_counter()
    sol = S.SteinICP(cfg, src, ref, theta0, sched)
    init_ms = (time.perf_counter() - t_init) * 1e3
    normals_ms = None
    if args.metric == "plane":
        # the init-time normals alone (k nearest neighbours of every reference
        # point and their PCA), standalone call, median of 5
        S.stein_icp_normals(ref, NORMAL_K)
        ts = []
        for _ in range(5):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            S.stein_icp_normals(ref, NORMAL_K)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t1) * 1e3)
        normals_ms = float(np.median(ts))
    if args.tiling:
        sol.set_tiling(*[int(x) for x in args.tiling.split(",")])
    tiling = sol.tiling()
    zeros = torch.zeros_like(theta0)

    def solve():
        S.stein_icp_set_state(sol.ctx, theta0, zeros, zeros, 0)
        sol.step(prob.T)

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solve()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    iters_per_s = prob.T / (ms_per_step / 1e3)
    M = len(prob.pair.ref)
    queries_per_s = prob.K * prob.m * iters_per_s

    # stage times (HIP events on the launch stream around each stage of one
    # profiled solve) and the NN kernel alone over back-to-back launches
    S.stein_icp_set_state(sol.ctx, theta0, zeros, zeros, 0)
    stage = sol.stage_times(prob.T)
    nn_ms = sol.time_nn(max(20, min(200, int(200 / max(stage["nn"] / prob.T, 1e-3)))))
    pairs_per_launch = prob.K * prob.m * M
    roofline = nn_roofline(args.nn, pairs_per_launch, nn_ms, measured_counters(prob.name, tiling, args.nn))
    mismatch, identical = None, None
    if args.nn in SCREENS:
        # against the FP32 search from the same state: the first iteration's
        # matches, and the particles after the whole solve (bit for bit)
        S.stein_icp_set_state(sol.ctx, theta0, zeros, zeros, 0)
        sol.step(1)
        mb = sol.diagnostics()["match"]
        cfg32 = S.stein_icp_default_config(num_particles=prob.K, batch_size=prob.m,
                                           schedule_rows=prob.schedule.shape[0], lr=prob.lr,
                                           metric=cfg.metric, normal_k=NORMAL_K)
        ref32 = S.SteinICP(cfg32, src, ref, theta0, sched)
        ref32.step(1)
        mismatch = float((mb != ref32.diagnostics()["match"]).double().mean().item())
        solve()
        S.stein_icp_set_state(ref32.ctx, theta0, zeros, zeros, 0)
        ref32.step(prob.T)
        identical = bool(torch.equal(sol.particles(), ref32.particles()))
        ref32.close()
    sol.close()

    out = {
        "metric": METRIC,
        "value": round(iters_per_s, 2),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.nn],
        "data": "synthetic",
        "config": {"workload": prob.name, "K": prob.K, "m": prob.m, "T": prob.T,
                   "N": len(prob.pair.src), "M": M, "nn": args.nn, "metric": args.metric,
                   "step": "one full solve of T iterations"},
        "nn_queries_per_s": round(queries_per_s, 1),
        "pair_evals_per_s": round(queries_per_s * M, 1),
        "stage_ms_per_iter": {k: round(v / prob.T, 5) for k, v in stage.items()},
        "init_ms": round(init_ms, 2),
        "normals_ms": None if normals_ms is None else round(normals_ms, 3),
        "nn_tiling": tiling,
        "nn_mismatch_vs_fp32": mismatch,
        "particles_identical_to_fp32_solve": identical,
        "nn_source_sha": nn_source_sha(args.nn),
        "torch": torch.__version__,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, plane=args.metric == "plane")
        if args.metric == "point":
            out["cpu_fast_reference"] = cpu_kdtree_reference(prob)
    out["host"] = gpu_info(args.host)
    out["device_ceilings"] = args.ceilings
    print(json.dumps(out), flush=True)


def run_batched(args):
    """64 uneven pairs advanced together by one context (one launch per stage
    for all pairs, captured graph), against the same pairs solved one after
    another by 64 single-pair contexts on the same stream."""
    import torch
    import synth
    from paper_2106_03287_amd import stein_icp as S

    probs = synth.batched_problems(args.pairs)
    P, K, m = len(probs), probs[0].K, probs[0].m
    T = args.iters or probs[0].T
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    srcs = [dev(p.pair.src) for p in probs]
    refs = [dev(p.pair.ref) for p in probs]
    scheds = [dev(p.schedule) for p in probs]
    th0 = dev(np.stack([p.theta0 for p in probs]))
    cfg = S.stein_icp_default_config(num_particles=K, batch_size=m, schedule_rows=probs[0].schedule.shape[0],
                                     lr=probs[0].lr, autotune=0 if args.tiling else args.autotune,
                                     nn_mode=NN_MODE[args.nn])
    t_init = time.perf_counter()
    batch = S.SteinICP.batch(cfg, srcs, refs, th0, scheds)
    init_ms = (time.perf_counter() - t_init) * 1e3
    if args.tiling:
        batch.set_tiling(*[int(x) for x in args.tiling.split(",")])
    tiling = batch.tiling()
    zeros = torch.zeros_like(th0)
    singles = [] if args.no_sequential else [S.SteinICP(cfg, srcs[i], refs[i], th0[i].contiguous(), scheds[i])
                                             for i in range(P)]
    z1 = torch.zeros_like(th0[0])

    def solve_batched():
        S.stein_icp_set_state(batch.ctx, th0, zeros, zeros, 0)
        batch.step(T)

    def solve_sequential():
        for i, sol in enumerate(singles):
            S.stein_icp_set_state(sol.ctx, th0[i], z1, z1, 0)
            sol.step(T)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    ms_b = timed(solve_batched, args.steps, args.warmup)
    ms_s, same = None, None
    if singles:
        ms_s = timed(solve_sequential, max(1, args.steps // 2), 1)
        same = bool(torch.equal(batch.particles(), torch.stack([s.particles()[0] for s in singles])))
    S.stein_icp_set_state(batch.ctx, th0, zeros, zeros, 0)
    stage = batch.stage_times(T)
    nn_ms = batch.time_nn(20)
    pairs_per_launch = sum(K * m * len(p.pair.ref) for p in probs)
    roofline = nn_roofline(args.nn, pairs_per_launch, nn_ms, measured_counters("batched", tiling, args.nn))
    value = P * T / (ms_b / 1e3)
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "pair-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_b, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.nn],
        "data": "synthetic",
        "config": {"workload": "batched", "pairs": P, "K": K, "m": m, "T": T,
                   "M_range": [min(len(p.pair.ref) for p in probs), max(len(p.pair.ref) for p in probs)],
                   "N_range": [min(len(p.pair.src) for p in probs), max(len(p.pair.src) for p in probs)],
                   "nn": args.nn, "step": "one batched solve of all pairs, T iterations"},
        "sequential_ms": None if ms_s is None else round(ms_s, 3),
        "sequential_pair_iters_per_s": None if ms_s is None else round(P * T / (ms_s / 1e3), 2),
        "speedup_vs_sequential": None if ms_s is None else round(ms_s / ms_b, 3),
        "batched_equals_sequential_bitwise": same,
        "stage_ms_per_iter": {k: round(v / T, 5) for k, v in stage.items()},
        "init_ms": round(init_ms, 2),
        "nn_tiling": tiling,
        "roofline": roofline,
    }
    for s_ in singles:
        s_.close()
    batch.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batched(probs, T)
    out["host"] = gpu_info(args.host)
    out["device_ceilings"] = args.ceilings
    print(json.dumps(out), flush=True)


def run_mc(args):
    """The paper's Monte-Carlo ground truth (Sec. V-A) on the Kinect pair:
    ``runs`` independent single-particle runs (K = 1: SGD-ICP with Adam),
    starts uniform in +-1 m and +-0.1745 rad, each with its own minibatches,
    advanced together by one batch context whose pairs share the clouds; then
    the Stein-ICP posterior (K = 100) on the same pair, timed the same way and
    scored against the runs (KL of normal fits, per-coordinate OVL), beside
    the score of 100 of the runs drawn at random and of one half of the runs
    against the other (the sampling floor)."""
    import torch
    import synth
    from paper_2106_03287_amd import stein_icp as S

    prob = synth.make_problem("kinect", 0)
    T = args.iters or prob.T
    R = args.runs
    nn = "f16" if args.nn == "auto" else args.nn
    nn_mode = NN_MODE[nn]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    src, ref = dev(prob.pair.src), dev(prob.pair.ref)
    cfg = S.stein_icp_default_config(num_particles=1, batch_size=prob.m, schedule_rows=T, lr=prob.lr,
                                     seed=synth.MC_SEED, init_half_trans=synth.MC_HALF_TRANS,
                                     init_half_rot=synth.MC_HALF_ROT, nn_mode=nn_mode,
                                     autotune=0 if args.tiling else 1)
    t_init = time.perf_counter()
    mc = S.SteinICP.batch(cfg, [src] * R, [ref] * R)      # library-drawn starts and minibatches
    init_ms = (time.perf_counter() - t_init) * 1e3
    if args.tiling:
        mc.set_tiling(*[int(x) for x in args.tiling.split(",")])
    th0 = mc.particles().clone()
    zeros = torch.zeros_like(th0)
    scfg = S.stein_icp_default_config(num_particles=prob.K, batch_size=prob.m, schedule_rows=prob.schedule.shape[0],
                                      lr=prob.lr, nn_mode=nn_mode)
    stein = S.SteinICP(scfg, src, ref, dev(prob.theta0), dev(prob.schedule))
    if nn in SCREENS:
        stein.set_tiling(*[int(x) for x in PINNED_TILING[("kinect", nn)].split(",")])
    sz = torch.zeros_like(dev(prob.theta0))

    def solve_mc():
        S.stein_icp_set_state(mc.ctx, th0, zeros, zeros, 0)
        mc.step(T)

    def solve_stein():
        S.stein_icp_set_state(stein.ctx, dev(prob.theta0), sz, sz, 0)
        stein.step(T)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    ms_mc = timed(solve_mc, args.steps, args.warmup)
    ms_stein = timed(solve_stein, args.steps, args.warmup)
    solve_mc()
    solve_stein()
    gt = mc.particles().cpu().numpy()[:, 0]
    post = stein.particles().cpu().numpy()[0]
    kl, ovl = S.stein_icp_posterior_scores(post, gt)
    rng = np.random.default_rng(0)
    sub = gt[rng.choice(R, min(prob.K, R), replace=False)]
    kl_sub, ovl_sub = S.stein_icp_posterior_scores(sub, gt)
    half = rng.permutation(R)
    kl_half, ovl_half = S.stein_icp_posterior_scores(gt[half[: R // 2]], gt[half[R // 2:]])
    S.stein_icp_set_state(mc.ctx, th0, zeros, zeros, 0)
    stage = mc.stage_times(T)
    nn_ms = mc.time_nn(50)
    tiling = mc.tiling()
    M = len(prob.pair.ref)
    pairs_per_launch = R * prob.m * M
    roofline = nn_roofline(nn, pairs_per_launch, nn_ms, measured_counters("mc", tiling, nn))
    r4 = lambda v: [round(float(x), 4) for x in v]  # noqa: E731
    out = {
        "metric": METRIC,
        "value": round(R * T / (ms_mc / 1e3), 2),
        "unit": "run-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_mc, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[nn],
        "data": "synthetic",
        "config": {"workload": "mc", "pair": "kinect", "runs": R, "K": 1, "m": prob.m, "T": T, "M": M,
                   "start_box": [synth.MC_HALF_TRANS, synth.MC_HALF_ROT], "nn": nn,
                   "step": "all runs advanced T iterations together (one batch context, shared clouds)"},
        "stein_ms_per_solve": round(ms_stein, 4),
        "stein_K": prob.K,
        "mc_over_stein_time": round(ms_mc / ms_stein, 2),
        "scores_stein_vs_mc": {"kl_trans": round(float(kl[0]), 4), "kl_rot": round(float(kl[1]), 4), "ovl": r4(ovl)},
        "scores_100_random_runs_vs_mc": {"kl_trans": round(float(kl_sub[0]), 4), "kl_rot": round(float(kl_sub[1]), 4),
                                         "ovl": r4(ovl_sub)},
        "scores_half_vs_half": {"kl_trans": round(float(kl_half[0]), 4), "kl_rot": round(float(kl_half[1]), 4),
                                "ovl": r4(ovl_half)},
        "stage_ms_per_iter": {k: round(v / T, 5) for k, v in stage.items()},
        "init_ms": round(init_ms, 2),
        "nn_tiling": tiling,
        "torch": torch.__version__,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_mc(prob, T)
    mc.close()
    stein.close()
    out["host"] = gpu_info(args.host)
    out["device_ceilings"] = args.ceilings
    print(json.dumps(out), flush=True)


def cpu_baseline_batched(probs, T, budget_s=15.0):
    """The FP64 oracle on this host's cores over the batched workload's pairs
    in order, one pair after another, each for the iterations that fit its
    share of about ``budget_s`` seconds; pair-iterations per second over the
    pairs it reached."""
    import oracle
    done, spent, names = 0, 0.0, []
    for i, p in enumerate(probs):
        cfg = oracle.make_config(p.K, p.m, len(p.pair.src), len(p.pair.ref), lr=p.lr)
        st = oracle.State(p.theta0)
        t0 = time.perf_counter()
        oracle.run(cfg, p.pair.src, p.pair.ref, p.schedule, 1, st)
        per = time.perf_counter() - t0
        n = int(max(0, min(T - 1, (budget_s / 4 - per) / max(per, 1e-6))))
        t0 = time.perf_counter()
        if n:
            oracle.run(cfg, p.pair.src, p.pair.ref, p.schedule, n, st)
        spent += per + time.perf_counter() - t0
        done += n + 1
        names.append(f"pair {i} (M={len(p.pair.ref)}): {n + 1}")
        if spent >= budget_s or i == 3:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": done / spent, "unit": "pair-iters/s", "cores": cores, "kind": "oracle",
            "sample": "FP64 oracle with OpenMP NN, pairs one after another, iterations from the start: "
                      + ", ".join(names)}


def cpu_baseline_mc(prob, T, budget_s=15.0):
    """The FP64 oracle's single-particle runs on this host's cores: as many
    iterations of one run as fit in about ``budget_s`` seconds."""
    import oracle
    import synth
    theta0 = synth.init_particles(synth.MC_SEED, 1, synth.MC_HALF_TRANS, synth.MC_HALF_ROT)
    sched = synth.minibatch_schedule(synth.MC_SEED, len(prob.pair.src), prob.m, T)
    cfg = oracle.make_config(1, prob.m, len(prob.pair.src), len(prob.pair.ref), lr=prob.lr)
    st = oracle.State(theta0)
    t0 = time.perf_counter()
    oracle.run(cfg, prob.pair.src, prob.pair.ref, sched, 1, st)
    per = time.perf_counter() - t0
    n = int(max(1, min(T - 1, budget_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    oracle.run(cfg, prob.pair.src, prob.pair.ref, sched, n, st)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": (n + 1) / (dt + per), "unit": "run-iters/s", "cores": cores, "kind": "oracle",
            "sample": f"iterations 1-{n + 1} of one single-particle run on the kinect pair (m={prob.m}, "
                      f"M={len(prob.pair.ref)}), FP64 oracle with OpenMP NN"}


# multiply-accumulates of one forward pass per pair: the per-point MLP on
# 2 x 4096 points plus the 512-256-600 head
PROPOSAL_MACS_PER_PAIR = 2 * 4096 * (3 * 64 + 64 * 128 + 128 * 256) + 512 * 256 + 256 * 600


def run_proposal(args):
    """Time to MMD <= 0.05 on held-out pairs of the proposal's test split
    (cuboid and Kinect-shaped, alternating): the committed network plus
    Stein ICP with the certified FP16 x 2 search, against plain Stein ICP with
    the FP32 search from the uniform draw; MMD against the plain posterior
    (300 iterations from another draw), dimensions standardised by its
    spread, unbiased per pair, aggregated as sqrt(mean)."""
    import multiprocessing as mp
    pool = mp.get_context("fork").Pool(args.workers) if args.workers > 1 else None   # before any GPU use
    import torch
    from paper_2106_03287_amd import proposal as PR
    from paper_2106_03287_amd import train_proposal as TP
    weights = os.path.join(ROOT, "paper_2106_03287_amd", "weights", "proposal_k100_p4096.npy")
    cfg = PR.stein_icp_proposal_default_config(num_particles=100, points=4096, max_batch=32)
    model = PR.Proposal(cfg, np.load(weights, allow_pickle=False))
    ds, X, _ = TP.build_dataset(model, "test", args.pairs, pool, label=False)
    if pool is not None:
        pool.close()
    T = args.iters or 300
    res = TP.time_to_mmd(model, ds, X, T=T)
    n = len(ds)
    # the network alone over every pair (inputs prepared), for its roofline
    B = cfg.max_batch
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(0, n, B):
            model.forward(X[j:j + B].contiguous())
        torch.cuda.synchronize()
        net_ms = (time.perf_counter() - t0) * 1e3
    achieved = n * PROPOSAL_MACS_PER_PAIR * 2 / (net_ms * 1e-3) / 1e12
    reached = res["n_star"]["proposal"] is not None
    out = {
        "metric": "time-to-MMD<=0.05 vs plain (proposal + FP16 x 2 search)",
        "value": round(res["proposal_ms"], 3) if reached else None,
        "unit": "ms",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": round(res["proposal_ms"], 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 network, f16+f32 search and f64 Stein ICP (proposal); f32 search (plain)",
        "data": "synthetic",
        "config": {"workload": "proposal", "pairs": n, "K": 100, "T_reference": T, "threshold": res["threshold"],
                   "nn_proposal": "f16", "nn_plain": "fp32",
                   "step": "network inputs, network and n* Stein iterations on every pair (proposal); "
                           "n* iterations from the uniform draw (plain)"},
        "n_star_proposal": res["n_star"]["proposal"],
        "n_star_plain": res["n_star"]["plain"],
        "plain_ms": round(res["plain_ms"], 3),
        "plain_iters_timed": res["plain_iters_timed"],
        "speedup_vs_plain": round(res["plain_ms"] / res["proposal_ms"], 3) if reached else None,
        "mmd_floor_plain_vs_plain": round(res["floor_plain_T_vs_reference"], 4),
        "n_star_by_kind": res["n_star_by_kind"],
        "mmd": res["mmd"],
        "mean_mmd2_u": res["mean_mmd2_u"],
        "mmd_by_kind": res["mmd_by_kind"],
        "fallbacks": res["fallbacks"],
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": MFMA_BF16_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / MFMA_BF16_PEAK_TFLOPS, 4), "traffic": None,
                     "kernel": "proposal forward (all kernels)",
                     "flops_per_pair": 2 * PROPOSAL_MACS_PER_PAIR, "avg_ms_per_pair": round(net_ms / n, 5)},
    }
    if CEILINGS:
        out["roofline"]["measured_peak"] = {"value": round(CEILINGS["mfma_bf16_tflops"], 1), "unit": "TFLOP/s",
                                            "probe": "mfma_bf16_tflops",
                                            "frac": round(achieved / CEILINGS["mfma_bf16_tflops"], 4)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_proposal(ds, res, T)
    model.close()
    out["host"] = gpu_info(args.host)
    out["device_ceilings"] = args.ceilings
    print(json.dumps(out), flush=True)


def cpu_baseline_proposal(ds, res, T):
    """The oracles on this host's cores for the proposal form's job, timed on
    the first pair of each kind and scaled to the pairs of that kind: the
    FP64 proposal network (per-point layers on 2 x 4096 points, BF16-rounded
    operands) and n* iterations of the FP64 Stein-ICP oracle (at most 30
    timed, the rest extrapolated)."""
    import oracle
    from oracle import proposal_oracle as PO
    from paper_2106_03287_amd import train_proposal as TP
    weights = np.load(os.path.join(ROOT, "paper_2106_03287_amd", "weights", "proposal_k100_p4096.npy"),
                      allow_pickle=False)
    n_star = res["n_star"]["proposal"] if res["n_star"]["proposal"] is not None else T
    total_ms, parts = 0.0, []
    for kind in ("cuboid", "kinect"):
        ids = [i for i, k in enumerate(ds.kind) if k == kind]
        if not ids:
            continue
        i = ids[0]
        src, ref = ds.src[i].cpu().numpy(), ds.ref[i].cpu().numpy()
        clouds = np.stack([PO.subsample(src, 4096), PO.subsample(ref, 4096)])[None]
        t0 = time.perf_counter()
        theta0 = PO.forward(weights.astype(np.float64), clouds, 100, bf16=True)["Y"][0]
        net_s = time.perf_counter() - t0
        m = TP.MINIBATCH[kind]
        sched = np.stack([np.random.default_rng(1000 + t).choice(len(src), m, replace=False) for t in range(T)])
        cfg = oracle.make_config(100, m, len(src), len(ref), lr=0.01)
        st = oracle.State(theta0)
        n_run = min(n_star, 30)
        t0 = time.perf_counter()
        if n_run:
            oracle.run(cfg, src, ref, sched.astype(np.int32), n_run, st)
        it_s = (time.perf_counter() - t0) / max(n_run, 1)
        pair_ms = (net_s + it_s * n_star) * 1e3
        total_ms += pair_ms * len(ids)
        parts.append(f"{kind}: network {net_s * 1e3:.0f} ms + {n_star} iterations x {it_s * 1e3:.1f} ms "
                     f"({n_run} timed) per pair, x {len(ids)} pairs")
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(total_ms, 1), "unit": "ms", "cores": cores, "kind": "oracle",
            "sample": "FP64 oracles, first pair of each kind, scaled to all pairs: " + "; ".join(parts)}


if __name__ == "__main__":
    main()
