"""Named workloads: a cloud pair, its initial particles, its minibatch schedule
and the hyper-parameters it is run with.

Sizes follow the five benchmark configurations of the project:
cuboid (N 500, M 2,000, K 100, m 100, T 50), Kinect-shaped tabletop
(N = M = 20,000, K 100, m 300, T 200), LiDAR-shaped street (N 20,000,
M 100,000, K 300, m 1,000, T 300) and the batched set of 64 uneven pairs
(K 100, m 300, T 150). Seeds: workload c, pair p uses 1_000_000 * c + p.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .clouds import (Pair, cuboid_pair, init_particles, kinect_pair, lidar_pair,
                     minibatch_schedule, resample_pair, rng_streams)

WORKLOADS = {
    "cuboid": dict(index=1, K=100, m=100, T=50, lr=0.01, half_trans=0.2, half_rot=np.pi / 4),
    "kinect": dict(index=2, K=100, m=300, T=200, lr=0.01, half_trans=0.2, half_rot=np.pi / 4),
    "lidar": dict(index=3, K=300, m=1000, T=300, lr=0.01, half_trans=0.2, half_rot=np.pi / 4),
    "batched": dict(index=4, K=100, m=300, T=150, lr=0.01, half_trans=0.2, half_rot=np.pi / 4),
}


@dataclass
class Problem:
    name: str
    pair: Pair
    theta0: np.ndarray        # float64 (K, 6)
    schedule: np.ndarray      # int32 (T, m)
    K: int
    m: int
    T: int
    lr: float
    seed: int
    extra: dict = field(default_factory=dict)


def _generate(name: str, seed: int) -> Pair:
    if name == "cuboid":
        return cuboid_pair(seed)
    if name == "kinect":
        return kinect_pair(seed)
    if name == "lidar":
        return lidar_pair(seed)
    raise KeyError(name)


def make_problem(name: str, pair_index: int = 0, *, K=None, m=None, T=None,
                 pair: Pair | None = None) -> Problem:
    """Build workload ``name`` with its seeded pair, initial particles and
    schedule. ``K``, ``m``, ``T`` override the defaults (for small tests)."""
    w = WORKLOADS[name]
    seed = 1_000_000 * w["index"] + pair_index
    pair = pair if pair is not None else _generate(name, seed)
    K = w["K"] if K is None else K
    m = w["m"] if m is None else m
    T = w["T"] if T is None else T
    centre = None
    if name == "lidar":
        # coarse guess around the true pose, standing in for an IMU or a
        # previous solution: +-0.1 m and +-2 deg
        _, rng, _ = rng_streams(seed + 7)
        centre = pair.theta_true + np.concatenate(
            [rng.uniform(-0.1, 0.1, 3), np.deg2rad(rng.uniform(-2.0, 2.0, 3))])
    theta0 = init_particles(seed, K, w["half_trans"], w["half_rot"], centre)
    sched = minibatch_schedule(seed, len(pair.src), m, T)
    return Problem(name, pair, theta0, sched, K, m, T, w["lr"], seed,
                   {"centre": centre})


def batched_problems(n_pairs: int = 64, *, K=None, m=None, T=None,
                     size_scale: float = 1.0) -> list[Problem]:
    """Batched workload: pairs alternate the cuboid and Kinect generators and
    are resampled to reference sizes log-uniform in [2,000, 50,000] and source
    sizes log-uniform in [1,000, 20,000] (``size_scale`` shrinks both for
    small tests)."""
    w = WORKLOADS["batched"]
    K = w["K"] if K is None else K
    m = w["m"] if m is None else m
    T = w["T"] if T is None else T
    out = []
    for p in range(n_pairs):
        seed = 1_000_000 * w["index"] + p
        rng, _, _ = rng_streams(seed)
        n_ref = int(round(np.exp(rng.uniform(np.log(2000), np.log(50000))) * size_scale))
        n_src = int(round(np.exp(rng.uniform(np.log(1000), np.log(20000))) * size_scale))
        n_ref, n_src = max(n_ref, 8), max(n_src, m)
        base = cuboid_pair(seed, n_src=n_src, n_ref=n_ref) if p % 2 == 0 else kinect_pair(seed)
        pair = resample_pair(base, rng, n_src, n_ref)
        theta0 = init_particles(seed, K, w["half_trans"], w["half_rot"])
        sched = minibatch_schedule(seed, n_src, m, T)
        out.append(Problem("batched", pair, theta0, sched, K, m, T, w["lr"], seed,
                           {"pair_index": p}))
    return out


# ---------------------------------------------------------------------------
# learned-proposal data: fresh seeded pairs of the cuboid and Kinect shapes
# ---------------------------------------------------------------------------

PROPOSAL_TRAIN_SEED = 5_000_000
PROPOSAL_TEST_SEED = 6_000_000


def proposal_pair_spec(split: str, i: int) -> tuple[str, int]:
    """(generator, seed) of pair i of the proposal's training or test split:
    even i cuboid, odd i Kinect-shaped, seeds disjoint from the benchmark
    workloads and between the splits."""
    base = {"train": PROPOSAL_TRAIN_SEED, "test": PROPOSAL_TEST_SEED}[split]
    return ("cuboid" if i % 2 == 0 else "kinect"), base + i


def generate_pair(spec: tuple[str, int]) -> tuple[str, int, Pair]:
    """Build one pair from a (generator, seed) spec (picklable, for worker
    processes)."""
    kind, seed = spec
    return kind, seed, _generate(kind, seed)


# ---------------------------------------------------------------------------
# Monte-Carlo ground truth: independent single-particle runs on one pair
# ---------------------------------------------------------------------------

MC_SEED = 7_000_000
MC_HALF_TRANS, MC_HALF_ROT = 1.0, 0.1745   # start box of the paper's Monte-Carlo runs (m, rad)


@dataclass
class MonteCarlo:
    problem: Problem          # the workload's Stein-ICP problem on the same pair
    runs: int
    theta0: np.ndarray        # float64 (runs, 1, 6)
    schedules: np.ndarray     # int32 (runs, T, m), one fresh stream per run


def mc_problem(name: str, pair_index: int = 0, runs: int = 1000, *, K=None, m=None, T=None,
               half_trans: float = MC_HALF_TRANS, half_rot: float = MC_HALF_ROT,
               pair: Pair | None = None) -> MonteCarlo:
    """``runs`` independent starts and minibatch streams for single-particle
    runs on workload ``name``'s pair, uniform in the workload's init centre
    +- (half_trans, half_rot). Run r uses seed MC_SEED + 100_000 c + r for
    workload index c."""
    prob = make_problem(name, pair_index, K=K, m=m, T=T, pair=pair)
    centre = prob.extra["centre"]
    base = MC_SEED + 100_000 * WORKLOADS[name]["index"]
    theta0 = np.stack([init_particles(base + r, 1, half_trans, half_rot, centre) for r in range(runs)])
    scheds = np.stack([minibatch_schedule(base + r, len(prob.pair.src), prob.m, prob.T) for r in range(runs)])
    return MonteCarlo(prob, runs, theta0, scheds)
