"""Seeded synthetic inputs for Stein ICP: point-cloud pairs, initial particle
sets and minibatch schedules.

This package is the only code shared by the FP64 oracle checks and the HIP
path. It holds none of the method's arithmetic: it draws random numbers and
builds scenes. Rigid transforms used to create a source cloud come from
``scipy.spatial.transform.Rotation``, never from the oracle or the library.
"""
from .clouds import (  # noqa: F401
    Pair,
    cuboid_pair,
    kinect_pair,
    lidar_pair,
    resample_pair,
    init_particles,
    minibatch_schedule,
    rng_streams,
)
from .workloads import (  # noqa: F401
    MC_HALF_ROT,
    MC_HALF_TRANS,
    MC_SEED,
    WORKLOADS,
    MonteCarlo,
    Problem,
    batched_problems,
    make_problem,
    mc_problem,
)
