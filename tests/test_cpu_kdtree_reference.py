"""The fast CPU form that bench.py reports beside the oracle (cKDTree
nearest neighbours, NumPy FP64) computes the same iteration as the oracle:
same matches and particles on the cuboid workload, away from near-ties."""
import numpy as np

import oracle
import synth
from bench import KDTreeReference


def test_kdtree_reference_follows_the_oracle():
    prob = synth.make_problem("cuboid", 3, T=5)
    ref = KDTreeReference(prob)
    cfg = oracle.make_config(prob.K, prob.m, len(prob.pair.src), len(prob.pair.ref), lr=prob.lr)
    st = oracle.State(prob.theta0)
    for t in range(5):
        j = ref.step()
        od = oracle.step(cfg, prob.pair.src, prob.pair.ref, prob.schedule[t % len(prob.schedule)], st)
        np.testing.assert_array_equal(j.reshape(prob.K, prob.m), np.asarray(od["match"]).reshape(prob.K, prob.m))
        np.testing.assert_allclose(ref.theta, st.theta, rtol=0, atol=1e-10)
