"""Host-side checks of the C ABI: the library loads and exports every declared
symbol, argument validation happens before any device call, and the host
generators behave. None of these launch a kernel."""
import ctypes as C
import json
import os
import re

import numpy as np
import pytest

from paper_2106_03287_amd import stein_icp as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "stein_icp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stein_icp_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = S.lib()
    declared = _declared_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(S.EXPORTS) == declared


def test_config_layout_and_defaults_follow_the_paper():
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_hyperparameters.json")))
    cfg = S.stein_icp_default_config()
    assert cfg.struct_size == C.sizeof(S.stein_icp_config)
    assert cfg.num_particles == gold["particles"]["value"]
    assert cfg.lr == gold["adam_step_lidar"]["value"]
    assert cfg.batch_size == gold["batch_lidar"]["value"]
    assert (cfg.beta1, cfg.beta2, cfg.eps) == (0.9, 0.999, 1e-8)
    assert cfg.bandwidth_mode == S.BW_MEDIAN and cfg.prior_mode == S.PRIOR_UNIFORM
    assert cfg.optimizer == S.OPT_ADAM and cfg.nn_mode == S.NN_FP32
    assert cfg.metric == S.METRIC_POINT and cfg.normal_k == 10


def _init_rc(cfg, n_src=100, n_ref=100, src=1, ref=1):
    ctx = C.c_void_p()
    rc = S.lib().stein_icp_init(C.byref(ctx), C.byref(cfg) if cfg is not None else None,
                                C.c_void_p(src), n_src, C.c_void_p(ref), n_ref, None, None, None)
    return rc, S.stein_icp_last_error()


@pytest.mark.parametrize("field,value,msg", [
    ("num_particles", 0, "num_particles"),
    ("num_particles", 1025, "num_particles"),
    ("batch_size", 0, "batch_size"),
    ("schedule_rows", 0, "schedule_rows"),
    ("lr", float("nan"), "lr"),
    ("lr", -1.0, "lr"),
    ("beta1", 1.0, "beta1"),
    ("eps", 0.0, "eps"),
    ("nn_mode", 7, "nn_mode"),
    ("optimizer", 5, "optimizer"),
    ("bandwidth_mode", 3, "bandwidth_mode"),
    ("prior_mode", 9, "prior_mode"),
    ("n_scale", -5, "n_scale"),
    ("use_graph", 2, "use_graph"),
    ("init_half_rot", float("inf"), "half"),
    ("metric", 2, "metric"),
    ("normal_k", 2, "normal_k"),
    ("normal_k", 33, "normal_k"),
])
def test_invalid_config_is_rejected_before_any_device_call(field, value, msg):
    cfg = S.stein_icp_default_config(batch_size=10)
    setattr(cfg, field, value)
    rc, err = _init_rc(cfg)
    assert rc == S.E_INVALID
    assert msg in err


def test_invalid_arguments_are_rejected():
    assert _init_rc(None)[0] == S.E_INVALID
    cfg = S.stein_icp_default_config(batch_size=10)
    cfg.struct_size = 8
    assert "struct_size" in _init_rc(cfg)[1]
    cfg = S.stein_icp_default_config(batch_size=200)
    rc, err = _init_rc(cfg, n_src=100)
    assert rc == S.E_INVALID and "batch_size" in err
    cfg = S.stein_icp_default_config(batch_size=10)
    assert _init_rc(cfg, src=0)[0] == S.E_INVALID
    assert _init_rc(cfg, n_ref=0)[0] == S.E_INVALID
    cfg = S.stein_icp_default_config(batch_size=10, bandwidth_mode=S.BW_FIXED, fixed_h_trans=0.0)
    assert _init_rc(cfg)[0] == S.E_INVALID
    cfg = S.stein_icp_default_config(batch_size=10, prior_mode=S.PRIOR_GAUSS_VONMISES,
                                     prior_var_trans=[1.0, 0.0, 1.0])
    assert _init_rc(cfg)[0] == S.E_INVALID
    assert S.lib().stein_icp_step(None, 1, None) == S.E_INVALID
    assert S.lib().stein_icp_particles(None, None, None) == S.E_INVALID
    assert S.lib().stein_icp_nn(None, 1, None, 1, 0, None, None, None) == S.E_INVALID
    fake = C.c_void_p(0x1000)   # never dereferenced: validation fails first
    for k in (0, 33):
        assert S.lib().stein_icp_knn(fake, 4, fake, 4, k, fake, fake, None) == S.E_INVALID
        assert "k must be" in S.stein_icp_last_error()
    assert S.lib().stein_icp_knn(fake, 4, fake, 4, 4, fake, None, None) == S.E_INVALID
    assert S.lib().stein_icp_knn(fake, 4, fake, 0, 4, fake, fake, None) == S.E_INVALID
    assert S.lib().stein_icp_knn(fake, 0, fake, 4, 4, fake, fake, None) == S.OK   # nothing to do
    for k in (2, 33):
        assert S.lib().stein_icp_normals(fake, 10, k, fake, None, None) == S.E_INVALID
    assert S.lib().stein_icp_normals(fake, 0, 10, fake, None, None) == S.E_INVALID
    assert S.lib().stein_icp_normals(fake, 10, 10, None, None, None) == S.E_INVALID
    assert S.lib().stein_icp_get_normals(None, fake, None) == S.E_INVALID
    S.lib().stein_icp_destroy(None)


def test_batch_init_validation():
    cfg = S.stein_icp_default_config(batch_size=10)
    ctx = C.c_void_p()
    rc = S.lib().stein_icp_batch_init(C.byref(ctx), C.byref(cfg), 0, None, None, None, None,
                                      None, None, None)
    assert rc == S.E_INVALID and "n_pairs" in S.stein_icp_last_error()


def test_library_schedule_rows_are_distinct_in_range_and_seeded():
    a = S.stein_icp_make_schedule(7, 1000, 300, 50)
    b = S.stein_icp_make_schedule(7, 1000, 300, 50)
    c = S.stein_icp_make_schedule(8, 1000, 300, 50)
    np.testing.assert_array_equal(a, b)
    assert not np.array_equal(a, c)
    assert a.min() >= 0 and a.max() < 1000
    for row in a:
        assert len(np.unique(row)) == 300
    # m == n is a permutation; every index is drawn about equally often
    full = S.stein_icp_make_schedule(1, 20, 20, 3)
    for row in full:
        assert sorted(row) == list(range(20))
    big = S.stein_icp_make_schedule(3, 100, 10, 20000)
    counts = np.bincount(big.ravel(), minlength=100)
    expected = big.size / 100
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert chi2 < 160  # 99 dof: mean 99, sd 14


def test_library_initial_particles_are_uniform_in_the_box():
    x = S.stein_icp_make_init(5, 4000, 0.2, np.pi / 4, [0.1, 0, 0, 0, 0, 1.0])
    assert x.shape == (4000, 6)
    lo = np.array([-0.1, -0.2, -0.2, -np.pi / 4, -np.pi / 4, 1 - np.pi / 4])
    hi = np.array([0.3, 0.2, 0.2, np.pi / 4, np.pi / 4, 1 + np.pi / 4])
    assert np.all(x >= lo) and np.all(x < hi)
    np.testing.assert_allclose(x.mean(0), (lo + hi) / 2, atol=0.03)
    np.testing.assert_array_equal(x, S.stein_icp_make_init(5, 4000, 0.2, np.pi / 4,
                                                            [0.1, 0, 0, 0, 0, 1.0]))
    with pytest.raises(S.SteinICPError):
        S.stein_icp_make_init(5, 0, 0.2, 0.1)
    with pytest.raises(S.SteinICPError):
        S.stein_icp_make_schedule(5, 10, 11, 1)


def test_peak_probes_are_exported_and_validate_before_launching():
    from paper_2106_03287_amd import peaks as P
    text = open(os.path.join(ROOT, "include", "stein_icp_peaks.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    declared = sorted(set(re.findall(r"\b(stein_icp_[a-z_0-9]+)\s*\(", text)))
    L = P.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(P.EXPORTS) == declared
    fake = C.c_void_p(16)   # never dereferenced: every case fails validation
    for kind, n, iters in ((7, 256, 1), (-1, 256, 1), (P.PEAK_COPY, 0, 1), (P.PEAK_FMA32, 100, 1),
                           (P.PEAK_MFMA_F16, 256, 0), (P.PEAK_MFMA_BF16, 256, (1 << 24) + 1)):
        assert L.stein_icp_peak_probe(kind, fake, fake, n, iters, 1.0, 1.0, None) == S.E_INVALID
    assert L.stein_icp_peak_probe(P.PEAK_COPY, None, fake, 16, 1, 1.0, 1.0, None) == S.E_INVALID
    assert P.peak_work(P.PEAK_COPY, 1000) == 32000.0
    assert P.peak_work(P.PEAK_FMA32, 256, 10) == 2 * 16 * 256 * 10
    assert P.peak_work(P.PEAK_MFMA_F16, 256, 3) == 4 * 4 * 2 * 32 * 32 * 16 * 3
    assert P.peak_work(9, 1, 1) < 0
