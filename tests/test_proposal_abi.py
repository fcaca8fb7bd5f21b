"""Host-side checks of the proposal C ABI: exports match the header, the
config defaults and the parameter count, and argument validation that fails
before any device call. No kernel is launched."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import proposal_oracle as PO
from paper_2106_03287_amd import proposal as PR
from paper_2106_03287_amd import stein_icp as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "stein_icp_proposal.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stein_icp_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_proposal_symbol():
    L = PR.lib()
    declared = _declared()
    assert len(declared) == 15
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(PR.EXPORTS) == declared


def test_default_config_and_parameter_count():
    cfg = PR.stein_icp_proposal_default_config()
    assert cfg.struct_size == C.sizeof(PR.stein_icp_proposal_config)
    assert (cfg.num_particles, cfg.points, cfg.max_batch, cfg.n_loss_scales) == (100, 4096, 32, 4)
    sig = np.array([[cfg.loss_sigma[s][d] for d in range(6)] for s in range(4)])
    assert np.allclose(sig[:, :3], np.array([0.01, 0.04, 0.16, 0.64])[:, None])
    assert np.allclose(sig[:, 3:], np.array([0.02, 0.08, 0.32, 1.28])[:, None])
    for K in (1, 2, 100, 1024):
        assert PR.stein_icp_proposal_param_count(K) == PO.param_count(K)
    assert PR.stein_icp_proposal_param_count(100) == 327128
    with pytest.raises(S.SteinICPError):
        PR.stein_icp_proposal_param_count(0)
    with pytest.raises(S.SteinICPError):
        PR.stein_icp_proposal_param_count(1025)


@pytest.mark.parametrize("field,value,msg", [
    ("num_particles", 0, "num_particles"), ("num_particles", 1025, "num_particles"),
    ("points", 0, "points"), ("points", 4097, "points"),
    ("max_batch", 0, "max_batch"), ("max_batch", 5000, "max_batch"),
    ("n_loss_scales", 0, "n_loss_scales"), ("n_loss_scales", 5, "n_loss_scales"),
    ("struct_size", 8, "struct_size"),
])
def test_invalid_config_is_rejected_before_any_device_call(field, value, msg):
    cfg = PR.stein_icp_proposal_default_config()
    setattr(cfg, field, value)
    with pytest.raises(S.SteinICPError, match=msg):
        PR.stein_icp_proposal_create(cfg)


def test_invalid_loss_width_is_rejected():
    cfg = PR.stein_icp_proposal_default_config()
    cfg.loss_sigma[1][4] = 0.0
    with pytest.raises(S.SteinICPError, match="loss_sigma"):
        PR.stein_icp_proposal_create(cfg)
    cfg.loss_sigma[1][4] = float("nan")
    with pytest.raises(S.SteinICPError, match="loss_sigma"):
        PR.stein_icp_proposal_create(cfg)


def test_gemm_and_mmd_validate_their_arguments():
    L = PR.lib()
    fake = C.c_void_p(0x1000)   # never dereferenced: validation fails first
    # leading dimension shorter than the row
    rc = L.stein_icp_gemm_bf16(0, 0, 4, 4, 8, fake, 4, fake, 4, fake, 4, None, 0, 0, 1, None, None)
    assert rc == S.E_INVALID and b"leading dimension" in L.stein_icp_last_error()
    rc = L.stein_icp_gemm_bf16(2, 0, 4, 4, 8, fake, 8, fake, 4, fake, 4, None, 0, 0, 1, None, None)
    assert rc == S.E_INVALID
    rc = L.stein_icp_gemm_bf16(0, 0, 4, 4, 8, fake, 8, fake, 4, fake, 4, None, 0, 0, 4, None, None)
    assert rc == S.E_INVALID and b"workspace" in L.stein_icp_last_error()
    rc = L.stein_icp_gemm_bf16(0, 0, 4, 4, 8, fake, 8, fake, 4, fake, 4, None, 0, 0, 65, fake, None)
    assert rc == S.E_INVALID
    sig = np.zeros((1, 6))
    rc = L.stein_icp_proposal_mmd(fake, fake, 1, 4, 1, sig.ctypes.data_as(C.c_void_p), fake, None)
    assert rc == S.E_INVALID and b"sigma" in L.stein_icp_last_error()
    sig = np.ones((5, 6))
    rc = L.stein_icp_proposal_mmd(fake, fake, 1, 4, 5, sig.ctypes.data_as(C.c_void_p), fake, None)
    assert rc == S.E_INVALID
    rc = L.stein_icp_proposal_mmd(fake, fake, 1, 1025, 1, sig.ctypes.data_as(C.c_void_p), fake, None)
    assert rc == S.E_INVALID


def test_init_params_shape_and_scale():
    p = PR.init_params(100, seed=3)
    assert p.dtype == np.float32 and p.size == PO.param_count(100)
    blocks = PO.unpack(p, 100)
    assert np.all(blocks["b1"] == 0) and np.all(blocks["b5"] == 0)
    assert np.abs(blocks["W1"]).max() <= np.sqrt(6 / 3)
    assert np.abs(blocks["W5"]).max() <= 0.01 * np.sqrt(6 / 256)
    assert np.array_equal(p, PR.init_params(100, seed=3))


# ------------------------------------------------------------------ weight files
WEIGHTS = os.path.join(ROOT, "paper_2106_03287_amd", "weights", "proposal_k100_p4096.npy")


def test_committed_weights_read_back_through_the_library():
    got, K = PR.stein_icp_proposal_read_weights(WEIGHTS)
    want = np.load(WEIGHTS, allow_pickle=False)
    assert K == 100 and got.dtype == np.float32
    assert np.array_equal(got, want)
    assert len(got) == PO.param_count(100)


@pytest.mark.parametrize("K", [1, 3, 1024])
def test_weight_files_written_by_numpy_give_their_particle_count(tmp_path, K):
    params = np.random.default_rng(K).standard_normal(PO.param_count(K)).astype(np.float32)
    path = tmp_path / f"w{K}.npy"
    np.save(path, params)
    got, k = PR.stein_icp_proposal_read_weights(str(path))
    assert k == K and np.array_equal(got, params)


def _bad(tmp_path, name, data):
    path = tmp_path / name
    path.write_bytes(data)
    with pytest.raises(S.SteinICPError) as e:
        PR.stein_icp_proposal_read_weights(str(path))
    assert e.value.code == S.E_INVALID
    return str(e.value)


def test_malformed_weight_files_are_rejected(tmp_path):
    good = open(WEIGHTS, "rb").read()
    assert "not a .npy" in _bad(tmp_path, "magic", b"XNUMPY" + good[6:])
    assert "truncated" in _bad(tmp_path, "short", good[:-4])
    f8 = tmp_path / "f8.npy"
    np.save(f8, np.zeros(PO.param_count(2), dtype=np.float64))
    assert "<f4" in _bad(tmp_path, "f8b.npy", f8.read_bytes())
    m2 = tmp_path / "m2.npy"
    np.save(m2, np.zeros((2, PO.param_count(2) // 2), dtype=np.float32))
    assert "one-dimensional" in _bad(tmp_path, "m2b.npy", m2.read_bytes())
    odd = tmp_path / "odd.npy"
    np.save(odd, np.zeros(PO.param_count(2) + 1, dtype=np.float32))
    assert "no particle count" in _bad(tmp_path, "oddb.npy", odd.read_bytes())
    nan = np.zeros(PO.param_count(1), dtype=np.float32)
    nan[5] = np.nan
    nf = tmp_path / "nan.npy"
    np.save(nf, nan)
    assert "not finite" in _bad(tmp_path, "nanb.npy", nf.read_bytes())
    with pytest.raises(S.SteinICPError):
        PR.stein_icp_proposal_read_weights(str(tmp_path / "missing.npy"))
