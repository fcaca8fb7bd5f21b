"""The device-ceiling probes (include/stein_icp_peaks.h) compute what they
state, so their times measure the work they claim: the copy copies, the FMA
chains and the matrix-core loops give the exact sums of their recurrences."""
import numpy as np
import pytest
import torch

from paper_2106_03287_amd import peaks as P

pytestmark = pytest.mark.gpu


def test_copy_probe_copies():
    n4 = 300_001
    a = torch.randn(n4 * 4, device="cuda")
    b = torch.zeros_like(a)
    P.peak_probe(P.PEAK_COPY, a, b, n4)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_fma_probe_runs_its_chains():
    n, iters = 1024, 777
    out = torch.zeros(n, dtype=torch.float32, device="cuda")
    P.peak_probe(P.PEAK_FMA32, None, out, n, iters, 1.0, 1.0)
    torch.cuda.synchronize()
    gid = np.arange(n, dtype=np.float64)
    want = 16 * gid + 120 + 16 * iters   # chains a_k = gid + k, each + iters
    np.testing.assert_array_equal(out.cpu().numpy(), want.astype(np.float32))


@pytest.mark.parametrize("kind,one", [(P.PEAK_MFMA_F16, 0x3C00), (P.PEAK_MFMA_BF16, 0x3F80)])
def test_mfma_probe_accumulates(kind, one):
    n, iters = 512, 100
    frag = torch.full((512,), one | (one << 16), dtype=torch.int32, device="cuda")
    out = torch.zeros(n, dtype=torch.float32, device="cuda")
    P.peak_probe(kind, frag, out, n, iters)
    torch.cuda.synchronize()
    # every product of ones over K = 16 adds 16 to each of the lane's 16
    # values of each of its four tiles
    np.testing.assert_array_equal(out.cpu().numpy(), np.full(n, 4 * 16 * 16 * iters, np.float32))


def test_measured_ceilings_are_plausible():
    m = P.measure(copy_mib=64, reps=2)
    print(m, flush=True)
    assert m["device"]["compute_units"] > 0 and m["device"]["wave_size"] == 64
    for key in ("hbm_copy_gbps", "fp32_fma_tflops", "mfma_f16_tflops", "mfma_bf16_tflops"):
        assert np.isfinite(m[key]) and m[key] > 0, key
