"""The allocation-free nearest-neighbour entry point against the allocating
one, through the C ABI: two calls in a row on the same GPU (the second with
a smaller input, so it runs on the first call's leftover scratch), each
bit-exact against stein_icp_nn in both search modes; a search larger than
the scratch is refused before anything is launched."""
import numpy as np
import pytest
import torch

from paper_2106_03287_amd import stein_icp as S

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _cloud(seed, nq, M, scale, centre):
    rng = np.random.default_rng(seed)
    ref = centre + rng.uniform(-scale, scale, (M, 3))
    q = ref[rng.integers(0, M, nq)] + rng.normal(0, 0.01 * scale, (nq, 3))
    q[: nq // 10] = ref[rng.integers(0, M, nq // 10)]          # exact hits
    return q.astype(np.float32), ref.astype(np.float32)


@pytest.mark.parametrize("mode", [S.NN_FP32, S.NN_BF16_RERANK, S.NN_F16_RERANK])
def test_noalloc_search_equals_the_allocating_search_on_two_calls(mode):
    cases = [_cloud(1, 30000, 20011, 0.5, np.array([0.3, -0.2, 1.0])),    # larger first
             _cloud(2, 777, 1000, 20.0, np.array([40.0, 5.0, -3.0]))]     # then smaller
    idx_out = torch.full((30000,), -7, dtype=torch.int32, device="cuda")
    d2_out = torch.full((30000,), -7.0, dtype=torch.float32, device="cuda")
    for c, (q, ref) in enumerate(cases):
        n = len(q)
        print(f"noalloc mode={mode} call {c}: nq={n} M={len(ref)}", flush=True)
        qd, rd = dev(q), dev(ref)
        want_i, want_d = S.stein_icp_nn(qd, rd, mode=mode)
        got_i, got_d = S.stein_icp_nn_noalloc(qd, rd, mode=mode, idx=idx_out[:n], d2=d2_out[:n])
        torch.cuda.synchronize()
        assert torch.equal(got_i, want_i)
        assert torch.equal(got_d.view(torch.int32), want_d.view(torch.int32))
    # the entries past the second call's queries were not written by it
    assert torch.equal(idx_out[777:], S.stein_icp_nn(dev(cases[0][0]), dev(cases[0][1]), mode=mode)[0][777:])


def test_noalloc_search_refuses_a_search_beyond_its_scratch():
    q = torch.zeros((2_500_000, 3), dtype=torch.float32, device="cuda")
    ref = torch.zeros((100_000, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(S.SteinICPError) as e:
        S.stein_icp_nn_noalloc(q, ref)
    assert e.value.code == S.E_INVALID and "32 MiB" in str(e.value)
