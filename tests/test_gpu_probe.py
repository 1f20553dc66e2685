"""The bandwidth probe (polsar_stream_copy) on the GPU: every output plane
equals its input plane, or, with fewer outputs than inputs, the FP32/FP64 sum
of the input planes j with j mod n_out == k, added in ascending j; ragged n
exercises the one-element tail."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_08084_amd import ops as o
    o.compute_units()
    return o


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("n_in,n_out", [(9, 10), (18, 9), (18, 19), (24, 10), (27, 28), (1, 1)])
@pytest.mark.parametrize("n", [1000, 1027])
def test_copy_probe(ops, dtype, n_in, n_out, n):
    rng = np.random.default_rng(n_in * 100 + n_out)
    npdt = np.float32 if dtype == torch.float32 else np.float64
    src_np = rng.standard_normal((n_in, n)).astype(npdt)
    src = ops.upload_planes(src_np, dtype)
    dst = ops.empty_planes(n_out, n, dtype)
    ops.stream_copy(src, dst, n_in, n_out, n)
    torch.cuda.synchronize()
    got = dst.cpu().numpy()
    for k in range(n_out):
        want = src_np[k % n_in].copy()
        for j in range(k + n_out, n_in, n_out):
            want = (want + src_np[j]).astype(npdt)
        assert np.array_equal(got[k], want), (k, n_in, n_out)
