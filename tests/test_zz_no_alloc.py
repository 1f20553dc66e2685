"""The allocation-free Wishart entry point against polsar_wishart_loglik on
the GPU: the same kernels at the same launch, so loss, per-pixel terms and
gradient agree bit for bit; two calls in a row, the second on a smaller
image, each checked against the workspace entry point on the same inputs."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1807_08084_amd import _lib as L
from paper_1807_08084_amd import ops, synth

pytestmark = pytest.mark.gpu


def _inputs(h, w, dtype, seed):
    img = synth.make_image(h, w, 8, (2, 2), (1e-2, 1.0), seed)
    z = img.planes.reshape(9, -1)
    return (ops.upload_planes(synth.wishart_sigma0(z), dtype, "cuda"), ops.upload_planes(z, dtype, "cuda"))


def _call(fn, s, z, n_looks, extra):
    n = s.shape[1]
    dt = L.F32 if s.dtype == torch.float32 else L.F64
    loss = torch.full((), float("nan"), dtype=torch.float64, device="cuda")
    ell = torch.full((n,), float("nan"), dtype=s.dtype, device="cuda")
    grad = ops.empty_planes(9, n, s.dtype, "cuda")
    grad.fill_(float("nan"))
    ctr = torch.zeros(3, dtype=torch.int64, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = fn(dt, L.FWD_BWD, n, P(s), s.stride(0), P(z), z.stride(0), float(n_looks), P(loss), P(ell), None,
            P(grad), grad.stride(0), *extra, P(ctr), stream)
    assert rc == L.OK, L.status_string(rc)
    torch.cuda.synchronize()
    return loss.item(), ell.cpu().numpy(), grad.cpu().numpy(), ctr.cpu().numpy()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_matches_the_workspace_entry(dtype):
    lib = L.lib()
    # 1000 x 1001 (ragged tail after the last full vector), then 300 x 301;
    # 4100 x 4100 crosses into the launch entry of large images (op 1)
    for h, w, seed in ((1000, 1001, 11), (300, 301, 12), (4100, 4100, 13), (77, 5, 14)):
        s, z = _inputs(h, w, dtype, seed)
        n = s.shape[1]
        ws = torch.zeros(ops.workspace_bytes(dtype, n) // 8 + 1, dtype=torch.float64, device="cuda")
        ref = _call(lib.polsar_wishart_loglik, s, z, 8.0,
                    (ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel() * 8)))
        got = _call(lib.polsar_wishart_loglik_noalloc, s, z, 8.0, ())
        print(f"{h}x{w} {dtype}: loss {got[0]!r} vs {ref[0]!r}", flush=True)
        assert np.isfinite(ref[0])
        assert got[0] == ref[0]
        assert np.array_equal(got[1], ref[1])
        assert np.array_equal(got[2], ref[2])
        assert np.array_equal(got[3], ref[3])
