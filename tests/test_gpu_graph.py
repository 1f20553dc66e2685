"""The per-call entry points allocate nothing when given their outputs and
workspace, so a caller can capture them in a HIP graph: replays (with eager
work and synchronisation between them) must repeat the eager results."""
import numpy as np
import pytest
import torch

from paper_1807_08084_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_08084_amd import ops as o
    o.compute_units()
    return o


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_captured_inverse_and_wishart_replay(ops, dtype):
    img, sig = synth.workload_wishart(seed=3, side=256)
    z = ops.upload_planes(img.planes.reshape(9, -1), dtype)
    s = ops.upload_planes(sig.reshape(9, -1), dtype)
    n = z.shape[1]
    out = ops.empty_planes(10, n, dtype)
    inv, det = out[:9], out[9]
    st = torch.empty(n, dtype=torch.uint8, device="cuda")
    ws = torch.empty(ops.workspace_bytes(dtype, n) // 8 + 1, dtype=torch.float64, device="cuda")
    # eager reference
    inv_e, det_e, st_e = ops.inv_det(z, "adjugate", "compensated", status=True)
    loss_e, grad_e, _ = ops.wishart_loglik(s, z, 8.0, forward=True, backward=True, workspace=ws)
    torch.cuda.synchronize()
    inv_e, det_e, st_e, loss_e, grad_e = (t.clone() for t in (inv_e, det_e, st_e, loss_e, grad_e))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm the binding on the capture stream
        ops.inv_det(z, "adjugate", "compensated", inv=inv, det=det, status=st)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ops.inv_det(z, "adjugate", "compensated", inv=inv, det=det, status=st)
        loss, grad, _ = ops.wishart_loglik(s, z, 8.0, forward=True, backward=True, workspace=ws)
    for rep in range(4):
        inv.zero_()
        det.zero_()
        grad.zero_()
        loss.zero_()
        junk = torch.randn(1 << 18, device="cuda").sum()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        assert torch.equal(inv, inv_e) and torch.equal(det, det_e) and torch.equal(st, st_e), rep
        assert torch.equal(loss, loss_e) and torch.equal(grad, grad_e), rep
