"""Batched launch over many images (one HIP graph) against the per-image calls and
the oracle: images of uneven sizes with 2x4 regions, lam in [1e-2, 1], N in
{3, 4, 8, 16} (the first images of the 64-image recipe, seed 7, plus ragged
odd-sized images)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1807_08084_amd import synth
from _helpers import to_np, tol_f32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_08084_amd import ops as o
    o.compute_units()
    return o


def same_loss(ops, dtype, a, b, n):
    """Bitwise when the batch cuts tiles like the per-call Wishart kernel on
    an image of n pixels, else equal to rounding of the FP64 sums."""
    w = ops.get_launch(ops.wishart_launch_op(n), dtype, "adjugate", "plain")
    bt = ops.get_launch(3, dtype, "adjugate", "compensated")
    if (w["block"], w["vector_bytes"], w["unroll"]) == (bt["block"], bt["vector_bytes"], 1):
        return a == b
    return abs(a - b) <= 1e-12 * abs(b)


def _images(dtype):
    imgs = synth.workload_batch(max_images=6)
    extra = [synth.make_image(37, 41, 3, (2, 4), (1e-2, 1.0), 99),   # odd size: scalar tail
             synth.make_image(5, 3, 16, (1, 1), (1e-2, 1.0), 98)]
    out = []
    for im in imgs + extra:
        z = im.planes.reshape(9, im.planes.shape[1], im.planes.shape[2])
        s = synth.wishart_sigma0(z.reshape(9, -1)).reshape(z.shape)
        out.append({"z": torch.from_numpy(z).to("cuda", dtype), "sigma": torch.from_numpy(s).to("cuda", dtype),
                    "n_looks": float(im.n_looks)})
    return out


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_batch_graph_equals_per_image_calls(ops, dtype):
    from paper_1807_08084_amd.batch import BatchPlan
    imgs = _images(dtype)
    ctr = torch.zeros(3, dtype=torch.int64, device="cuda")
    plan = BatchPlan(imgs, "adjugate", "compensated", ell=True, counters=ctr)
    assert plan.tiles > len(imgs)
    plan.run()
    torch.cuda.synchronize()
    ctr_loop = torch.zeros(3, dtype=torch.int64, device="cuda")
    for i, im in enumerate(imgs):
        inv, det, st = ops.inv_det(im["z"], "adjugate", "compensated", status=True, counters=ctr_loop)
        loss, grad, ell = ops.wishart_loglik(im["sigma"], im["z"], im["n_looks"], forward=True, backward=True,
                                             ell=True)
        torch.cuda.synchronize()
        assert torch.equal(plan.inv[i], inv) and torch.equal(plan.det[i], det) and torch.equal(plan.status[i], st)
        assert torch.equal(plan.grad[i], grad) and torch.equal(plan.ell[i], ell)
        assert same_loss(ops, dtype, plan.loss[i].item(), loss.item(), im["z"][0].numel())
    assert torch.equal(ctr, ctr_loop)
    plan.close()


def test_batch_vs_oracle_and_replays(ops):
    from paper_1807_08084_amd.batch import BatchPlan
    imgs = _images(torch.float32)
    plan = BatchPlan(imgs, "adjugate", "compensated")
    plan.run()
    torch.cuda.synchronize()
    first = [(plan.inv[i].clone(), plan.grad[i].clone()) for i in range(len(imgs))]
    loss0 = plan.loss.clone()
    for i, im in enumerate(imgs):
        z = im["z"].reshape(9, -1).double().cpu().numpy()
        s = im["sigma"].reshape(9, -1).double().cpu().numpy()
        inv_o, det_o = oracle.ge(z)
        k = oracle.kappa(z)
        e = oracle.inv_rel_err(to_np(plan.inv[i]).reshape(9, -1), inv_o)
        assert np.all(e <= tol_f32(k))
        ell_o, _ = oracle.wishart(s, z, im["n_looks"], grad=False)
        assert abs(plan.loss[i].item() - math.fsum(ell_o)) <= 1e-5 * abs(math.fsum(ell_o)) + 1e-3
    # replays, with eager work and synchronisation in between, repeat the result
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda").sum()
        plan.inv[0].zero_()
        plan.loss.zero_()
        torch.cuda.synchronize()
        plan.run()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for i in range(len(imgs)):
            assert torch.equal(plan.inv[i], first[i][0]) and torch.equal(plan.grad[i], first[i][1])
        assert torch.equal(plan.loss, loss0)
    plan.run_eager()
    torch.cuda.synchronize()
    assert torch.equal(plan.loss, loss0)
    plan.close()


def test_batch_inv_only_and_cholesky(ops):
    from paper_1807_08084_amd.batch import BatchPlan
    imgs = _images(torch.float64)
    plan = BatchPlan(imgs, "cholesky", "plain", wishart_fwd=False, wishart_bwd=False)
    plan.run()
    torch.cuda.synchronize()
    for i, im in enumerate(imgs):
        inv, det, st = ops.inv_det(im["z"], "cholesky", "plain", status=True)
        assert torch.equal(plan.inv[i], inv) and torch.equal(plan.det[i], det) and torch.equal(plan.status[i], st)
    plan.close()


def test_batch_grid_kinds_agree(ops):
    """One block per tile (the FP32 default) and a persistent grid give the
    same bits: every output, and the losses (partial sums are per tile)."""
    from paper_1807_08084_amd.batch import BatchPlan
    imgs = _images(torch.float32)
    assert ops.get_launch(3, torch.float32, "adjugate", "compensated")["grid_per_cu"] == 0
    a = BatchPlan(imgs, "adjugate", "compensated", ell=True)
    b = BatchPlan(imgs, "adjugate", "compensated", ell=True, grid_per_cu=2)
    a.run()
    b.run()
    torch.cuda.synchronize()
    for i in range(len(imgs)):
        for x, y in ((a.inv, b.inv), (a.det, b.det), (a.status, b.status), (a.grad, b.grad), (a.ell, b.ell)):
            assert torch.equal(x[i], y[i])
    assert torch.equal(a.loss, b.loss)
    a.close()
    b.close()
