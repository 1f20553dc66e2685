"""Launch autotuners on small inputs: the winner is a valid configuration,
is installed, leaves results bitwise unchanged, and survives a JSON
save/load round trip (the small recipe, 256x256, seed 0)."""
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


def _space_ok(cfg):
    return (cfg["block"] in (64, 128, 256) and cfg["unroll"] in (1, 2) and cfg["grid_per_cu"] in (0, 8)
            and cfg["nontemporal"] == 1 and cfg["vector_bytes"] in (16, 8)
            and cfg["blocks_per_cu"] in (0, 2, 3, 4, 5, 6, 8))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_autotune_inv_det(ops, dtype):
    z = torch.from_numpy(synth.workload_small().planes.reshape(9, -1)).to("cuda", dtype)
    keep = ops.get_launch(0, dtype, "adjugate", "compensated")
    inv0, det0, st0 = ops.inv_det(z, "adjugate", "compensated", status=True)
    try:
        cfg, ms = ops.autotune_inv_det(z, "adjugate", "compensated", reps=2)
        assert _space_ok(cfg) and ms > 0
        assert ops.get_launch(0, dtype, "adjugate", "compensated") == cfg
        inv, det, st = ops.inv_det(z, "adjugate", "compensated", status=True)
        torch.cuda.synchronize()
        assert torch.equal(inv, inv0) and torch.equal(det, det0) and torch.equal(st, st0)
    finally:
        ops.set_launch(0, dtype, "adjugate", "compensated", keep)


def test_tune_wishart_and_json_round_trip(ops, tmp_path):
    from paper_1807_08084_amd import tune
    img = synth.workload_small()
    z = torch.from_numpy(img.planes.reshape(9, -1)).to("cuda", torch.float32)
    s = torch.from_numpy(synth.wishart_sigma0(img.planes.reshape(9, -1))).to("cuda", torch.float32)
    op = ops.wishart_launch_op(z.shape[1])
    assert op == 5  # a 256x256 image is a small one
    keep = ops.get_launch(op, torch.float32, "adjugate", "plain")
    loss0, grad0, _ = ops.wishart_loglik(s, z, 4.0, forward=True, backward=True)
    try:
        cfg, ms = tune.tune_wishart(s, z, 4.0, reps=2)
        assert ms > 0 and ops.get_launch(op, torch.float32, "adjugate", "plain") == cfg
        loss, grad, _ = ops.wishart_loglik(s, z, 4.0, forward=True, backward=True)
        torch.cuda.synchronize()
        assert torch.equal(grad, grad0)
        assert abs(loss.item() - loss0.item()) <= 1e-12 * abs(loss0.item())
        path = str(tmp_path / "launch.json")
        tune.save(path, {"wishart_small/f32/adjugate/plain": {"cfg": cfg, "ms": ms}})
        ops.set_launch(op, torch.float32, "adjugate", "plain", keep)
        assert tune.load(path) == 1
        assert ops.get_launch(op, torch.float32, "adjugate", "plain") == cfg
    finally:
        ops.set_launch(op, torch.float32, "adjugate", "plain", keep)


def test_tune_batch_installs_a_valid_launch(ops):
    """The batch tuner's pick is installed as the op-3 entry (so it passed
    the launch checks), and a plan built on it gives the per-image calls'
    results bit for bit (the first three images of the 64-image recipe)."""
    from paper_1807_08084_amd import tune
    from paper_1807_08084_amd.batch import BatchPlan
    items = []
    for im in synth.workload_batch(max_images=3):
        z = im.planes.reshape(9, -1)
        items.append({"z": torch.from_numpy(z).to("cuda", torch.float32),
                      "sigma": torch.from_numpy(synth.wishart_sigma0(z)).to("cuda", torch.float32),
                      "n_looks": float(im.n_looks)})
    keep = ops.get_launch(3, torch.float32, "adjugate", "compensated")
    try:
        cfg, ms = tune.tune_batch(items, reps=2)
        assert ms > 0 and ops.get_launch(3, torch.float32, "adjugate", "compensated") == cfg
        plan = BatchPlan(items, "adjugate", "compensated")
        plan.run()
        torch.cuda.synchronize()
        for i, it in enumerate(items):
            inv, det, st = ops.inv_det(it["z"], "adjugate", "compensated", status=True)
            _, grad, _ = ops.wishart_loglik(it["sigma"], it["z"], it["n_looks"], forward=True, backward=True)
            torch.cuda.synchronize()
            assert torch.equal(plan.inv[i], inv) and torch.equal(plan.det[i], det)
            assert torch.equal(plan.status[i], st) and torch.equal(plan.grad[i], grad)
        plan.close()
    finally:
        ops.set_launch(3, torch.float32, "adjugate", "compensated", keep)
