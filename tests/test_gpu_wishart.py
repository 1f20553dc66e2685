"""GPU Wishart forward/backward against the oracle, finite differences and
autograd (S = Z + 0.1 tr(Z)/3 I, Z with N=8 looks, 2x2 regions, lam in
[1e-2, 1], seed 3)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1807_08084_amd import synth
from _helpers import flat9, to_np

pytestmark = pytest.mark.gpu
N = 8.0


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_08084_amd import ops as o
    o.compute_units()
    return o


@pytest.fixture(scope="module")
def case():
    img, sig = synth.workload_wishart(seed=3, side=128)
    z = img.planes.reshape(9, -1)
    s = sig.reshape(9, -1)
    out = {}
    for key, conv in (("f64", lambda a: a), ("f32", lambda a: a.astype(np.float32).astype(np.float64))):
        zz, ss = conv(z), conv(s)
        (eh, el), (gh, gl) = oracle.wishart128(ss, zz, N)
        out[key] = dict(z=zz, s=ss, eh=eh, el=el, gh=gh, gl=gl, ks=oracle.kappa(ss))
    return out


def _loss_ref(r):
    return math.fsum(r["eh"]) + math.fsum(r["el"])


def _grad_err(g, r):
    d = (flat9(g) - r["gh"]) - r["gl"]
    return np.linalg.norm(d, axis=0) / np.linalg.norm(r["gh"], axis=0)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_forward_backward_vs_oracle(ops, case, dtype):
    key = "f64" if dtype == torch.float64 else "f32"
    r = case[key]
    S = torch.from_numpy(r["s"]).to("cuda", dtype)
    Z = torch.from_numpy(r["z"]).to("cuda", dtype)
    loss, grad, ell = ops.wishart_loglik(S, Z, N, forward=True, backward=True, ell=True)
    torch.cuda.synchronize()
    ref = _loss_ref(r)
    rel = abs(loss.item() - ref) / abs(ref)
    e_ell = np.abs(to_np(ell) - r["eh"] - r["el"]) / np.maximum(np.abs(r["eh"]), 1.0)
    eg = _grad_err(to_np(grad), r)
    print(f"{key}: loss rel err {rel:.2e}, ell max {e_ell.max():.2e}, grad max {eg.max():.2e}")
    if dtype == torch.float64:
        assert rel <= 1e-12 and e_ell.max() <= 1e-12 and eg.max() <= 1e-12
    else:
        assert rel <= 1e-5
        assert np.all(eg <= 2e-6 * r["ks"] ** 2)
    # separate passes agree with the fused one
    l2, _, _ = ops.wishart_loglik(S, Z, N, forward=True)
    _, g2, _ = ops.wishart_loglik(S, Z, N, forward=False, backward=True)
    assert torch.equal(l2, loss) and torch.equal(g2, grad)


def test_gradient_vs_finite_differences(ops, case):
    """Central differences of the GPU's own FP64 per-pixel terms."""
    r = case["f64"]
    m = 64
    S = torch.from_numpy(np.ascontiguousarray(r["s"][:, :m])).cuda()
    Z = torch.from_numpy(np.ascontiguousarray(r["z"][:, :m])).cuda()
    _, g, _ = ops.wishart_loglik(S, Z, N, forward=False, backward=True)
    g = to_np(g)
    h = 1e-6 * to_np(S[0] + S[1] + S[2]) / 3.0
    fd = np.empty_like(g)
    for k in range(9):
        sp, sm = S.clone(), S.clone()
        sp[k] += torch.from_numpy(h).cuda()
        sm[k] -= torch.from_numpy(h).cuda()
        _, _, ep = ops.wishart_loglik(sp, Z, N, ell=True)
        _, _, em = ops.wishart_loglik(sm, Z, N, ell=True)
        fd[k] = (to_np(ep) - to_np(em)) / (to_np(sp[k]) - to_np(sm[k]))
    err = np.linalg.norm(fd - g, axis=0) / np.linalg.norm(g, axis=0)
    assert err.max() <= 1e-5, err.max()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_autograd_function(ops, case, dtype):
    r = case["f64" if dtype == torch.float64 else "f32"]
    S = torch.from_numpy(r["s"]).to("cuda", dtype).requires_grad_(True)
    Z = torch.from_numpy(r["z"]).to("cuda", dtype)
    loss = ops.wishart_nll(S, Z, N)
    (3.0 * loss).backward()
    _, g, _ = ops.wishart_loglik(S.detach(), Z, N, forward=False, backward=True)
    _, g3, _ = ops.wishart_loglik(S.detach(), Z, N, forward=False, backward=True,
                                  grad_loss=torch.tensor(3.0, dtype=torch.float64, device="cuda"))
    assert torch.equal(S.grad, g3)
    assert torch.allclose(S.grad, 3.0 * g, rtol=1e-6 if dtype == torch.float32 else 1e-14)


def test_closed_form_at_sigma_equal_z(ops, case):
    r = case["f64"]
    Z = torch.from_numpy(r["z"]).cuda()
    loss, g, ell = ops.wishart_loglik(Z, Z, N, forward=True, backward=True, ell=True)
    det = np.linalg.det(oracle.full_from_planes(r["z"])).real
    assert np.allclose(to_np(ell), N * (np.log(det) + 3.0), rtol=1e-13, atol=1e-12)
    ginv = np.abs(oracle.ge(r["z"])[0]).max(axis=0)
    assert np.all(np.abs(to_np(g)).max(axis=0) <= 1e-11 * N * ginv)


@pytest.mark.parametrize("n", [1, 3, 5, 1001])
def test_ragged_and_deterministic(ops, case, n):
    r = case["f64"]
    S = torch.from_numpy(np.ascontiguousarray(r["s"][:, :n])).cuda()
    Z = torch.from_numpy(np.ascontiguousarray(r["z"][:, :n])).cuda()
    l1, g1, _ = ops.wishart_loglik(S, Z, N, forward=True, backward=True)
    l2, g2, _ = ops.wishart_loglik(S, Z, N, forward=True, backward=True)
    assert torch.equal(l1, l2) and torch.equal(g1, g2)
    ref = math.fsum(r["eh"][:n]) + math.fsum(r["el"][:n])
    assert abs(l1.item() - ref) <= 1e-12 * abs(ref)
    assert _grad_err(to_np(g1), {k: (v[:, :n] if k in ("gh", "gl") else v) for k, v in r.items()}).max() <= 1e-12


def test_empty_sum_is_zero(ops):
    S = torch.empty((9, 0), dtype=torch.float64, device="cuda")
    loss, _, _ = ops.wishart_loglik(S, S.clone(), N, forward=True)
    assert loss.item() == 0.0


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("n_cut", [0, 77])
def test_every_launch_shape_with_minimal_workspace(ops, case, dtype, n_cut):
    """The loss matches the oracle and the gradient is bitwise the same for
    every launch shape, each run with a workspace of exactly the size the
    library asks for (one partial per tile of the smallest shape)."""
    r = case["f64" if dtype == torch.float64 else "f32"]
    n = r["z"].shape[1] - n_cut
    S = torch.from_numpy(np.ascontiguousarray(r["s"][:, :n])).to("cuda", dtype)
    Z = torch.from_numpy(np.ascontiguousarray(r["z"][:, :n])).to("cuda", dtype)
    nbytes = ops.workspace_bytes(dtype, n)
    assert nbytes == max(1, (n + 63) // 64) * 8
    ref = math.fsum(r["eh"][:n]) + math.fsum(r["el"][:n])
    op = ops.wishart_launch_op(n)
    keep = ops.get_launch(op, dtype, "adjugate", "plain")
    grads = []
    try:
        for block in (64, 128, 256):
            for unroll in (1, 2):
                for vb, gpc in ((16, 0), (8, 8)):
                    ops.set_launch(op, dtype, "adjugate", "plain", dict(block=block, unroll=unroll, grid_per_cu=gpc,
                                                                        nontemporal=1, vector_bytes=vb,
                                                                        blocks_per_cu=0))
                    ws = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
                    loss, g, _ = ops.wishart_loglik(S, Z, N, forward=True, backward=True, workspace=ws)
                    torch.cuda.synchronize()
                    tol = 1e-12 if dtype == torch.float64 else 1e-5
                    assert abs(loss.item() - ref) <= tol * abs(ref), (block, unroll, vb, gpc)
                    grads.append(g)
    finally:
        ops.set_launch(op, dtype, "adjugate", "plain", keep)
    assert all(torch.equal(grads[0], g) for g in grads[1:])


@pytest.mark.parametrize("width", [4095, 4097])
def test_both_launch_entries_at_the_size_boundary(ops, width):
    """2048 x 4095 and 2048 x 4097 pixels sit on either side of 2^23, where
    the Wishart call switches launch entry (op 5 below, op 1 from there on):
    the loss against the FP64 oracle's, and the gradient on sampled pixels
    against the oracle's."""
    n = 2048 * width
    assert ops.wishart_launch_op(n) == (5 if n < (1 << 23) else 1)
    img = synth.make_image(2048, width, 8, (2, 2), (1e-2, 1.0), 17)
    z = img.planes.reshape(9, -1).astype(np.float32).astype(np.float64)
    s = synth.wishart_sigma0(z).astype(np.float32).astype(np.float64)
    Z = torch.from_numpy(z).to("cuda", torch.float32)
    S = torch.from_numpy(s).to("cuda", torch.float32)
    loss, g, _ = ops.wishart_loglik(S, Z, N, forward=True, backward=True)
    torch.cuda.synchronize()
    ell, _ = oracle.wishart(s, z, N, grad=False)
    ref = math.fsum(ell)
    assert abs(loss.item() - ref) <= 1e-5 * abs(ref)
    idx = np.sort(np.random.default_rng(width).choice(n, 4000, replace=False))
    (_, _), (gh, gl) = oracle.wishart128(s[:, idx], z[:, idx], N)
    ks = oracle.kappa(s[:, idx])
    d = (to_np(g).reshape(9, -1)[:, idx] - gh) - gl
    err = np.linalg.norm(d, axis=0) / np.linalg.norm(gh, axis=0)
    assert np.all(err <= 2e-6 * ks * ks), err.max()


@pytest.mark.parametrize("launch_n", [40000, 70000])
def test_low_accuracy_count(ops, case, launch_n):
    """counters[1] counts the positive-definite S whose plain determinant may
    be off by more than 1e-3 relative (the a-priori bound, pinned on the host
    against the __float128 oracle in test_host_pixel.py).  The Wishart image's
    well-conditioned S (kappa <= ~30) counts none; Haar-rotated FP32 S with
    eigenvalues (1, l2, 10^-U(0, 6)) count exactly the pixels whose host-built
    bound exceeds the threshold, up to the rounding differences of contracted
    FMAs on the device (pixels within 1% of the threshold may go either way)."""
    from host import pixel
    r = case["f32"]
    S = torch.from_numpy(np.ascontiguousarray(r["s"])).to("cuda", torch.float32)
    Z = torch.from_numpy(np.ascontiguousarray(r["z"])).to("cuda", torch.float32)
    ctr = torch.zeros(3, dtype=torch.int64, device="cuda")
    ops.wishart_loglik(S, Z, N, forward=True, backward=True, counters=ctr)
    assert ctr.tolist() == [0, 0, 0]
    rng = np.random.default_rng(77)
    m = launch_n
    U = synth.haar_unitary(rng, m)
    eig = np.stack([np.ones(m), 10.0 ** -rng.uniform(0, 2, m), 10.0 ** -rng.uniform(0, 6, m)], 1)
    s32 = synth.pack(np.einsum("mij,mj,mkj->mik", U, eig, np.conj(U))).astype(np.float32)
    assert np.all(oracle.pd_class(s32.astype(np.float64)) == 0)
    det, bound = pixel.det_plain_bound_f32(s32)
    ratio = bound.astype(np.float64) / det.astype(np.float64)
    lo, hi = int(np.sum(ratio > 1.01e-3)), int(np.sum(ratio >= 0.99e-3))
    assert lo > 100  # the set exercises the flag
    St = ops.upload_planes(s32, torch.float32)
    ctr.zero_()
    ops.wishart_loglik(St, St, N, forward=True, backward=True, counters=ctr)
    c = ctr.tolist()
    assert c[0] == 0 and c[2] == 0
    assert lo <= c[1] <= hi, (lo, c[1], hi)
    # FP64: the same matrices widened are far inside the threshold
    St64 = ops.upload_planes(s32.astype(np.float64), torch.float64)
    ctr.zero_()
    ops.wishart_loglik(St64, St64, N, forward=True, counters=ctr)
    assert ctr.tolist() == [0, 0, 0]
