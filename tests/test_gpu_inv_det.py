"""GPU parity of polsar_inv_det against the CPU oracle (256x256, N=4, 2x2
regions, lam in [1e-2, 1], seed 0), edge cases, ragged sizes and bitwise
invariants.  All calls go through the C ABI (ctypes binding)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1807_08084_amd import synth
from _helpers import U32, U64, flat9, to_np, tol_f32, tol_f64_comp, tol_plain

pytestmark = pytest.mark.gpu

COMBOS = [  # (dtype, method, precision)
    (torch.float64, "adjugate", "compensated"),
    (torch.float64, "adjugate", "plain"),
    (torch.float64, "cholesky", "plain"),
    (torch.float32, "adjugate", "compensated"),
    (torch.float32, "adjugate", "plain"),
    (torch.float32, "adjugate", "wide"),
    (torch.float32, "cholesky", "plain"),
    (torch.float32, "cholesky", "compensated"),
    (torch.float32, "cholesky", "wide"),
]


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_08084_amd import ops as o
    o.compute_units()
    return o


@pytest.fixture(scope="module")
def small():
    img = synth.workload_small()
    z64 = img.planes.reshape(9, -1)
    ref = {}
    for key, z in (("f64", z64), ("f32", z64.astype(np.float32).astype(np.float64))):
        (ih, il), (dh, dl) = oracle.ge128(z)
        ref[key] = dict(z=z, ih=ih, il=il, dh=dh, dl=dl, k=oracle.kappa(z), pd=oracle.pd_class(z))
    return ref


def _run(ops, z_np, dtype, method, prec, **kw):
    z = torch.from_numpy(np.ascontiguousarray(z_np)).to(device="cuda", dtype=dtype)
    inv, det, st = ops.inv_det(z, method, prec, status=True, **kw)
    torch.cuda.synchronize()
    return to_np(inv), to_np(det), st.cpu().numpy()


def _tol(dtype, method, prec, k):
    if dtype == torch.float64 and method == "adjugate" and prec == "compensated":
        return tol_f64_comp(k)
    if dtype == torch.float32 and method == "adjugate" and prec == "compensated":
        return tol_f32(k)
    if prec == "wide":
        return 4 * U32 + tol_plain(U64, k)
    if dtype == torch.float32 and prec == "compensated":  # Cholesky with FP64 fallback
        return tol_plain(U32, k)
    return tol_plain(U64 if dtype == torch.float64 else U32, k)


@pytest.mark.parametrize("dtype,method,prec", COMBOS)
def test_parity_small_image(ops, small, dtype, method, prec):
    r = small["f64" if dtype == torch.float64 else "f32"]
    inv, det, st = _run(ops, r["z"], dtype, method, prec)
    assert np.all(r["pd"] == 0)
    e_inv = oracle.inv_rel_err(inv, r["ih"], r["il"])
    e_det = oracle.det_rel_err(det, r["dh"], r["dl"])
    tol = _tol(dtype, method, prec, r["k"])
    print(f"{dtype} {method} {prec}: max inv err {e_inv.max():.3e} det err {e_det.max():.3e} "
          f"kappa max {r['k'].max():.3e}")
    assert np.all(e_inv <= tol), (e_inv.max(), np.argmax(e_inv / tol))
    assert np.all(e_det <= tol), (e_det.max(), np.argmax(e_det / tol))
    assert set(np.unique(st)) <= {0, 1}
    if not (dtype == torch.float32 and prec == "compensated"):
        assert np.all(st == 0)


def _padded(ops, z_np, n, pitch, dtype):
    buf = torch.zeros((9, pitch), dtype=dtype, device="cuda")
    buf[:, :n] = torch.from_numpy(np.ascontiguousarray(z_np[:, :n])).to(device="cuda", dtype=dtype)
    return buf[:, :n]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("method,prec", [("adjugate", "compensated"), ("adjugate", "plain"), ("cholesky", "plain")])
def test_ragged_sizes_vector_and_scalar_paths(ops, small, dtype, method, prec):
    r = small["f64" if dtype == torch.float64 else "f32"]
    for n in (1, 2, 3, 5, 7, 63, 255, 1021, 4099):
        zv = _padded(ops, r["z"], n, ((n + 3) // 4) * 4 + 4, dtype)   # 16-byte planes: vector path
        zs = torch.from_numpy(np.ascontiguousarray(r["z"][:, :n])).to(device="cuda", dtype=dtype)
        outs = []
        for z in (zv, zs):
            inv, det, st = ops.inv_det(z, method, prec, status=True)
            outs.append((to_np(inv), to_np(det), st.cpu().numpy()))
        torch.cuda.synchronize()
        for a, b in zip(outs[0], outs[1]):
            assert np.array_equal(a, b), n   # same per-pixel arithmetic on both paths
        inv, det, _ = outs[0]
        k = r["k"][:n]
        tol = _tol(dtype, method, prec, k)
        assert np.all(oracle.inv_rel_err(inv, r["ih"][:, :n], r["il"][:, :n]) <= tol)
        assert np.all(oracle.det_rel_err(det, r["dh"][:n], r["dl"][:n]) <= tol)


def _edge_planes():
    cols = []
    def add(a, d, f, b=0j, c=0j, e=0j):
        cols.append([a, d, f, b.real, b.imag, c.real, c.imag, e.real, e.imag])
    add(1, 1, 1)                       # identity
    add(4, 0.25, 16)                   # diagonal, powers of four
    add(2.0 ** 20, 2.0 ** -20, 1)      # diagonal, wide range
    add(0, 0, 0)                       # zero matrix: det 0
    add(1, -1, 1)                      # indefinite
    add(1, 1, 1, b=1 + 0j)             # singular
    add(np.nan, 1, 1)                  # non-finite input
    add(np.inf, 1, 1)
    add(1, 1, 1, e=np.inf + 0j)
    add(4, 5, 6, 1 + 1j, 2j, 1 - 1j)   # the worked example
    add(0, 0, 0, 1 + 0j, 1 + 0j, 1 + 0j)  # eigenvalues (2, -1, -1): det 2 > 0, a = 0
    add(1, 1, -1, 2 + 0j)              # eigenvalues (3, -1, -1): det 3 > 0, a > 0, ad - |b|^2 < 0
    return np.array(cols, dtype=np.float64).T


@pytest.mark.parametrize("dtype,method,prec", COMBOS)
def test_edge_cases(ops, dtype, method, prec):
    z = _edge_planes()
    inv, det, st = _run(ops, z, dtype, method, prec)
    assert st[0] == 0 and np.array_equal(inv[:, 0], [1, 1, 1, 0, 0, 0, 0, 0, 0]) and det[0] == 1
    assert st[1] == 0 and np.array_equal(inv[:3, 1], [0.25, 4, 0.0625]) and det[1] == 16
    assert np.allclose(inv[:3, 2], [2.0 ** -20, 2.0 ** 20, 1], rtol=4 * U32) and det[2] == 1
    assert st[3] == 2 and st[4] == 2 and st[5] == 2
    assert st[6] == 3 and st[7] == 3 and st[8] == 3
    assert st[9] == 0
    assert st[10] == 2 and st[11] == 2          # indefinite with a positive determinant
    if method == "adjugate":
        assert det[10] > 0 and det[11] > 0      # (Cholesky meets a negative pivot: NaN)
    want = np.array([28, 20, 18, -8, -4, 2, -10, -2, 6]) / 80.0
    u = U64 if dtype == torch.float64 else U32
    assert np.allclose(inv[:, 9], want, rtol=16 * u, atol=16 * u) and abs(det[9] - 80) <= 80 * 16 * u


def test_counters_match_status(ops):
    z = np.ascontiguousarray(np.concatenate([_edge_planes()] * 37, axis=1))
    for dtype, method, prec in COMBOS:
        zt = torch.from_numpy(z).to(device="cuda", dtype=dtype)
        ctr = torch.zeros(3, dtype=torch.int64, device="cuda")
        _, _, st = ops.inv_det(zt, method, prec, status=True, counters=ctr)
        s = st.cpu().numpy()
        c = ctr.cpu().numpy()
        assert c[0] == np.sum(s == 2) and c[1] == np.sum(s == 1) and c[2] == np.sum(s == 3), (method, prec)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_in_place(ops, small, dtype):
    r = small["f64" if dtype == torch.float64 else "f32"]
    z = torch.from_numpy(r["z"]).to(device="cuda", dtype=dtype)
    inv_ref, det_ref, _ = ops.inv_det(z, "adjugate", "compensated")
    zz = z.clone()
    _, det, _ = ops.inv_det(zz, "adjugate", "compensated", inv=zz)
    torch.cuda.synchronize()
    assert torch.equal(zz, inv_ref) and torch.equal(det, det_ref)


@pytest.mark.parametrize("dtype,method,prec", COMBOS)
def test_bitwise_invariants(ops, small, dtype, method, prec):
    """Scaling by 4^j scales det by 64^j and the inverse by 4^-j exactly;
    conjugating Z conjugates the inverse and keeps det, exactly."""
    r = small["f64" if dtype == torch.float64 else "f32"]
    z = r["z"][:, :20000]
    inv, det, st = _run(ops, z, dtype, method, prec)
    inv2, det2, st2 = _run(ops, z * 16.0, dtype, method, prec)
    assert np.array_equal(inv2, inv / 16.0) and np.array_equal(det2, det * 4096.0) and np.array_equal(st, st2)
    zc = z.copy()
    zc[[4, 6, 8]] *= -1
    inv3, det3, _ = _run(ops, zc, dtype, method, prec)
    invc = inv.copy()
    invc[[4, 6, 8]] *= -1
    assert np.array_equal(inv3, invc) and np.array_equal(det3, det)


def test_results_independent_of_launch(ops, small):
    z = torch.from_numpy(small["f32"]["z"]).to(device="cuda", dtype=torch.float32)
    keep = ops.get_launch(0, torch.float32, "adjugate", "compensated")
    outs = []
    try:
        for cfg in ({"block": 64, "unroll": 1, "grid_per_cu": 0, "nontemporal": 0, "vector_bytes": 16},
                    {"block": 256, "unroll": 4, "grid_per_cu": 2, "nontemporal": 1, "vector_bytes": 16},
                    {"block": 128, "unroll": 2, "grid_per_cu": 8, "nontemporal": 1, "vector_bytes": 8},
                    {"block": 64, "unroll": 4, "grid_per_cu": 0, "nontemporal": 0, "vector_bytes": 8},
                    {"block": 64, "unroll": 1, "grid_per_cu": 0, "nontemporal": 1, "vector_bytes": 16,
                     "blocks_per_cu": 4},
                    {"block": 256, "unroll": 2, "grid_per_cu": 8, "nontemporal": 1, "vector_bytes": 16,
                     "blocks_per_cu": 2}):
            ops.set_launch(0, torch.float32, "adjugate", "compensated", cfg)
            inv, det, st = ops.inv_det(z, "adjugate", "compensated", status=True)
            outs.append((inv.clone(), det.clone(), st.clone()))
    finally:
        ops.set_launch(0, torch.float32, "adjugate", "compensated", keep)
    for o in outs[1:]:
        assert all(torch.equal(a, b) for a, b in zip(outs[0], o))


@pytest.fixture(scope="module")
def rerouting():
    """The precision recipe (N=3, per-pixel Sigma, lam in [1e-8, 1]) at 512x512:
    about a third of the FP32 pixels are recomputed in FP64.  Reference: the
    host build of the same per-pixel arithmetic."""
    pixel = pytest.importorskip("host.pixel")
    z = synth.workload_precision(seed=11, side=512).planes.reshape(9, -1).astype(np.float32)
    inv, det, st, _ = pixel.adjugate_comp_f32(z)
    assert 0.2 < np.mean(st == 1) < 0.5
    return z, inv, det, st


@pytest.mark.parametrize("cfg", [
    {"block": 128, "unroll": 1, "grid_per_cu": 0, "nontemporal": 1, "vector_bytes": 16},
    {"block": 64, "unroll": 1, "grid_per_cu": 1, "nontemporal": 0, "vector_bytes": 16},
    {"block": 256, "unroll": 2, "grid_per_cu": 2, "nontemporal": 1, "vector_bytes": 16, "blocks_per_cu": 2},
    {"block": 128, "unroll": 2, "grid_per_cu": 8, "nontemporal": 1, "vector_bytes": 8, "blocks_per_cu": 4},
    {"block": 64, "unroll": 2, "grid_per_cu": 64, "nontemporal": 1, "vector_bytes": 16, "blocks_per_cu": 8},
    {"block": 128, "unroll": 1, "grid_per_cu": 0, "nontemporal": 1, "vector_bytes": 8, "blocks_per_cu": 8},
])
@pytest.mark.parametrize("n_cut,offset", [(0, 0), (3, 0), (1, 1)])
def test_reroute_queue_matches_host(ops, rerouting, cfg, n_cut, offset):
    """FP32 compensated results, statuses and counters are bitwise those of
    the host build for every launch shape: one tile per block and
    persistent blocks, one vector per lane or two sharing one FP64 queue
    (the 256-lane block with two falls back to one: its queue would not fit),
    16- and 8-byte vectors, a ragged length, and planes off 16-byte
    alignment (one pixel per lane)."""
    z, inv_h, det_h, st_h = rerouting
    n = z.shape[1] - n_cut - offset
    sl = slice(offset, offset + n)
    buf = torch.from_numpy(np.ascontiguousarray(z[:, :n + offset])).to("cuda")
    zt = buf[:, offset:]
    keep = ops.get_launch(0, torch.float32, "adjugate", "compensated")
    try:
        ops.set_launch(0, torch.float32, "adjugate", "compensated", cfg)
        ctr = torch.zeros(3, dtype=torch.int64, device="cuda")
        inv, det, st = ops.inv_det(zt, "adjugate", "compensated", status=True, counters=ctr)
        torch.cuda.synchronize()
    finally:
        ops.set_launch(0, torch.float32, "adjugate", "compensated", keep)
    s = st.cpu().numpy()
    assert np.array_equal(s, st_h[sl])
    assert np.array_equal(inv.cpu().numpy().view(np.uint32), inv_h[:, sl].view(np.uint32))
    assert np.array_equal(det.cpu().numpy().view(np.uint32), det_h[sl].view(np.uint32))
    c = ctr.cpu().numpy()
    assert c[0] == np.sum(s == 2) and c[1] == np.sum(s == 1) and c[2] == np.sum(s == 3)


def test_reroute_queue_in_place(ops, rerouting):
    z, inv_h, det_h, _ = rerouting
    zz = torch.from_numpy(z).to("cuda")
    _, det, _ = ops.inv_det(zz, "adjugate", "compensated", inv=zz)
    torch.cuda.synchronize()
    assert np.array_equal(zz.cpu().numpy().view(np.uint32), inv_h.view(np.uint32))
    assert np.array_equal(det.cpu().numpy().view(np.uint32), det_h.view(np.uint32))
