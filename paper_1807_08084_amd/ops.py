"""torch-facing calls of the C ABI.  Argument marshalling only: every step of
the computation runs in the HIP kernels of libpolsar.so.

Tensors hold packed planes with the plane index first: shape (9, ...) on the
GPU, float32 or float64, each plane contiguous (plane pitch = stride(0)).
Plane order a, d, f, Re b, Im b, Re c, Im c, Re e, Im e (upper triangle).
Work is enqueued on torch's current stream.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L

_METHODS = {"adjugate": L.ADJUGATE, "cholesky": L.CHOLESKY}
_PRECS = {"plain": L.PLAIN, "compensated": L.COMPENSATED, "wide": L.WIDE}


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return L.F32
    if t.dtype == torch.float64:
        return L.F64
    raise TypeError(f"planes must be float32 or float64, got {t.dtype}")


def _planes(t: torch.Tensor, name: str) -> tuple[int, int]:
    """(n, pitch) of a (9, ...) plane tensor; each plane must be contiguous."""
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dim() < 2 or t.shape[0] != 9:
        raise ValueError(f"{name} must have shape (9, ...), got {tuple(t.shape)}")
    n = t[0].numel()
    if not t[0].is_contiguous():
        raise ValueError(f"{name}: each plane must be contiguous")
    return n, t.stride(0)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def recommended_pitch(dtype: torch.dtype, n: int) -> int:
    return int(L.lib().polsar_recommended_pitch(L.F32 if dtype == torch.float32 else L.F64, int(n)))


def empty_planes(k: int, shape, dtype: torch.dtype, device="cuda") -> torch.Tensor:
    """Uninitialised (k, *shape) planes laid out with the recommended pitch
    (a view into a (k, pitch) buffer; each plane contiguous)."""
    shape = tuple(shape) if isinstance(shape, (tuple, list, torch.Size)) else (int(shape),)
    n = 1
    for s in shape:
        n *= s
    buf = torch.empty((k, recommended_pitch(dtype, n)), dtype=dtype, device=device)
    return buf[:, :n].view((k,) + shape) if len(shape) > 1 else buf[:, :n]


def upload_planes(planes, dtype: torch.dtype, device="cuda") -> torch.Tensor:
    """Copy host planes (9, ...) into device planes with the recommended pitch."""
    t = torch.as_tensor(planes)
    out = empty_planes(t.shape[0], t.shape[1:], dtype, device)
    out.copy_(t.to(dtype))
    return out


def inv_det(z: torch.Tensor, method: str = "adjugate", precision: str = "compensated", *,
            inv: torch.Tensor | None = None, det: torch.Tensor | None = None,
            status: bool | torch.Tensor = False, counters: torch.Tensor | None = None,
            want_inv: bool = True, want_det: bool = True, stream=None):
    """Inverse and determinant of every packed matrix of ``z``.

    Returns (inv, det, status) where each is a new tensor (or the one given),
    or None when not requested.  ``counters``: int64 tensor of 3 on the GPU,
    added to ([not_pd, rerouted, nonfinite]).
    """
    dt = _dtype_code(z)
    n, zp = _planes(z, "z")
    shape = z.shape[1:]
    if inv is None and det is None and want_inv and want_det:
        out = empty_planes(10, shape, z.dtype, z.device)  # 9 inverse planes + det, one pitch
        inv, det = out[:9], out[9]
    if inv is None and want_inv:
        inv = empty_planes(9, shape, z.dtype, z.device)
    ip = _planes(inv, "inv")[1] if inv is not None else 0
    if det is None and want_det:
        det = torch.empty(shape, dtype=z.dtype, device=z.device)
    st = None
    if isinstance(status, torch.Tensor):
        st = status
    elif status:
        st = torch.empty(shape, dtype=torch.uint8, device=z.device)
    if counters is not None and (counters.dtype != torch.int64 or counters.numel() != 3 or not counters.is_cuda):
        raise ValueError("counters must be a GPU int64 tensor of 3 elements")
    rc = L.lib().polsar_inv_det(dt, _METHODS[method], _PRECS[precision], n, _ptr(z), zp,
                                _ptr(inv), ip, _ptr(det), _ptr(st), _ptr(counters), _stream(stream))
    L.check(rc, "polsar_inv_det")
    return inv, det, st


def multilook_inv_det(looks: torch.Tensor, n_looks: int, method: str = "adjugate",
                      precision: str = "compensated", *, want_z: bool = False, status: bool = False,
                      counters: torch.Tensor | None = None, stream=None):
    """Fused multilook + inverse/determinant from (6N, ...) look planes.

    Returns (z or None, inv, det, status or None)."""
    dt = _dtype_code(looks)
    if looks.dim() < 2 or looks.shape[0] != 6 * n_looks:
        raise ValueError(f"looks must have shape (6N, ...) with N={n_looks}")
    if not looks.is_cuda or not looks[0].is_contiguous():
        raise ValueError("looks must be GPU planes, each contiguous")
    shape = looks.shape[1:]
    n, lp = looks[0].numel(), looks.stride(0)
    out = empty_planes(10, shape, looks.dtype, looks.device)
    inv, det = out[:9], out[9]
    z = empty_planes(9, shape, looks.dtype, looks.device) if want_z else None
    st = torch.empty(shape, dtype=torch.uint8, device=looks.device) if status else None
    rc = L.lib().polsar_multilook_inv_det(dt, _METHODS[method], _PRECS[precision], n, int(n_looks), _ptr(looks),
                                          lp, _ptr(z), z.stride(0) if z is not None else 0, _ptr(inv),
                                          inv.stride(0), _ptr(det), _ptr(st), _ptr(counters), _stream(stream))
    L.check(rc, "polsar_multilook_inv_det")
    return z, inv, det, st


def boxcar_inv_det(s: torch.Tensor, radius: int, method: str = "adjugate", precision: str = "compensated", *,
                   want_z: bool = False, status: bool = False, counters: torch.Tensor | None = None, stream=None):
    """Spatial (boxcar) multilook of a single-look image s (6, H, W) over a
    (2r+1)^2 window clipped at the border, fused with the inverse/determinant.

    Returns (z or None, inv, det, status or None), shaped (9, H, W) / (H, W)."""
    dt = _dtype_code(s)
    if s.dim() != 3 or s.shape[0] != 6 or not s.is_cuda or not s[0].is_contiguous():
        raise ValueError("s must be GPU planes of shape (6, H, W), each contiguous")
    H, W = int(s.shape[1]), int(s.shape[2])
    shape = (H, W)
    out = empty_planes(10, shape, s.dtype, s.device)
    inv, det = out[:9], out[9]
    z = empty_planes(9, shape, s.dtype, s.device) if want_z else None
    st = torch.empty(shape, dtype=torch.uint8, device=s.device) if status else None
    rc = L.lib().polsar_boxcar_inv_det(dt, _METHODS[method], _PRECS[precision], H, W, int(radius), _ptr(s),
                                       s.stride(0), _ptr(z), z.stride(0) if z is not None else 0, _ptr(inv),
                                       inv.stride(0), _ptr(det), _ptr(st), _ptr(counters), _stream(stream))
    L.check(rc, "polsar_boxcar_inv_det")
    return z, inv, det, st


def blockdiag_inv_det(z: torch.Tensor, n_blocks: int, method: str = "adjugate", precision: str = "compensated",
                      *, block_det: bool = False, status: bool = False, counters: torch.Tensor | None = None,
                      stream=None):
    """Block-diagonal pixels: z (9K, ...) -> (inv (9K, ...), det product, block dets or None, status or None)."""
    dt = _dtype_code(z)
    if z.dim() < 2 or z.shape[0] != 9 * n_blocks or not z.is_cuda or not z[0].is_contiguous():
        raise ValueError(f"z must be GPU planes of shape (9*{n_blocks}, ...)")
    shape = z.shape[1:]
    n, zp = z[0].numel(), z.stride(0)
    out = empty_planes(9 * n_blocks + 1, shape, z.dtype, z.device)
    inv, det = out[:9 * n_blocks], out[9 * n_blocks]
    bd = empty_planes(n_blocks, shape, z.dtype, z.device) if block_det else None
    st = torch.empty(shape, dtype=torch.uint8, device=z.device) if status else None
    rc = L.lib().polsar_blockdiag_inv_det(dt, _METHODS[method], _PRECS[precision], n, int(n_blocks), _ptr(z), zp,
                                          _ptr(inv), inv.stride(0), _ptr(det), _ptr(bd),
                                          bd.stride(0) if bd is not None else 0, _ptr(st), _ptr(counters),
                                          _stream(stream))
    L.check(rc, "polsar_blockdiag_inv_det")
    return inv, det, bd, st


class Streamer:
    """Out-of-core inverse/determinant of host-resident planes, chunk by chunk
    through two device buffer sets and two streams (polsar_streamer_*)."""

    def __init__(self, dtype: torch.dtype, chunk_pixels: int, method: str = "adjugate",
                 precision: str = "compensated"):
        self.dtype = dtype
        self._h = ctypes.c_void_p()
        L.check(L.lib().polsar_streamer_create(L.F32 if dtype == torch.float32 else L.F64, _METHODS[method],
                                               _PRECS[precision], int(chunk_pixels), ctypes.byref(self._h)),
                "polsar_streamer_create")

    def run(self, z: torch.Tensor, inv: torch.Tensor | None = None, det: torch.Tensor | None = None,
            status: torch.Tensor | None = None, counters: torch.Tensor | None = None):
        """z: (9, ...) CPU planes (pinned for full speed); outputs CPU tensors,
        allocated pinned when not given.  Synchronous."""
        if z.is_cuda or z.dtype != self.dtype or z.shape[0] != 9 or not z[0].is_contiguous():
            raise ValueError("z must be CPU planes (9, ...) of the streamer's dtype")
        shape = z.shape[1:]
        n = z[0].numel()
        if inv is None:
            inv = torch.empty((9,) + tuple(shape), dtype=z.dtype, pin_memory=True)
        if det is None:
            det = torch.empty(shape, dtype=z.dtype, pin_memory=True)
        rc = L.lib().polsar_streamer_run(self._h, n, _ptr(z), z.stride(0), _ptr(inv), inv.stride(0), _ptr(det),
                                         _ptr(status), _ptr(counters))
        L.check(rc, "polsar_streamer_run")
        return inv, det, status

    def close(self):
        if self._h:
            L.lib().polsar_streamer_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_DIST = {"kl": 0, "bhattacharyya": 1}


def nlm_wishart(z: torch.Tensor, aux: torch.Tensor, n_looks: float, radius: int, h: float,
                distance: str = "kl", want_wsum: bool = False, stream=None):
    """Nonlocal-means filter of a (9, H, W) covariance image with Wishart
    stochastic distances over a (2r+1)^2 window.  aux: the (9, H, W) inverse
    planes for "kl", the (H, W) determinant plane for "bhattacharyya" (as
    inv_det returns them).  Returns (out (9, H, W), wsum (H, W) or None)."""
    dt = _dtype_code(z)
    if z.dim() != 3 or z.shape[0] != 9 or not z.is_cuda or not z[0].is_contiguous():
        raise ValueError("z must be GPU planes of shape (9, H, W), each plane contiguous")
    H, W = z.shape[1], z.shape[2]
    if distance == "kl":
        if aux.shape != z.shape or not aux[0].is_contiguous():
            raise ValueError("aux must be the (9, H, W) inverse planes")
        ap = aux.stride(0)
    else:
        if aux.shape != z.shape[1:] or not aux.is_contiguous():
            raise ValueError("aux must be the (H, W) determinant plane")
        ap = 0
    if aux.dtype != z.dtype:
        raise TypeError("aux must have z's dtype")
    out = empty_planes(9, (H, W), z.dtype, z.device)
    ws = torch.empty((H, W), dtype=z.dtype, device=z.device) if want_wsum else None
    rc = L.lib().polsar_nlm_wishart(dt, _DIST[distance], H, W, int(radius), float(n_looks), float(h), _ptr(z),
                                    z.stride(0), _ptr(aux), ap, _ptr(out), out.stride(0), _ptr(ws), _stream(stream))
    L.check(rc, "polsar_nlm_wishart")
    return out, ws


def workspace_bytes(dtype: torch.dtype, n: int) -> int:
    return int(L.lib().polsar_wishart_workspace_bytes(L.F32 if dtype == torch.float32 else L.F64, n))


def wishart_loglik(sigma: torch.Tensor, z: torch.Tensor, n_looks: float, *, forward: bool = True,
                   backward: bool = False, grad_loss: torch.Tensor | None = None, ell: bool = False,
                   counters: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                   grad: torch.Tensor | None = None, stream=None):
    """L = sum N (ln det S + tr(S^-1 Z)) and/or its packed gradient.

    ``grad``: planes to write the gradient into (else new ones).
    Returns (loss 0-d float64 GPU tensor or None, grad or None, ell or None).
    """
    if sigma.dtype != z.dtype:
        raise TypeError("sigma and z must have the same dtype")
    dt = _dtype_code(sigma)
    n, sp = _planes(sigma, "sigma")
    nz, zp = _planes(z, "z")
    if nz != n:
        raise ValueError("sigma and z differ in size")
    mode = (L.FWD if forward else 0) | (L.BWD if backward else 0)
    if mode == 0:
        raise ValueError("nothing to do")
    loss = torch.empty((), dtype=torch.float64, device=sigma.device) if forward else None
    if not backward:
        grad = None
    elif grad is None:
        grad = empty_planes(9, sigma.shape[1:], sigma.dtype, sigma.device)
    elif grad.dtype != sigma.dtype or grad[0].numel() != n:
        raise ValueError("grad must match sigma")
    gp = _planes(grad, "grad")[1] if grad is not None else 0
    el = torch.empty(sigma.shape[1:], dtype=sigma.dtype, device=sigma.device) if (ell and forward) else None
    wsb = workspace_bytes(sigma.dtype, n) if forward else 0
    if forward and (workspace is None or workspace.numel() * workspace.element_size() < wsb):
        workspace = torch.empty(max(1, (wsb + 7) // 8), dtype=torch.float64, device=sigma.device)
    if grad_loss is not None:
        grad_loss = grad_loss.to(dtype=torch.float64).reshape(()).contiguous()
    ws_size = workspace.numel() * workspace.element_size() if workspace is not None else 0
    rc = L.lib().polsar_wishart_loglik(dt, mode, n, _ptr(sigma), sp, _ptr(z), zp, float(n_looks),
                                       _ptr(loss), _ptr(el), _ptr(grad_loss), _ptr(grad), gp,
                                       _ptr(workspace), ws_size, _ptr(counters), _stream(stream))
    L.check(rc, "polsar_wishart_loglik")
    return loss, grad, el


class WishartNLL(torch.autograd.Function):
    """L(S) = sum_px N (ln det S + tr(S^-1 Z)) with the hand-written adjoint.

    forward(sigma, z, n_looks) -> 0-d float64 tensor.  backward recomputes
    S^-1 from the adjugate (nothing but the inputs is saved) and returns the
    gradient with respect to the packed real planes of S (off-diagonal
    components doubled; what finite differences on the planes measure).
    """

    @staticmethod
    def forward(ctx, sigma, z, n_looks):
        loss, _, _ = wishart_loglik(sigma, z, n_looks, forward=True)
        ctx.save_for_backward(sigma, z)
        ctx.n_looks = float(n_looks)
        return loss

    @staticmethod
    def backward(ctx, g):
        sigma, z = ctx.saved_tensors
        _, grad, _ = wishart_loglik(sigma, z, ctx.n_looks, forward=False, backward=True, grad_loss=g)
        return grad, None, None


def wishart_nll(sigma: torch.Tensor, z: torch.Tensor, n_looks: float) -> torch.Tensor:
    return WishartNLL.apply(sigma, z, n_looks)


def stream_copy(src: torch.Tensor, dst: torch.Tensor, n_in: int, n_out: int, n: int, stream=None):
    """Bandwidth probe: n_in planes of src -> n_out planes of dst."""
    dt = _dtype_code(src)
    rc = L.lib().polsar_stream_copy(dt, n, _ptr(src), src.stride(0), n_in, _ptr(dst), dst.stride(0), n_out,
                                    _stream(stream))
    L.check(rc, "polsar_stream_copy")


def get_launch(op: int, dtype: torch.dtype, method: str = "adjugate", precision: str = "compensated") -> dict:
    c = L.Launch()
    d = L.F32 if dtype == torch.float32 else L.F64
    L.check(L.lib().polsar_get_launch(op, d, _METHODS[method], _PRECS[precision], ctypes.byref(c)),
            "polsar_get_launch")
    return c.as_dict()


def wishart_launch_op(n: int) -> int:
    """The launch-table op (1, or 5 for small images) of a Wishart call on n pixels."""
    return int(L.lib().polsar_wishart_launch_op(int(n)))


def inv_det_launch_op(n: int) -> int:
    """The launch-table op (0, or 6 for large images) of an inverse call on n pixels."""
    return int(L.lib().polsar_inv_det_launch_op(int(n)))


def set_launch(op: int, dtype: torch.dtype, method: str, precision: str, cfg: dict) -> None:
    c = L.Launch(**cfg)
    d = L.F32 if dtype == torch.float32 else L.F64
    L.check(L.lib().polsar_set_launch(op, d, _METHODS[method], _PRECS[precision], ctypes.byref(c)),
            "polsar_set_launch")


def autotune_inv_det(z: torch.Tensor, method: str = "adjugate", precision: str = "compensated",
                     reps: int = 5, stream=None) -> tuple[dict, float]:
    """Time every launch configuration on z (scratch outputs), install the best
    in the table entry that calls of this size use (inv_det_launch_op)."""
    dt = _dtype_code(z)
    n, zp = _planes(z, "z")
    inv = torch.empty_like(z, memory_format=torch.contiguous_format)
    det = torch.empty(z.shape[1:], dtype=z.dtype, device=z.device)
    best = L.Launch()
    ms = ctypes.c_float(0)
    rc = L.lib().polsar_autotune_inv_det(dt, _METHODS[method], _PRECS[precision], n, _ptr(z), zp, _ptr(inv),
                                         inv.stride(0), _ptr(det), reps, ctypes.byref(best), ctypes.byref(ms),
                                         _stream(stream))
    L.check(rc, "polsar_autotune_inv_det")
    return best.as_dict(), float(ms.value)


def compute_units() -> int:
    c = ctypes.c_int(0)
    L.check(L.lib().polsar_device_compute_units(ctypes.byref(c)), "polsar_device_compute_units")
    return c.value
