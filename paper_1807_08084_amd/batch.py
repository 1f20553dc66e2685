"""Batched launch over many images (one HIP graph)."""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from .ops import _METHODS, _PRECS, _dtype_code, _planes, _ptr, _stream, empty_planes


class BatchPlan:
    """Inverse/determinant of each image's Z and the Wishart term/gradient of
    its S against the same Z, for many images in one launch (one block per
    tile, or a persistent grid: the op-3 entry of the launch table).

    ``images``: list of dicts with keys ``z`` (9, ...) and, for the Wishart
    ops, ``sigma`` (same shape) and ``n_looks``.  Output tensors are allocated
    here and exposed as ``inv[i]``, ``det[i]``, ``status[i]``, ``grad[i]``,
    ``ell[i]`` and ``loss`` (float64, one per image).
    """

    def __init__(self, images, method="adjugate", precision="compensated", inv_det=True,
                 wishart_fwd=True, wishart_bwd=True, status=True, ell=False, grad_loss=None,
                 counters=None, grid_per_cu=0):
        if not images:
            raise ValueError("no images")
        dev = images[0]["z"].device
        dtype = images[0]["z"].dtype
        self.ops = (L.OP_INV_DET if inv_det else 0) | (L.OP_WISHART_FWD if wishart_fwd else 0) | \
                   (L.OP_WISHART_BWD if wishart_bwd else 0)
        self.inputs = images
        self.inv, self.det, self.status, self.grad, self.ell = [], [], [], [], []
        self.loss = torch.zeros(len(images), dtype=torch.float64, device=dev)
        self.grad_loss = grad_loss
        self.counters = counters
        arr = (L.Image * len(images))()
        for i, im in enumerate(images):
            z = im["z"]
            if z.dtype != dtype or z.device != dev:
                raise ValueError("all images must share dtype and device")
            n, zp = _planes(z, "z")
            r = arr[i]
            r.n, r.z, r.z_pitch = n, z.data_ptr(), zp
            shape = z.shape[1:]
            inv = det = None
            if inv_det:
                out = empty_planes(10, shape, dtype, dev)  # 9 inverse planes + det, one pitch
                inv, det = out[:9], out[9]
            st = torch.empty(shape, dtype=torch.uint8, device=dev) if (inv_det and status) else None
            self.inv.append(inv)
            self.det.append(det)
            self.status.append(st)
            if inv is not None:
                r.inv, r.inv_pitch = inv.data_ptr(), inv.stride(0)
            if det is not None:
                r.det = det.data_ptr()
            if st is not None:
                r.status = st.data_ptr()
            g = el = None
            if wishart_fwd or wishart_bwd:
                s = im["sigma"]
                ns, sp = _planes(s, "sigma")
                if ns != n or s.dtype != dtype:
                    raise ValueError("sigma must match z")
                r.sigma, r.s_pitch, r.n_looks = s.data_ptr(), sp, float(im["n_looks"])
                if wishart_bwd:
                    g = empty_planes(9, shape, dtype, dev)
                    r.grad, r.g_pitch = g.data_ptr(), g.stride(0)
                if wishart_fwd:
                    r.loss = self.loss.data_ptr() + 8 * i
                    if ell:
                        el = torch.empty(shape, dtype=dtype, device=dev)
                        r.ell = el.data_ptr()
            self.grad.append(g)
            self.ell.append(el)
        self._h = ctypes.c_void_p()
        rc = L.lib().polsar_batch_create(arr, len(images), _dtype_code(images[0]["z"]), _METHODS[method],
                                         _PRECS[precision], self.ops, _ptr(grad_loss), _ptr(counters),
                                         int(grid_per_cu), ctypes.byref(self._h))
        L.check(rc, "polsar_batch_create")

    @property
    def tiles(self) -> int:
        return int(L.lib().polsar_batch_tiles(self._h))

    def run(self, stream=None) -> None:
        """One graph launch on the stream (torch's current one by default)."""
        L.check(L.lib().polsar_batch_run(self._h, _stream(stream)), "polsar_batch_run")

    def run_eager(self, stream=None) -> None:
        L.check(L.lib().polsar_batch_run_eager(self._h, _stream(stream)), "polsar_batch_run_eager")

    def close(self) -> None:
        if self._h:
            L.lib().polsar_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
