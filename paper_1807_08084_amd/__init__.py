"""MI355X (gfx950) per-pixel inverse and determinant of 3x3 complex Hermitian
PolSAR covariance matrices (adjugate method, Cholesky for comparison), and the
Wishart log-likelihood with its adjoint.

The compute runs in libpolsar.so (hand-written HIP); this package is a thin
ctypes binding.  ``synth`` draws seeded inputs and needs no GPU.
"""
from . import synth  # noqa: F401

__all__ = ["inv_det", "multilook_inv_det", "wishart_loglik", "wishart_nll", "WishartNLL", "BatchPlan", "synth"]


def __getattr__(name):
    # the binding (and torch) load on first use, so the generator stays light
    if name in ("inv_det", "multilook_inv_det", "blockdiag_inv_det", "Streamer", "nlm_wishart", "upload_planes", "empty_planes", "recommended_pitch",
                "wishart_loglik", "wishart_nll", "WishartNLL", "autotune_inv_det",
                "get_launch", "set_launch", "stream_copy", "compute_units", "workspace_bytes"):
        from . import ops
        return getattr(ops, name)
    if name == "BatchPlan":
        from .batch import BatchPlan
        return BatchPlan
    raise AttributeError(name)
