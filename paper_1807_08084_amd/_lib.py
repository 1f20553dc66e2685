"""ctypes loader for libpolsar.so.  Fails loudly when the library is absent:
there is no CPU fallback."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libpolsar.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "polsar.h")

OK, E_ARG, E_ALIGN, E_UNSUPPORTED, E_HIP, E_WORKSPACE, E_ALIAS = 0, -1, -2, -3, -4, -5, -6
F32, F64 = 0, 1
ADJUGATE, CHOLESKY = 0, 1
PLAIN, COMPENSATED, WIDE = 0, 1, 2
FWD, BWD, FWD_BWD = 1, 2, 3
OP_INV_DET, OP_WISHART_FWD, OP_WISHART_BWD = 1, 2, 4
PX_OK, PX_REROUTED, PX_NOT_PD, PX_NONFINITE = 0, 1, 2, 3


class PolsarError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {status_string(code)} ({code})")


class Launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("unroll", ctypes.c_int),
                ("grid_per_cu", ctypes.c_int), ("nontemporal", ctypes.c_int),
                ("vector_bytes", ctypes.c_int), ("blocks_per_cu", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Image(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64),
                ("z", ctypes.c_void_p), ("z_pitch", ctypes.c_int64),
                ("inv", ctypes.c_void_p), ("inv_pitch", ctypes.c_int64),
                ("det", ctypes.c_void_p),
                ("status", ctypes.c_void_p),
                ("sigma", ctypes.c_void_p), ("s_pitch", ctypes.c_int64),
                ("grad", ctypes.c_void_p), ("g_pitch", ctypes.c_int64),
                ("ell", ctypes.c_void_p),
                ("loss", ctypes.c_void_p),
                ("n_looks", ctypes.c_double)]


_L = None


def lib():
    global _L
    if _L is None:
        if not os.path.exists(SO):
            raise RuntimeError(f"{SO} is not built; build it with __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950). There is no CPU fallback.")
        L = ctypes.CDLL(SO)
        i, i64, vp, d, sz = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_double, ctypes.c_size_t
        L.polsar_inv_det.argtypes = [i, i, i, i64, vp, i64, vp, i64, vp, vp, vp, vp]
        L.polsar_multilook_inv_det.argtypes = [i, i, i, i64, i, vp, i64, vp, i64, vp, i64, vp, vp, vp, vp]
        L.polsar_boxcar_inv_det.argtypes = [i, i, i, i64, i64, i, vp, i64, vp, i64, vp, i64, vp, vp, vp, vp]
        L.polsar_blockdiag_inv_det.argtypes = [i, i, i, i64, i, vp, i64, vp, i64, vp, vp, i64, vp, vp, vp]
        L.polsar_streamer_create.argtypes = [i, i, i, i64, ctypes.POINTER(vp)]
        L.polsar_streamer_run.argtypes = [vp, i64, vp, i64, vp, i64, vp, vp, vp]
        L.polsar_streamer_destroy.argtypes = [vp]
        L.polsar_streamer_destroy.restype = None
        L.polsar_nlm_wishart.argtypes = [i, i, i64, i64, i, d, d, vp, i64, vp, i64, vp, i64, vp, vp]
        L.polsar_wishart_loglik.argtypes = [i, i, i64, vp, i64, vp, i64, d, vp, vp, vp, vp, i64, vp, sz, vp, vp]
        L.polsar_wishart_workspace_bytes.argtypes = [i, i64]
        L.polsar_wishart_loglik_noalloc.argtypes = [i, i, i64, vp, i64, vp, i64, ctypes.c_double, vp, vp, vp, vp,
                                                    i64, vp, vp]
        L.polsar_wishart_workspace_bytes.restype = sz
        L.polsar_batch_create.argtypes = [ctypes.POINTER(Image), i, i, i, i, ctypes.c_uint, vp, vp, i,
                                          ctypes.POINTER(vp)]
        L.polsar_batch_run.argtypes = [vp, vp]
        L.polsar_batch_run_eager.argtypes = [vp, vp]
        L.polsar_batch_tiles.argtypes = [vp]
        L.polsar_batch_tiles.restype = i64
        L.polsar_batch_destroy.argtypes = [vp]
        L.polsar_batch_destroy.restype = None
        L.polsar_get_launch.argtypes = [i, i, i, i, ctypes.POINTER(Launch)]
        L.polsar_set_launch.argtypes = [i, i, i, i, ctypes.POINTER(Launch)]
        L.polsar_wishart_launch_op.argtypes = [i64]
        L.polsar_inv_det_launch_op.argtypes = [i64]
        L.polsar_autotune_inv_det.argtypes = [i, i, i, i64, vp, i64, vp, i64, vp, i, ctypes.POINTER(Launch),
                                              ctypes.POINTER(ctypes.c_float), vp]
        L.polsar_stream_copy.argtypes = [i, i64, vp, i64, i, vp, i64, i, vp]
        L.polsar_status_string.argtypes = [i]
        L.polsar_status_string.restype = ctypes.c_char_p
        L.polsar_version.argtypes = []
        L.polsar_version.restype = ctypes.c_char_p
        L.polsar_device_compute_units.argtypes = [ctypes.POINTER(ctypes.c_int)]
        L.polsar_recommended_pitch.argtypes = [i, i64]
        L.polsar_recommended_pitch.restype = i64
        _L = L
    return _L


def status_string(code: int) -> str:
    return lib().polsar_status_string(code).decode()


def check(code: int, what: str) -> None:
    if code != OK:
        raise PolsarError(code, what)


def declared_symbols() -> list[str]:
    """Function names declared in include/polsar.h."""
    import re
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(polsar_[a-z_0-9]+)\s*\(", text)))
