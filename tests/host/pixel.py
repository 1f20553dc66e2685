"""ctypes access to the host build of the per-pixel compensated arithmetic."""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libpixel_host.so")
_L = None


def lib():
    global _L
    if _L is None:
        src = os.path.join(HERE, "pixel_host.cpp")
        hdr = os.path.join(HERE, "..", "..", "paper_1807_08084_amd", "csrc", "pixel.hpp")
        if not os.path.exists(SO) or os.path.getmtime(SO) < max(os.path.getmtime(src), os.path.getmtime(hdr)):
            tmp = SO + ".tmp"
            subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp",
                                   "-ffp-contract=off", "-o", tmp, src])
            os.replace(tmp, SO)
        L = ctypes.CDLL(SO)
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        L.host_adjugate_comp_f32.argtypes = [i64, vp, i64, vp, vp, vp, vp, ctypes.c_int]
        L.host_adjugate_comp_f32.restype = i64
        L.host_adjugate_comp_f64.argtypes = [i64, vp, i64, vp, vp, vp, ctypes.c_int]
        L.host_adjugate_comp_f64.restype = i64
        L.host_det_plain_bound_f32.argtypes = [i64, vp, i64, vp, vp, ctypes.c_int]
        L.host_det_plain_bound_f32.restype = None
        L.host_sum_pair_f32.argtypes = [i64, vp, vp, vp, vp, ctypes.c_int]
        L.host_sum_pair_f32.restype = None
        L.host_diag_cofactors_f32.argtypes = [i64, vp, i64, vp, vp, vp]
        L.host_diag_cofactors_f32.restype = None
        _L = L
    return _L


def _threads():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def adjugate_comp_f32(z):
    z = np.ascontiguousarray(np.asarray(z, dtype=np.float32).reshape(9, -1))
    n = z.shape[1]
    inv, det = np.empty((9, n), np.float32), np.empty(n, np.float32)
    st, bound = np.empty(n, np.uint8), np.empty(n, np.float32)
    lib().host_adjugate_comp_f32(n, _p(z), n, _p(inv), _p(det), _p(st), _p(bound), _threads())
    return inv, det, st, bound


def adjugate_comp_f64(z):
    z = np.ascontiguousarray(np.asarray(z, dtype=np.float64).reshape(9, -1))
    n = z.shape[1]
    inv, det, st = np.empty((9, n)), np.empty(n), np.empty(n, np.uint8)
    lib().host_adjugate_comp_f64(n, _p(z), n, _p(inv), _p(det), _p(st), _threads())
    return inv, det, st


def det_plain_bound_f32(z):
    """Plain FP32 determinant and its a-priori error bound (host build)."""
    z = np.ascontiguousarray(np.asarray(z, dtype=np.float32).reshape(9, -1))
    n = z.shape[1]
    det, bound = np.empty(n, np.float32), np.empty(n, np.float32)
    lib().host_det_plain_bound_f32(n, _p(z), n, _p(det), _p(bound), _threads())
    return det, bound


def sum_pair_f32(a, b, fast):
    """(s, e) of the kernels' TwoSum (fast False) or FastTwoSum (fast True)."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    s, e = np.empty_like(a), np.empty_like(a)
    lib().host_sum_pair_f32(a.size, _p(a), _p(b), _p(s), _p(e), 1 if fast else 0)
    return s, e


def diag_cofactors_f32(z):
    """The diagonal cofactors (hi, lo) of the FP32 step and its order flag."""
    z = np.ascontiguousarray(np.asarray(z, dtype=np.float32).reshape(9, -1))
    n = z.shape[1]
    hi, lo, ordered = np.empty((3, n), np.float32), np.empty((3, n), np.float32), np.empty(n, np.uint8)
    lib().host_diag_cofactors_f32(n, _p(z), n, _p(hi), _p(lo), _p(ordered))
    return hi, lo, ordered.astype(bool)
