"""CPU oracle for the 3x3 Hermitian inverse, determinant and Wishart term.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package; the GPU library and its
Python binding never do, and the two share no code.

``liboracle.so`` is built from ``oracle.cpp`` by :func:`build` (g++, OpenMP,
libquadmath, ``-ffp-contract=off``).  Python side: thin ctypes marshalling of
numpy arrays; plane layout (9, n) float64, the upper triangle in the order
a, d, f, Re b, Im b, Re c, Im c, Re e, Im e (Section 2.1).

Functions and the passages they follow:
  * ge / ge128       -- inverse and det from the plain definition A X = I by
                        complex Gaussian elimination with partial pivoting and
                        back substitution.
  * chol / chol128   -- the Cholesky form (Section 2.2 relations, Alg. 1) with
                        the conjugation of l21 corrected.
  * pd_class         -- positive-definiteness by the signs of the squared
                        Cholesky pivots in __float128 (Section 3.1's full-rank
                        check, made a sign check).
  * multilook128      -- Z = (1/N) sum_l S(l) S(l)^H from single-look vectors
                        (Introduction, Eq. (ZN), the outer product).
  * wishart / wishart128 -- N (ln det S + tr(S^-1 Z)) and its gradient
                        N (S^-1 - S^-1 Z S^-1) in the packed real convention
                        (Introduction: the densities depend on the covariance
                        through its determinant and inverse).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.cpp")
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so in place (g++, no GPU code)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lquadmath"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        i64, dp, u8p, c_int = ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int
        L.oracle_ge_f64.argtypes = [i64, dp, i64, dp, i64, dp, dp, c_int]
        L.oracle_ge_f128.argtypes = [i64, dp, i64, dp, dp, i64, dp, dp, dp, c_int]
        L.oracle_chol_f64.argtypes = [i64, dp, i64, dp, i64, dp, dp, c_int]
        L.oracle_chol_f128.argtypes = [i64, dp, i64, dp, dp, i64, dp, dp, c_int]
        L.oracle_pd_class.argtypes = [i64, dp, i64, u8p, c_int]
        L.oracle_wishart_f64.argtypes = [i64, dp, i64, dp, i64, ctypes.c_double, dp, dp, i64, c_int]
        L.oracle_wishart_f128.argtypes = [i64, dp, i64, dp, i64, ctypes.c_double, dp, dp, dp, dp, i64, c_int]
        L.oracle_multilook_f128.argtypes = [i64, dp, i64, c_int, dp, dp, i64, dp, c_int]
        for f in ("oracle_ge_f64", "oracle_ge_f128", "oracle_chol_f64", "oracle_chol_f128",
                  "oracle_pd_class", "oracle_wishart_f64", "oracle_wishart_f128", "oracle_multilook_f128"):
            getattr(L, f).restype = i64
        _lib = L
    return _lib


def threads() -> int:
    return len(os.sched_getaffinity(0))


def _planes(z) -> np.ndarray:
    z = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
    if z.shape[0] != 9:
        raise ValueError("expected 9 planes")
    return z.reshape(9, -1)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def ge(z, nthreads=None, checks=False):
    """FP64 brute force. Returns (inv (9,n), det (n,)[, chk (2,n)])."""
    z = _planes(z)
    n = z.shape[1]
    inv = np.empty((9, n))
    det = np.empty(n)
    chk = np.empty((2, n)) if checks else None
    lib().oracle_ge_f64(n, _p(z), n, _p(inv), n, _p(det), _p(chk) if checks else None,
                        nthreads or threads())
    return (inv, det, chk) if checks else (inv, det)


def ge128(z, nthreads=None, checks=False):
    """__float128 brute force. Returns ((inv_hi, inv_lo), (det_hi, det_lo)[, chk])."""
    z = _planes(z)
    n = z.shape[1]
    ih, il = np.empty((9, n)), np.empty((9, n))
    dh, dl = np.empty(n), np.empty(n)
    chk = np.empty((2, n)) if checks else None
    lib().oracle_ge_f128(n, _p(z), n, _p(ih), _p(il), n, _p(dh), _p(dl),
                         _p(chk) if checks else None, nthreads or threads())
    return ((ih, il), (dh, dl), chk) if checks else ((ih, il), (dh, dl))


def chol(z, nthreads=None, pivots=False):
    """FP64 Cholesky form. Returns (inv, det[, piv2 (3,n)])."""
    z = _planes(z)
    n = z.shape[1]
    inv, det = np.empty((9, n)), np.empty(n)
    piv = np.empty((3, n)) if pivots else None
    lib().oracle_chol_f64(n, _p(z), n, _p(inv), n, _p(det), _p(piv) if pivots else None,
                          nthreads or threads())
    return (inv, det, piv) if pivots else (inv, det)


def chol128(z, nthreads=None):
    z = _planes(z)
    n = z.shape[1]
    ih, il = np.empty((9, n)), np.empty((9, n))
    dh, dl = np.empty(n), np.empty(n)
    lib().oracle_chol_f128(n, _p(z), n, _p(ih), _p(il), n, _p(dh), _p(dl), nthreads or threads())
    return (ih, il), (dh, dl)


def pd_class(z, nthreads=None) -> np.ndarray:
    """uint8 per pixel: 0 positive definite, 2 not, 3 non-finite input."""
    z = _planes(z)
    n = z.shape[1]
    cls = np.empty(n, dtype=np.uint8)
    lib().oracle_pd_class(n, _p(z), n, _p(cls), nthreads or threads())
    return cls


def wishart(sigma, z, n_looks, nthreads=None, grad=True):
    """FP64 per-pixel ell (n,) and packed gradient (9, n)."""
    s, zz = _planes(sigma), _planes(z)
    n = s.shape[1]
    ell = np.empty(n)
    g = np.empty((9, n)) if grad else None
    lib().oracle_wishart_f64(n, _p(s), n, _p(zz), n, float(n_looks), _p(ell),
                             _p(g) if grad else None, n, nthreads or threads())
    return ell, g


def wishart128(sigma, z, n_looks, nthreads=None, grad=True):
    """__float128 per-pixel ell and gradient, each as a (hi, lo) pair."""
    s, zz = _planes(sigma), _planes(z)
    n = s.shape[1]
    eh, el = np.empty(n), np.empty(n)
    gh = np.empty((9, n)) if grad else None
    gl = np.empty((9, n)) if grad else None
    lib().oracle_wishart_f128(n, _p(s), n, _p(zz), n, float(n_looks), _p(eh), _p(el),
                              _p(gh) if grad else None, _p(gl) if grad else None, n,
                              nthreads or threads())
    return (eh, el), ((gh, gl) if grad else None)


def multilook128(looks, n_looks, nthreads=None):
    """Z = (1/N) sum S S^H in __float128 from (6N, ...) look planes.
    Returns ((z_hi, z_lo) (9, n), mag (9, n)) with mag bounding sum|terms|/N."""
    lk = np.ascontiguousarray(np.asarray(looks, dtype=np.float64))
    if lk.shape[0] != 6 * n_looks:
        raise ValueError("expected 6N look planes")
    lk = lk.reshape(6 * n_looks, -1)
    n = lk.shape[1]
    zh, zl, mag = np.empty((9, n)), np.empty((9, n)), np.empty((9, n))
    lib().oracle_multilook_f128(n, _p(lk), n, int(n_looks), _p(zh), _p(zl), n, _p(mag), nthreads or threads())
    return (zh, zl), mag


# ------------------------------------------------------------ error metrics
def full_from_planes(p: np.ndarray) -> np.ndarray:
    """(9, n) -> (n, 3, 3) complex Hermitian, exact."""
    a, d, f, br, bi, cr, ci, er, ei = p
    n = p.shape[1]
    X = np.empty((n, 3, 3), dtype=np.complex128)
    X[:, 0, 0], X[:, 1, 1], X[:, 2, 2] = a, d, f
    X[:, 0, 1] = br + 1j * bi
    X[:, 0, 2] = cr + 1j * ci
    X[:, 1, 2] = er + 1j * ei
    X[:, 1, 0] = np.conj(X[:, 0, 1])
    X[:, 2, 0] = np.conj(X[:, 0, 2])
    X[:, 2, 1] = np.conj(X[:, 1, 2])
    return X


_WEIGHT = np.array([1, 1, 1, 2, 2, 2, 2, 2, 2], dtype=np.float64)[:, None]


def inv_rel_err(x, ref_hi, ref_lo=None) -> np.ndarray:
    """Per-pixel ||X - X_ref||_F / ||X_ref||_F over the full Hermitian matrix
    (off-diagonal components count twice), reference as hi (+ lo)."""
    x = np.asarray(x, dtype=np.float64).reshape(9, -1)
    diff = x - ref_hi
    if ref_lo is not None:
        diff = diff - ref_lo
    num = np.sqrt((_WEIGHT * diff * diff).sum(axis=0))
    den = np.sqrt((_WEIGHT * ref_hi * ref_hi).sum(axis=0))
    return num / den


def det_rel_err(d, ref_hi, ref_lo=None) -> np.ndarray:
    d = np.asarray(d, dtype=np.float64).reshape(-1)
    diff = d - ref_hi
    if ref_lo is not None:
        diff = diff - ref_lo
    return np.abs(diff) / np.abs(ref_hi)


def kappa(z) -> np.ndarray:
    """2-norm condition number of each stored matrix (FP64 eigvalsh)."""
    w = np.linalg.eigvalsh(full_from_planes(_planes(z)))
    with np.errstate(divide="ignore", invalid="ignore"):
        k = w[:, -1] / w[:, 0]
    return np.where(w[:, 0] > 0, k, np.inf)
