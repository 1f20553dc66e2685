"""Seeded synthetic PolSAR covariance images.

This module is the only code shared by the GPU path's tests and the CPU
oracle's tests: it draws inputs and holds none of the inversion or
determinant arithmetic.

Model (Introduction, Eq. (ZN) and the Wishart model it cites): each pixel
has N independent looks S(l) in C^3 drawn circular complex Gaussian with
covariance Sigma, and the multilook covariance is Z = (1/N) sum_l S(l) S(l)^H
(the outer product; the equation prints S^H S, a scalar, which cannot be
meant).  Z is a 3x3 Hermitian positive semi-definite matrix, positive
definite almost surely when N >= 3.

Storage: the upper triangle (Section 2.1: a, d, f real on the diagonal, b, c,
e complex above it) as nine real planes in the order

    0:a  1:d  2:f  3:Re b  4:Im b  5:Re c  6:Im c  7:Re e  8:Im e

Recipe:
  * Sigma_c = U diag(lam) U^H with U Haar-distributed on U(3): Gram-Schmidt
    of a complex Ginibre matrix, which equals QR with a positive real
    diagonal in R (Mezzadri, "How to generate random matrices from the
    classical compact groups", 2007).  lam_k = exp(Uniform(ln lo, ln hi)).
  * Looks S = U diag(sqrt(lam)) w, w_k = (x + i y)/sqrt(2), x, y ~ N(0, 1).
    The square-root factor U diag(sqrt(lam)) needs no factorisation.
  * The image is an Ry x Rx grid of equal regions; pixel (y, x) belongs to
    region (floor(y Ry / H), floor(x Rx / W)).  With per_pixel=True each
    pixel draws its own U and lam instead.
  * Pixels are drawn in fixed chunks of CHUNK pixels (row-major order), each
    chunk from its own SeedSequence child, so the image does not depend on
    how the work is split.
  * FP32 inputs are the round-to-nearest FP32 rounding of the FP64 planes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

CHUNK = 1 << 18
PLANES = ("a", "d", "f", "br", "bi", "cr", "ci", "er", "ei")


def haar_unitary(rng: np.random.Generator, m: int) -> np.ndarray:
    """m Haar-random 3x3 unitaries, shape (m, 3, 3), columns orthonormal."""
    g = (rng.standard_normal((m, 3, 3)) + 1j * rng.standard_normal((m, 3, 3))) / math.sqrt(2.0)
    q = np.empty_like(g)
    for k in range(3):
        v = g[:, :, k].copy()
        for j in range(k):  # modified Gram-Schmidt
            proj = np.sum(np.conj(q[:, :, j]) * v, axis=1)
            v -= proj[:, None] * q[:, :, j]
        q[:, :, k] = v / np.linalg.norm(v, axis=1)[:, None]
    return q


def loguniform(rng: np.random.Generator, lo: float, hi: float, shape) -> np.ndarray:
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=shape))


def pack(zfull: np.ndarray) -> np.ndarray:
    """(m, 3, 3) Hermitian -> (9, m) real planes in the storage order above."""
    return np.stack([
        zfull[:, 0, 0].real, zfull[:, 1, 1].real, zfull[:, 2, 2].real,
        zfull[:, 0, 1].real, zfull[:, 0, 1].imag,
        zfull[:, 0, 2].real, zfull[:, 0, 2].imag,
        zfull[:, 1, 2].real, zfull[:, 1, 2].imag,
    ])


def unpack(planes: np.ndarray) -> np.ndarray:
    """(9, ...) real planes -> (..., 3, 3) complex Hermitian (exact)."""
    p = np.asarray(planes, dtype=np.float64)
    shp = p.shape[1:]
    z = np.empty(shp + (3, 3), dtype=np.complex128)
    a, d, f, br, bi, cr, ci, er, ei = p
    b, c, e = br + 1j * bi, cr + 1j * ci, er + 1j * ei
    z[..., 0, 0] = a
    z[..., 1, 1] = d
    z[..., 2, 2] = f
    z[..., 0, 1] = b
    z[..., 1, 0] = np.conj(b)
    z[..., 0, 2] = c
    z[..., 2, 0] = np.conj(c)
    z[..., 1, 2] = e
    z[..., 2, 1] = np.conj(e)
    return z


def _multilook(rng: np.random.Generator, root: np.ndarray, n_looks: int, looks_out=None) -> np.ndarray:
    """Packed Z = (1/N) sum_l S S^H with S = root w, w ~ CN(0, I); root (m, 3, 3).

    Returns (9, m) planes; the diagonal is summed as |S_i|^2, exactly real.
    If ``looks_out`` (6N, m) is given, the looks are written there: plane
    6l + 2i + 0/1 = Re/Im of component i (HH, HV, VV) of look l.
    """
    m = root.shape[0]
    w = (rng.standard_normal((m, n_looks, 3)) + 1j * rng.standard_normal((m, n_looks, 3))) / math.sqrt(2.0)
    s = [root[:, None, i, 0] * w[:, :, 0] + root[:, None, i, 1] * w[:, :, 1]
         + root[:, None, i, 2] * w[:, :, 2] for i in range(3)]
    if looks_out is not None:
        for ll in range(n_looks):
            for i in range(3):
                looks_out[6 * ll + 2 * i] = s[i][:, ll].real
                looks_out[6 * ll + 2 * i + 1] = s[i][:, ll].imag
    out = np.empty((9, m), dtype=np.float64)
    for k in range(3):
        out[k] = (s[k].real ** 2 + s[k].imag ** 2).sum(axis=1) / n_looks
    for k, (i, j) in enumerate(((0, 1), (0, 2), (1, 2))):
        p = (s[i] * np.conj(s[j])).sum(axis=1) / n_looks
        out[3 + 2 * k] = p.real
        out[4 + 2 * k] = p.imag
    return out


def _workers() -> int:
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


@dataclass
class Image:
    planes: np.ndarray          # (9, H, W) float64 (or float32 after .astype)
    n_looks: int
    sigma_regions: np.ndarray   # (R, 3, 3) complex, the regional covariances
    region_of: np.ndarray | None = None  # (H, W) int region index (None if per-pixel)
    looks: np.ndarray | None = None      # (6N, H, W) float64 single-look vectors, if requested


def make_image(H: int, W: int, n_looks: int, regions=(2, 2), lam_range=(1e-2, 1.0),
               seed=0, per_pixel: bool = False, rows: tuple[int, int] | None = None,
               with_looks: bool = False) -> Image:
    """Draw one synthetic multilook image; see the module docstring.

    ``seed`` is an int or a numpy SeedSequence.  ``rows=(y0, y1)`` draws only
    that row band (identical to the same rows of the full image).
    """
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    ss_reg, ss_pix = ss.spawn(2)
    Ry, Rx = regions
    R = Ry * Rx
    rng_r = np.random.default_rng(ss_reg)
    U = haar_unitary(rng_r, R)
    lam = loguniform(rng_r, lam_range[0], lam_range[1], (R, 3))
    sig = np.einsum("rij,rj,rkj->rik", U, lam, np.conj(U))
    root_r = U * np.sqrt(lam)[:, None, :]

    n = H * W
    y0, y1 = (0, H) if rows is None else rows
    p0, p1 = y0 * W, y1 * W
    nchunks = (n + CHUNK - 1) // CHUNK
    children = ss_pix.spawn(nchunks)
    out = np.empty((9, p1 - p0), dtype=np.float64)
    looks = np.empty((6 * n_looks, p1 - p0), dtype=np.float64) if with_looks else None

    def chunk(k: int) -> None:
        c0, c1 = k * CHUNK, min(n, (k + 1) * CHUNK)
        rng = np.random.default_rng(children[k])
        m = c1 - c0
        if per_pixel:
            Up = haar_unitary(rng, m)
            lp = loguniform(rng, lam_range[0], lam_range[1], (m, 3))
            root = Up * np.sqrt(lp)[:, None, :]
        else:
            idx = np.arange(c0, c1)
            reg = (idx // W * Ry // H) * Rx + (idx % W * Rx // W)
            root = root_r[reg]
        lk = np.empty((6 * n_looks, c1 - c0)) if with_looks else None
        z = _multilook(rng, root, n_looks, lk)
        s0, s1 = max(c0, p0), min(c1, p1)
        out[:, s0 - p0:s1 - p0] = z[:, s0 - c0:s1 - c0]
        if with_looks:
            looks[:, s0 - p0:s1 - p0] = lk[:, s0 - c0:s1 - c0]

    ks = range(p0 // CHUNK, (p1 + CHUNK - 1) // CHUNK) if p1 > p0 else range(0)
    if len(ks) > 1:
        from concurrent.futures import ThreadPoolExecutor  # numpy releases the GIL here
        with ThreadPoolExecutor(_workers()) as ex:
            list(ex.map(chunk, ks))
    else:
        for k in ks:
            chunk(k)
    region_of = None
    if not per_pixel:
        yy, xx = np.meshgrid(np.arange(y0, y1), np.arange(W), indexing="ij")
        region_of = (yy * Ry // H) * Rx + (xx * Rx // W)
    if with_looks:
        looks = looks.reshape(6 * n_looks, y1 - y0, W)
    return Image(out.reshape(9, y1 - y0, W), n_looks, sig, region_of, looks)


def wishart_sigma0(z_planes: np.ndarray, ridge: float = 0.1) -> np.ndarray:
    """Initial parameter Sigma = Z + ridge * tr(Z)/3 * I on packed planes."""
    s = np.array(z_planes, dtype=np.float64, copy=True)
    tr = s[0] + s[1] + s[2]
    for k in range(3):
        s[k] = s[k] + ridge * tr / 3.0
    return s


# ---------------------------------------------------------------- workloads
# The workloads: shapes, looks, region grids and eigenvalue ranges.

def workload_small(seed=0):
    """256x256, N=4, 2x2 regions, lam in [1e-2, 1]."""
    return make_image(256, 256, 4, (2, 2), (1e-2, 1.0), seed)


def workload_scale(seed=1, rows=None, with_looks=False):
    """4096x4096, N=4, 4x4 regions, lam in [1e-3, 1]."""
    return make_image(4096, 4096, 4, (4, 4), (1e-3, 1.0), seed, rows=rows, with_looks=with_looks)


def workload_scale8192(seed=5, rows=None):
    """8192x8192 with the 4096x4096 recipe: N=4, 4x4 regions, lam in [1e-3, 1]."""
    return make_image(8192, 8192, 4, (4, 4), (1e-3, 1.0), seed, rows=rows)


def workload_boxcar(seed=4, side=4096):
    """Single-look image for the boxcar multilook: side x side, 4x4 regions,
    lam in [1e-3, 1]; returns the (6, side*side) FP64 planes of S."""
    return make_image(side, side, 1, (4, 4), (1e-3, 1.0), seed, with_looks=True).looks.reshape(6, -1)


def workload_precision(seed=2, side=8192, rows=None):
    """8192x8192, N=3, per-pixel Sigma with lam in [1e-8, 1]."""
    return make_image(side, side, 3, (1, 1), (1e-8, 1.0), seed, per_pixel=True, rows=rows)


def workload_wishart(seed=3, side=2048, rows=None):
    """2048x2048, N=8, Z as the small workload (2x2 regions, lam in [1e-2, 1])."""
    img = make_image(side, side, 8, (2, 2), (1e-2, 1.0), seed, rows=rows)
    return img, wishart_sigma0(img.planes)


def batch_shapes(seed=7, count=64):
    """Sides log-uniform in [128, 4096] (H and W independent) and N from {3,4,8,16}."""
    rng = np.random.default_rng(seed)
    hw = np.rint(np.exp(rng.uniform(math.log(128), math.log(4096), size=(count, 2)))).astype(np.int64)
    looks = rng.choice(np.array([3, 4, 8, 16]), count)
    return [(int(h), int(w), int(n)) for (h, w), n in zip(hw, looks)]


def workload_batch(seed=7, count=64, max_images=None):
    """64 images of uneven shapes, 2x4 regions each, lam in [1e-2, 1]."""
    shapes = batch_shapes(seed, count)
    kids = np.random.SeedSequence(seed).spawn(count)
    sel = range(count if max_images is None else min(count, max_images))
    return [make_image(shapes[i][0], shapes[i][1], shapes[i][2], (2, 4), (1e-2, 1.0), kids[i]) for i in sel]


# ------------------------------------------------------------ the paper's shapes
# Stand-ins for the inputs of the paper's timing experiment (Section 4 and
# Table 2), for quoting beside its numbers: simulated matrices M M^H with the
# real and imaginary parts of the 3x3 M independent uniform on [-1, 1]
# (5,469,354 of them), and a 450 x 600 image in place of the AIRSAR scene
# (the small workload's recipe at that shape; the scene itself is not here).
PAPER_SIMULATED_COUNT = 5_469_354


def workload_paper_simulated(seed=6, count=PAPER_SIMULATED_COUNT) -> np.ndarray:
    """(9, count) FP64 planes of M M^H, drawn in fixed chunks of CHUNK
    matrices, one SeedSequence child each."""
    out = np.empty((9, count))
    kids = np.random.SeedSequence(seed).spawn((count + CHUNK - 1) // CHUNK)

    def chunk(k: int) -> None:
        c0, c1 = k * CHUNK, min(count, (k + 1) * CHUNK)
        rng = np.random.default_rng(kids[k])
        m = rng.uniform(-1.0, 1.0, (c1 - c0, 3, 3)) + 1j * rng.uniform(-1.0, 1.0, (c1 - c0, 3, 3))
        out[:, c0:c1] = pack(m @ np.conj(np.transpose(m, (0, 2, 1))))

    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(chunk, range(len(kids))))
    return out


def workload_airsar_standin(seed=8):
    """450 x 600, N=4, 2x2 regions, lam in [1e-2, 1]."""
    return make_image(450, 600, 4, (2, 2), (1e-2, 1.0), seed)
