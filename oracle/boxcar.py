"""Oracle of the spatial (boxcar) multilook of a single-look PolSAR image.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. (ZN) forms Z as the mean of N outer products S S^H of single-look
scattering vectors S = (S_HH, S_HV, S_VV).  In the boxcar form the N looks
of pixel (y, x) are the single-look pixels of its (2r+1) x (2r+1)
neighbourhood, clipped at the image border:

    Z(y, x) = (1 / |W|) sum_{(y', x') in W(y, x)} S(y', x') S(y', x')^H,
    W(y, x) = [max(0, y-r), min(H-1, y+r)] x [max(0, x-r), min(W-1, x+r)].

Two independent constructions:
  * boxcar128 -- gathers each pixel's window as its looks and hands them to
                 the pinned __float128 multilook oracle (multilook128);
  * boxcar64  -- plain FP64 numpy: for every window offset, adds the shifted
                 outer-product planes where the neighbour exists, then
                 divides by the count.
Single-look planes are (6, H*W): Re S_HH, Im S_HH, Re S_HV, Im S_HV,
Re S_VV, Im S_VV; Z is packed as everywhere else (a, d, f, Re b, Im b,
Re c, Im c, Re e, Im e) with b = S_HH conj(S_HV), c = S_HH conj(S_VV),
e = S_HV conj(S_VV).
"""
from __future__ import annotations

import numpy as np

from . import multilook128


def window_counts(H: int, W: int, r: int) -> np.ndarray:
    """|W(y, x)| for every pixel, (H*W,): clipped rows times clipped columns."""
    ys, xs = np.arange(H), np.arange(W)
    rows = np.minimum(H - 1, ys + r) - np.maximum(0, ys - r) + 1
    cols = np.minimum(W - 1, xs + r) - np.maximum(0, xs - r) + 1
    return (rows[:, None] * cols[None, :]).reshape(-1)


def outer_planes(s: np.ndarray) -> np.ndarray:
    """S S^H packed, (9, n), in FP64 from (6, n) single-look planes."""
    hr, hi, vr, vi, wr, wi = np.asarray(s, dtype=np.float64)
    return np.stack([hr * hr + hi * hi, vr * vr + vi * vi, wr * wr + wi * wi,
                     hr * vr + hi * vi, hi * vr - hr * vi,
                     hr * wr + hi * wi, hi * wr - hr * wi,
                     vr * wr + vi * wi, vi * wr - vr * wi])


def boxcar64(s: np.ndarray, H: int, W: int, r: int) -> np.ndarray:
    """Z of every pixel in FP64, (9, H*W)."""
    o = outer_planes(s).reshape(9, H, W)
    acc = np.zeros((9, H, W))
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            # pixels (y, x) whose neighbour (y+dy, x+dx) lies in the image
            y0, y1 = max(0, -dy), min(H, H - dy)
            x0, x1 = max(0, -dx), min(W, W - dx)
            if y0 < y1 and x0 < x1:
                acc[:, y0:y1, x0:x1] += o[:, y0 + dy:y1 + dy, x0 + dx:x1 + dx]
    return acc.reshape(9, -1) / window_counts(H, W, r)


def boxcar128(s: np.ndarray, H: int, W: int, r: int, pixels=None):
    """Z of the given pixels (default all) in __float128 through the
    multilook oracle: ((z_hi, z_lo) (9, m), mag (9, m)), mag bounding the
    mean of |terms| (as multilook128 returns it)."""
    s = np.asarray(s, dtype=np.float64).reshape(6, H * W)
    pix = np.arange(H * W) if pixels is None else np.asarray(pixels, dtype=np.int64)
    counts = window_counts(H, W, r)[pix]
    m = pix.size
    zh, zl, mag = np.empty((9, m)), np.empty((9, m)), np.empty((9, m))
    for n_looks in np.unique(counts):
        sel = np.nonzero(counts == n_looks)[0]
        p = pix[sel]
        y, x = p // W, p % W
        looks = np.empty((6 * n_looks, sel.size))
        for j in range(sel.size):
            yy = np.arange(max(0, y[j] - r), min(H - 1, y[j] + r) + 1)
            xx = np.arange(max(0, x[j] - r), min(W - 1, x[j] + r) + 1)
            win = (yy[:, None] * W + xx[None, :]).reshape(-1)
            looks[:, j] = s[:, win].T.reshape(-1)  # look l -> planes 6l..6l+5
        (h, lo), mg = multilook128(looks, int(n_looks))
        zh[:, sel], zl[:, sel], mag[:, sel] = h, lo, mg
    return (zh, zl), mag
