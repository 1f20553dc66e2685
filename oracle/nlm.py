"""Oracle of the nonlocal-means filter with Wishart stochastic distances.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain FP64 numpy:
full complex matrices, numpy.linalg.inv / det for every pixel, then for each
window offset the distance between every pixel and its neighbour:

  symmetrized Kullback-Leibler  N/2 (tr(Zp^-1 Zq) + tr(Zq^-1 Zp)) - 3N
  Bhattacharyya                 N (ln det((Zp + Zq)/2) - (ln det Zp + ln det Zq)/2)

(the densities of the Introduction enter only through determinants and
inverses), weights exp(-d/h) over the window clipped at the border, and the
weighted mean of the neighbours' covariances.

The two distances between complex Wishart laws of equal looks N are those
of Frery, Nascimento and Cintra, "Analytic expressions for stochastic
distances between relaxed complex Wishart distributions", IEEE Trans.
Geosci. Remote Sens. 52(2), 2014.  The Bhattacharyya form follows from the
Wishart density: the integral of sqrt(f_p f_q) is |A|^-N / (|Zp||Zq|)^(N/2)
with A = (Zp^-1 + Zq^-1)/2, and |A| = |(Zp + Zq)/2| / (|Zp||Zq|) since
Zp^-1 + Zq^-1 = Zp^-1 (Zp + Zq) Zq^-1.
"""
from __future__ import annotations

import numpy as np

from . import full_from_planes


def distances(zp: np.ndarray, zq: np.ndarray, n_looks: float, distance: str) -> np.ndarray:
    """d between stacks of full Hermitian matrices (..., 3, 3)."""
    if distance == "kl":
        t1 = np.trace(np.linalg.inv(zp) @ zq, axis1=-2, axis2=-1).real
        t2 = np.trace(np.linalg.inv(zq) @ zp, axis1=-2, axis2=-1).real
        return n_looks / 2.0 * (t1 + t2) - 3.0 * n_looks
    ld = lambda m: np.log(np.linalg.det(m).real)  # noqa: E731
    return n_looks * (ld((zp + zq) / 2.0) - (ld(zp) + ld(zq)) / 2.0)


def nlm_wishart(z: np.ndarray, height: int, width: int, radius: int, n_looks: float, h: float,
                distance: str = "kl"):
    """z: (9, H*W) planes.  Returns (out (9, H*W), wsum (H*W,))."""
    Z = full_from_planes(np.asarray(z, dtype=np.float64).reshape(9, -1)).reshape(height, width, 3, 3)
    acc = np.zeros((height, width, 3, 3), dtype=np.complex128)
    wsum = np.zeros((height, width))
    for dy in range(-radius, radius + 1):
        for dx in range(-radius, radius + 1):
            y0, y1 = max(0, -dy), min(height, height - dy)
            x0, x1 = max(0, -dx), min(width, width - dx)
            if y0 >= y1 or x0 >= x1:
                continue
            zp = Z[y0:y1, x0:x1]
            zq = Z[y0 + dy:y1 + dy, x0 + dx:x1 + dx]
            w = np.exp(-distances(zp, zq, n_looks, distance) / h)
            acc[y0:y1, x0:x1] += w[..., None, None] * zq
            wsum[y0:y1, x0:x1] += w
    out = acc / wsum[..., None, None]
    m = out.reshape(-1, 3, 3)
    planes = np.stack([m[:, 0, 0].real, m[:, 1, 1].real, m[:, 2, 2].real, m[:, 0, 1].real, m[:, 0, 1].imag,
                       m[:, 0, 2].real, m[:, 0, 2].imag, m[:, 1, 2].real, m[:, 1, 2].imag])
    return planes, wsum.reshape(-1)
