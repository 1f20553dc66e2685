"""Shared test helpers: tolerances and error reductions against the oracle."""
import numpy as np

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def tol_f64_comp(kappa):
    """FP64 compensated: 1e-12 relative up to kappa 1e6 (the stated bar);
    above it the Dot2 error term grows like u^2 kappa^2, so the bar is
    widened by (kappa/1e6)^2."""
    k = np.asarray(kappa, dtype=np.float64)
    return 1e-12 * np.maximum(1.0, (k / 1e6) ** 2)


def tol_f32(kappa):
    """FP32 bar: 2e-6 * kappa."""
    return 2e-6 * np.asarray(kappa, dtype=np.float64)


def tol_plain(u, kappa, c=64.0):
    """Plain-form comparison rows: the adjugate's error grows like u kappa^2
    when two eigenvalues are small; Cholesky's is below that."""
    k = np.asarray(kappa, dtype=np.float64)
    return c * u * np.maximum(k, 1.0) ** 2


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def flat9(a):
    return np.asarray(a, dtype=np.float64).reshape(9, -1)


W9 = np.array([1, 1, 1, 2, 2, 2, 2, 2, 2], dtype=np.float64)[:, None]  # Frobenius weights of the packing


def oracle_z_storage(zh, zl, mag, n_terms, u):
    """The oracle's multilook Z rounded to the storage type (unit roundoff u),
    and delta bounding the relative Frobenius distance from it to any Z that
    meets the fused kernels' Z check (u |Z| + (4 n + 4) u64 mag per
    component).  A fused kernel inverts its own Z, so its inverse may differ
    from the oracle's inverse of this Z by about kappa * delta on top of the
    inversion tolerance; both are computed from oracle values only."""
    z = zh + zl
    zt = z.astype(np.float32).astype(np.float64) if u == U32 else z
    comp = 2 * u * np.abs(zh) + (4 * n_terms + 4) * U64 * mag
    delta = np.sqrt((W9 * comp * comp).sum(0)) / np.sqrt((W9 * zh * zh).sum(0))
    return zt, delta
