"""The kernels' compensated per-pixel arithmetic, compiled for the host (no GPU),
against the __float128 oracle on hard matrices: Haar-rotated, eigenvalues
(1, l2, 10^-k) with one or two small eigenvalues, kappa up to 1e10.

Checks the FP64 bar (1e-12 up to kappa 1e6), the FP32 bar (2e-6 kappa) after
rerouting, and that the a-posteriori determinant bound covers the true error
of every pixel that was not rerouted."""
import numpy as np
import pytest

import oracle
from paper_1807_08084_amd import synth
from _helpers import tol_f32, tol_f64_comp

pixel = pytest.importorskip("host.pixel")


def hard(rng, m, kmax=10.0):
    k = rng.uniform(0.0, kmax, size=m)
    lam3 = 10.0 ** -k
    two_small = rng.random(m) < 0.5
    lam2 = np.where(two_small, lam3 * 10.0 ** rng.uniform(0, 1, m), 10.0 ** -rng.uniform(0, 0.5, m))
    eig = np.stack([np.ones(m), lam2, lam3], axis=1)
    U = synth.haar_unitary(rng, m)
    Z = np.einsum("mij,mj,mkj->mik", U, eig, np.conj(U))
    return synth.pack(Z)


def test_f64_compensated_meets_1e12():
    rng = np.random.default_rng(31)
    z = hard(rng, 40000, 8.0)
    inv, det, st = pixel.adjugate_comp_f64(z)
    k = oracle.kappa(z)
    (ih, il), (dh, dl) = oracle.ge128(z)
    ok = k <= 1e8
    e_inv = oracle.inv_rel_err(inv, ih, il)
    e_det = oracle.det_rel_err(det, dh, dl)
    assert np.all(st[ok] == 0)
    assert np.all(e_inv[ok] <= tol_f64_comp(k[ok])), e_inv[ok].max()
    assert np.all(e_det[ok] <= tol_f64_comp(k[ok])), e_det[ok].max()
    assert np.all(e_inv[k <= 1e6] <= 1e-12) and np.all(e_det[k <= 1e6] <= 1e-12)


def test_f32_compensated_reroute_and_bound():
    rng = np.random.default_rng(32)
    z32 = hard(rng, 60000, 10.0).astype(np.float32)
    z = z32.astype(np.float64)
    inv, det, st, bound = pixel.adjugate_comp_f32(z32)
    pd = oracle.pd_class(z) == 0
    k = oracle.kappa(z)
    (ih, il), (dh, dl) = oracle.ge128(z)
    e_inv = oracle.inv_rel_err(inv, ih, il)
    e_det = oracle.det_rel_err(det, dh, dl)
    assert np.all(e_inv[pd] <= tol_f32(k[pd])) and np.all(e_det[pd] <= tol_f32(k[pd]))
    # the bound covers the true error wherever the FP32 result was kept
    kept = st == 0
    true_err = np.abs((det.astype(np.float64) - dh) - dl)
    assert kept.sum() > 10000
    assert np.all(true_err[kept] <= bound[kept].astype(np.float64))
    # kept pixels meet the 1e-6 relative determinant target
    assert np.all(e_det[kept] <= 1e-6)
    # reroutes happen for ill-conditioned matrices only
    assert np.all(st[k < 100] == 0)
    assert np.mean(st[(k > 1e6) & pd] == 1) > 0.5
    # every oracle-PD pixel comes out positive definite (kept or fixed by FP64)
    assert np.all(st[pd & (k < 1e7)] <= 1)


def test_f32_bound_covers_tiny_entries():
    """Near rank-2 matrices scaled by 10^s, s uniform in [-12, 12]: below about
    1e-10 the FP32 products underflow and the error-free transformations stop
    being exact; the bound's underflow term must still cover the true error of
    every kept pixel (such pixels are recomputed in FP64 instead)."""
    rng = np.random.default_rng(34)
    m = 40000
    U = synth.haar_unitary(rng, m)
    scale = 10.0 ** rng.uniform(-12, 12, m)
    eig = np.stack([np.ones(m), 10.0 ** -rng.uniform(0, 3, m), 10.0 ** -rng.uniform(5, 12, m)], 1) * scale[:, None]
    z32 = synth.pack(np.einsum("mij,mj,mkj->mik", U, eig, np.conj(U))).astype(np.float32)
    inv, det, st, bound = pixel.adjugate_comp_f32(z32)
    (ih, il), (dh, dl) = oracle.ge128(z32.astype(np.float64))
    kept = st == 0
    err = np.abs((det.astype(np.float64) - dh) - dl)
    assert kept.sum() > 5000
    assert np.all(err[kept] <= bound[kept].astype(np.float64))
    assert np.all(err[kept] <= 1e-6 * np.abs(dh[kept]))
    # the tiniest matrices are all recomputed (or not positive definite)
    assert np.all(st[scale < 1e-11] != 0)


def test_indefinite_with_positive_determinant_is_not_pd():
    """Eigenvalues (-l1, -l2, l3): det > 0 but not positive definite; the
    leading-minor test flags every one (the oracle's pivot signs agree)."""
    rng = np.random.default_rng(33)
    m = 5000
    eig = np.stack([-10.0 ** -rng.uniform(0, 3, m), -10.0 ** -rng.uniform(0, 3, m), 10.0 ** -rng.uniform(0, 3, m)], 1)
    U = synth.haar_unitary(rng, m)
    z = synth.pack(np.einsum("mij,mj,mkj->mik", U, eig, np.conj(U)))
    assert np.all(oracle.pd_class(z) == 2)
    _, det64, st64 = pixel.adjugate_comp_f64(z)
    assert np.all(det64 > 0) and np.all(st64 == 2)
    _, det32, st32, _ = pixel.adjugate_comp_f32(z.astype(np.float32))
    assert np.all(st32 == 2)


def test_plain_det_bound_covers_true_error():
    """The a-priori bound of the plain FP32 determinant (the Wishart term's
    low-accuracy flag) covers the true error on hard matrices up to kappa 1e10
    and on scaled ones whose products underflow; it is loose by construction,
    but not absurdly so (median bound / error below 1e3 where the error is
    not zero)."""
    rng = np.random.default_rng(35)
    z = hard(rng, 60000)
    m = 20000
    U = synth.haar_unitary(rng, m)
    scale = 10.0 ** rng.uniform(-12, 12, m)
    eig = np.stack([np.ones(m), 10.0 ** -rng.uniform(0, 3, m), 10.0 ** -rng.uniform(0, 8, m)], 1) * scale[:, None]
    z = np.concatenate([z, synth.pack(np.einsum("mij,mj,mkj->mik", U, eig, np.conj(U)))], axis=1)
    z32 = z.astype(np.float32)
    det, bound = pixel.det_plain_bound_f32(z32)
    _, (dh, dl) = oracle.ge128(z32.astype(np.float64))
    err = np.abs((det.astype(np.float64) - dh) - dl)
    assert np.all(err <= bound.astype(np.float64))
    nz = err > 0
    assert np.median(bound[nz] / err[nz]) < 1e3
    # a planted mistake, the cofactors' own product magnitudes S_i left out
    # of the bound (gamma_8 sum |x_i| |c_i| only), fails on this data: where
    # a cofactor cancels, its rounding error dwarfs |x_i c_i|
    w = z32.astype(np.float64)
    a, d, f, br, bi, cr, ci, er, ei = w
    cof = [d * f - er * er - ei * ei, cr * er + ci * ei - br * f, ci * er - cr * ei - bi * f,
           br * er - bi * ei - cr * d, br * ei + bi * er - ci * d]
    xs = [a, br, bi, cr, ci]
    g8 = 8 * 2.0 ** -24 / (1 - 8 * 2.0 ** -24)
    planted = g8 * sum(np.abs(x) * np.abs(c) for x, c in zip(xs, cof))
    assert np.any(err > planted)


def test_fast_two_sum_exact_when_ordered():
    """FastTwoSum gives TwoSum's (s, e) bit for bit whenever |a| >= |b|, and
    s + e equals a + b exactly (checked in rationals), over pairs spanning
    the exponent range with opposite and equal signs."""
    from fractions import Fraction
    rng = np.random.default_rng(41)
    m = 20000
    a = (rng.standard_normal(m) * 10.0 ** rng.uniform(-20, 20, m)).astype(np.float32)
    b = (rng.standard_normal(m) * np.abs(a) * 10.0 ** -rng.uniform(0, 12, m)).astype(np.float32)
    b[:100] = -a[:100]                       # exact cancellation
    b[100:200] = -np.nextafter(a[100:200], 0)  # near cancellation
    swap = np.abs(b) > np.abs(a)
    a[swap], b[swap] = b[swap], a[swap]
    s0, e0 = pixel.sum_pair_f32(a, b, fast=False)
    s1, e1 = pixel.sum_pair_f32(a, b, fast=True)
    assert np.array_equal(s0.view(np.uint32), s1.view(np.uint32))
    assert np.array_equal(e0.view(np.uint32), e1.view(np.uint32))
    for i in rng.choice(m, 400, replace=False).tolist() + list(range(0, 200, 20)):
        assert Fraction(float(s1[i])) + Fraction(float(e1[i])) == Fraction(float(a[i])) + Fraction(float(b[i]))
    # out of order it is not error-free in general: the planted case must fail
    s2, e2 = pixel.sum_pair_f32(np.float32([1e-8]), np.float32([1.0]), fast=True)
    assert Fraction(float(s2[0])) + Fraction(float(e2[0])) != Fraction(float(np.float32(1e-8))) + 1


def test_ordered_diagonal_cofactors():
    """The diagonal cofactors' ordered form: on positive-definite matrices the
    flag holds (hard ones up to kappa 1e10 included) and hi + lo is within the
    Dot2 bound of the exact cofactor; a matrix whose lower 2x2 minor is
    indefinite (|e|^2 > d f) clears the flag and is sent to the FP64 path,
    which classifies it not positive definite."""
    from fractions import Fraction
    rng = np.random.default_rng(43)
    z32 = hard(rng, 20000, 10.0).astype(np.float32)
    pd = oracle.pd_class(z32.astype(np.float64)) == 0
    hi, lo, ordered = pixel.diag_cofactors_f32(z32)
    ordered_pd = ordered[pd]
    # the first sum is always ordered for PD input; the second may fail only
    # where the minor nearly vanishes, which the reroute absorbs
    assert ordered_pd.mean() > 0.99
    w = z32.astype(np.float64)
    a, d, f, br, bi, cr, ci, er, ei = w
    exact = [d * f - er * er - ei * ei, a * f - cr * cr - ci * ci, a * d - br * br - bi * bi]  # FP32 products exact in FP64
    mags = [d * f + er * er + ei * ei, a * f + cr * cr + ci * ci, a * d + br * br + bi * bi]
    u = 2.0 ** -24
    for k in range(3):
        idx = np.flatnonzero(pd & ordered)[:2000]
        got = hi[k, idx].astype(np.float64) + lo[k, idx].astype(np.float64)
        assert np.all(np.abs(got - exact[k][idx]) <= 4 * u * u * mags[k][idx] + 1e-300)
    # an indefinite lower minor: er^2 > d f
    bad = np.float32([[4.0], [1.0], [1.0], [0.1], [0.0], [0.1], [0.0], [2.0], [0.0]])
    _, _, ordered_bad = pixel.diag_cofactors_f32(bad)
    assert not ordered_bad[0]
    _, _, st, _ = pixel.adjugate_comp_f32(bad)
    assert st[0] == 2
