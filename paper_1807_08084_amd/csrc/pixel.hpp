// Per-pixel arithmetic of the 3x3 Hermitian inverse and determinant.
//
// Packed layout of one matrix (Section 2.1, "Preliminaries and Notation"):
// the upper triangle a, d, f (real diagonal) and b, c, e (complex), held as
//   z[0]=a z[1]=d z[2]=f z[3]=Re b z[4]=Im b z[5]=Re c z[6]=Im c z[7]=Re e z[8]=Im e
// The inverse is returned in the same packing.
//
// Every function here is __host__ __device__ so the same source can be
// compiled for the host and exercised by logic tests; the kernels in
// polsar.hip inline them.
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define PX_HD __host__ __device__ __forceinline__
#else
#define PX_HD inline
#endif

namespace px {

// Per-pixel status, also the values of the optional status plane.
enum : int { ST_OK = 0, ST_REROUTED = 1, ST_NOT_PD = 2, ST_NONFINITE = 3 };

PX_HD float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
PX_HD double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
PX_HD float abs_(float x) { return __builtin_fabsf(x); }
PX_HD double abs_(double x) { return __builtin_fabs(x); }
// Correctly rounded square root; natural logarithm from the math library.
PX_HD float sqrt_(float x) { return sqrtf(x); }
PX_HD double sqrt_(double x) { return sqrt(x); }
PX_HD float log_(float x) { return logf(x); }
PX_HD double log_(double x) { return log(x); }
template <class T> PX_HD bool finite_(T x) { return __builtin_isfinite(x); }

template <class T> struct Eps;
// u: unit roundoff; eta: smallest normal number, a bound on the absolute
// error one operation can add when its result is subnormal (or flushed).
template <> struct Eps<float> {
  static constexpr double u = 5.9604644775390625e-08;   // 2^-24
  static constexpr double eta = 1.1754943508222875e-38;  // 2^-126
};
template <> struct Eps<double> {
  static constexpr double u = 1.1102230246251565e-16;   // 2^-53
  static constexpr double eta = 2.2250738585072014e-308;  // 2^-1022
};

// ---------------------------------------------------------------------------
// Alg. 2 (Section 3.1), evaluated directly.
// Cofactors from Eq. (adjoint_elements), split into real parts:
//   a_c = d f - |e|^2                  d_c = a f - |c|^2        f_c = a d - |b|^2
//   b_c = c conj(e) - b f   ->  Re: cr er + ci ei - br f     Im: ci er - cr ei - bi f
//   c_c = b e - c d         ->  Re: br er - bi ei - cr d     Im: br ei + bi er - ci d
//   e_c = c conj(b) - a e   ->  Re: cr br + ci bi - a er     Im: ci br - cr bi - a ei
// Determinant from the real-part expansion along row 0 (Eq. detr):
//   det = a a_c + Re b Re b_c + Im b Im b_c + Re c Re c_c + Im c Im c_c
// then t = 1/det (the one division) and A^{-1} = t * adj(A) (Eq. inv_adjoint).
// ---------------------------------------------------------------------------
template <class T>
PX_HD void cofactors_plain(const T z[9], T c[9]) {
  const T a = z[0], d = z[1], f = z[2], br = z[3], bi = z[4], cr = z[5], ci = z[6], er = z[7], ei = z[8];
  c[0] = d * f - (er * er + ei * ei);
  c[1] = a * f - (cr * cr + ci * ci);
  c[2] = a * d - (br * br + bi * bi);
  c[3] = cr * er + ci * ei - br * f;
  c[4] = ci * er - cr * ei - bi * f;
  c[5] = br * er - bi * ei - cr * d;
  c[6] = br * ei + bi * er - ci * d;
  c[7] = cr * br + ci * bi - a * er;
  c[8] = ci * br - cr * bi - a * ei;
}

template <class T>
PX_HD T det_from_cofactors(const T z[9], const T c[9]) {
  return z[0] * c[0] + z[3] * c[3] + z[4] * c[4] + z[5] * c[5] + z[6] * c[6];
}

// Classify an evaluated pixel: non-finite beats not-positive-definite.
// Positive definiteness by Sylvester's criterion on the leading principal
// minors a, f_c = a d - |b|^2 (a cofactor already at hand) and det.
template <class T>
PX_HD int classify(T det, T t, T a, T minor2) {
  if (!finite_(det)) return ST_NONFINITE;
  if (!(det > T(0)) || !(a > T(0)) || !(minor2 > T(0))) return ST_NOT_PD;
  if (!finite_(t)) return ST_NONFINITE;
  return ST_OK;
}

template <class T>
PX_HD int adjugate_plain(const T z[9], T x[9], T& det) {
  T c[9];
  cofactors_plain(z, c);
  det = det_from_cofactors(z, c);
  const T t = T(1) / det;
#pragma unroll
  for (int k = 0; k < 9; ++k) x[k] = t * c[k];
  return classify(det, t, z[0], c[2]);
}

// FP32 storage, FP64 arithmetic: the same formulas on exactly widened inputs.
PX_HD int adjugate_wide(const float z[9], float x[9], float& det) {
  double zd[9], xd[9], dd;
#pragma unroll
  for (int k = 0; k < 9; ++k) zd[k] = (double)z[k];
  int st = adjugate_plain(zd, xd, dd);
#pragma unroll
  for (int k = 0; k < 9; ++k) x[k] = (float)xd[k];
  det = (float)dd;
  const float t = 1.0f / det;
  int st32 = classify(det, t, z[0], 1.0f);  // the minors were checked in FP64
  return st32 > st ? st32 : st;
}

// ---------------------------------------------------------------------------
// Compensated evaluation of the same formulas.
// Each cofactor component is a signed dot product of three products, taken
// with the Dot2 scheme of Ogita, Rump and Oishi ("Accurate sum and dot
// product", SIAM J. Sci. Comput. 26(6), 2005, Alg. 5.3): error-free products
// by FMA (TwoProduct) and error-free additions (TwoSum), the rounding errors
// gathered in a second word.  The result is kept as an unevaluated pair
// hi + lo with |hi + lo - exact| <= gamma_3^2 * sum|products|.
// The determinant is the Dot2 sum of the five products a*a_c.hi, ...; the
// five products with the low words are added into its error word.
// FP contraction is disabled here: every fused operation is explicit.
// ---------------------------------------------------------------------------
template <class T> struct DW { T hi, lo; };

template <class T>
PX_HD void two_sum(T a, T b, T& s, T& e) {
#if defined(__clang__)
#pragma clang fp contract(off)
#endif
  s = a + b;
  const T bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Error-free addition when |a| >= |b| (Dekker's FastTwoSum): a + b = s + e
// exactly, in three operations instead of TwoSum's six.
template <class T>
PX_HD void fast_two_sum(T a, T b, T& s, T& e) {
#if defined(__clang__)
#pragma clang fp contract(off)
#endif
  s = a + b;
  e = b - (s - a);
}

// Dot2 of (x1 y1 + x2 y2 + x3 y3).  The products' rounding errors (FMA)
// and the additions' (TwoSum) are exact; only the two rounded additions
// that gather them into the low word, t = q + r and s = s + t, lose
// anything, each at most u times its rounded result (round to nearest).
// rerr returns their running error sum |t1| + |s1| + |t2| + |s2|, so that
// |hi + lo - exact| <= u * rerr.
// ORDERED: the additions are FastTwoSums, exact only while the running sum
// is at least as large in magnitude as the product added to it; `ordered`
// is cleared where that fails (a diagonal cofactor of a positive-definite
// matrix, x1 y1 - |.|^2 - |.|^2, passes its first test always; NaN fails).
// Where it holds the result equals the TwoSum form's bit for bit.
template <class T, bool ORDERED = false>
PX_HD DW<T> dot3(T x1, T y1, T x2, T y2, T x3, T y3, T& rerr, bool* ordered = nullptr) {
#if defined(__clang__)
#pragma clang fp contract(off)
#endif
  T p = x1 * y1;
  T s = fma_(x1, y1, -p);
  T h = x2 * y2;
  T r = fma_(x2, y2, -h);
  T q;
  if constexpr (ORDERED) {
    *ordered = *ordered && abs_(p) >= abs_(h);
    fast_two_sum(p, h, p, q);
  } else {
    two_sum(p, h, p, q);
  }
  T t = q + r;
  s = s + t;
  rerr = abs_(t) + abs_(s);
  h = x3 * y3;
  r = fma_(x3, y3, -h);
  if constexpr (ORDERED) {
    *ordered = *ordered && abs_(p) >= abs_(h);
    fast_two_sum(p, h, p, q);
  } else {
    two_sum(p, h, p, q);
  }
  t = q + r;
  s = s + t;
  rerr = rerr + (abs_(t) + abs_(s));
  return DW<T>{p, s};
}

// ordered (FP32 step only, null otherwise): the diagonal cofactors take the
// FastTwoSum form and clear *ordered where its condition fails.
template <class T>
PX_HD void cofactors_comp(const T z[9], DW<T> c[9], T rerr[9], bool* ordered = nullptr) {
  const T a = z[0], d = z[1], f = z[2], br = z[3], bi = z[4], cr = z[5], ci = z[6], er = z[7], ei = z[8];
  if (ordered) {
    c[0] = dot3<T, true>(d, f, -er, er, -ei, ei, rerr[0], ordered);
    c[1] = dot3<T, true>(a, f, -cr, cr, -ci, ci, rerr[1], ordered);
    c[2] = dot3<T, true>(a, d, -br, br, -bi, bi, rerr[2], ordered);
  } else {
    c[0] = dot3(d, f, -er, er, -ei, ei, rerr[0]);
    c[1] = dot3(a, f, -cr, cr, -ci, ci, rerr[1]);
    c[2] = dot3(a, d, -br, br, -bi, bi, rerr[2]);
  }
  c[3] = dot3(cr, er, ci, ei, -br, f, rerr[3]);
  c[4] = dot3(ci, er, -cr, ei, -bi, f, rerr[4]);
  c[5] = dot3(br, er, -bi, ei, -cr, d, rerr[5]);
  c[6] = dot3(br, ei, bi, er, -ci, d, rerr[6]);
  c[7] = dot3(cr, br, ci, bi, -a, er, rerr[7]);
  c[8] = dot3(ci, br, -cr, bi, -a, ei, rerr[8]);
}

// Compensated determinant from the row-0 expansion, x = (a, Re b, Im b,
// Re c, Im c): the Dot2 sum of the five products x_i hi_i, then the five
// x_i lo_i added into its low word.  Returns the rounded det and the
// a-posteriori bound E >= |det_returned - det(A)| from a running error
// analysis: every rounded addition into the low word (t = q + r, s = s + t,
// and each s = fma(x_i, lo_i, s)) is off by at most u times its rounded
// result, R being the sum of those results' magnitudes; the cofactors are
// off by at most u rerr_i each, C = sum |x_i| rerr_i; the final rounding
// adds u |det|.  Where results are subnormal (or flushed to zero) the
// error-free transformations stop being exact: each of the at most 48
// operations of the determinant and 22 of each cofactor can then add eta,
// the smallest normal number, which the term 64 eta (1 + sum |x_i|) covers:
//   E = (1 + 64u) [u (|det| + R + C) + 64 eta (1 + sum |x_i|)],
// the (1 + 64u) covering the rounding of R, C and E themselves.  With
// entries far below 1e-10 in FP32 that term exceeds 1e-6 |det| and the
// pixel is recomputed in FP64, where nothing underflows.
template <class T>
PX_HD T det_comp(const T z[9], const DW<T> c[9], const T rerr[9], T& bound) {
#if defined(__clang__)
#pragma clang fp contract(off)
#endif
  const T x[5] = {z[0], z[3], z[4], z[5], z[6]};
  const int idx[5] = {0, 3, 4, 5, 6};
  T p = x[0] * c[0].hi;
  T s = fma_(x[0], c[0].hi, -p);
  T R = T(0);
  T C = abs_(x[0]) * rerr[0];
  T X = abs_(x[0]);
#pragma unroll
  for (int i = 1; i < 5; ++i) {
    const T h = x[i] * c[idx[i]].hi;
    const T r = fma_(x[i], c[idx[i]].hi, -h);
    T q;
    C = fma_(abs_(x[i]), rerr[idx[i]], C);
    X = X + abs_(x[i]);
    two_sum(p, h, p, q);
    const T t = q + r;
    s = s + t;
    R = R + (abs_(t) + abs_(s));
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    s = fma_(x[i], c[idx[i]].lo, s);
    R = R + abs_(s);
  }
  const T det = p + s;
  constexpr T u = (T)Eps<T>::u;
  constexpr T eta64 = (T)(64.0 * Eps<T>::eta);
  bound = (T(1) + T(64) * u) * fma_(eta64, T(1) + X, u * ((abs_(det) + R) + C));
  return det;
}

template <class T>
PX_HD void scale_comp(const DW<T> c[9], T t, T x[9]) {
#if defined(__clang__)
#pragma clang fp contract(off)
#endif
#pragma unroll
  for (int k = 0; k < 9; ++k) x[k] = fma_(c[k].hi, t, c[k].lo * t);
}

// Compensated FP64 (no reroute: FP64 is the widest type on the path).
PX_HD int adjugate_comp(const double z[9], double x[9], double& det) {
  DW<double> c[9];
  double rerr[9], bound;
  cofactors_comp(z, c, rerr);
  det = det_comp(z, c, rerr, bound);
  const double t = 1.0 / det;
  scale_comp(c, t, x);
  return classify(det, t, z[0], c[2].hi + c[2].lo);
}

// Relative threshold on the determinant bound above which an FP32 pixel is
// recomputed in FP64.
constexpr float REROUTE_REL = 1e-6f;

// Compensated FP32 with selective FP64 recompute.  A pixel whose bound
// exceeds REROUTE_REL * |det|, or whose det is not positive or not finite,
// is recomputed by the compensated FP64 path from its exactly widened
// inputs and rounded to FP32 (status ST_REROUTED when that succeeds).
//
// adjugate_comp_try: the FP32 step; returns true and the result when the
// pixel is accepted, false when it must be recomputed (x then holds the
// scaled FP32 cofactors, which the recompute replaces: scaling every pixel
// costs less than branching around the scale).
PX_HD bool adjugate_comp_try(const float z[9], float x[9], float& det, float* bound_out = nullptr) {
  DW<float> c[9];
  float rerr[9], bound;
  bool ordered = true;
  cofactors_comp(z, c, rerr, &ordered);
  det = det_comp(z, c, rerr, bound);
  if (bound_out) *bound_out = bound;
  const float t = 1.0f / det;
  const bool ok = ordered && det > 0.0f && finite_(det) && finite_(t) && !(bound > REROUTE_REL * det) &&
                  z[0] > 0.0f && c[2].hi + c[2].lo > 0.0f;
  scale_comp(c, t, x);
  return ok;
}

// Cofactors of an FP32 matrix in FP64.  A product of two FP32 numbers has at
// most 48 significant bits, so FP64 holds every cofactor product exactly
// (the exponent range covers all finite FP32 products); each component is
// then a sum of three exact terms, and two error-free additions leave it as
// hi + lo with |hi + lo - exact| <= u(|e1 + e2|) <= 2u^2 sum|products|,
// within the Dot2 bound of cofactors_comp at a third fewer operations.
PX_HD DW<double> sum3_exact(double p1, double p2, double p3) {
  double s, e1, e2;
  two_sum(p1, p2, s, e1);
  two_sum(s, p3, s, e2);
  return DW<double>{s, e1 + e2};
}

// The cofactors that enter the determinant (a_c, b_c, c_c) and the leading
// minor f_c of the positive-definiteness check are kept as hi + lo; d_c and
// e_c only scale into inverse entries, whose FP32 rounding covers the error
// of a plain sum of the three exact products (at most 2u sum|products|,
// below 7e-8 of the inverse's norm for condition numbers up to 1e8), so
// they are summed plainly (lo = 0) at a third of the operations.
PX_HD DW<double> sum3_plain(double p1, double p2, double p3) { return DW<double>{(p1 + p2) + p3, 0.0}; }

PX_HD void cofactors_widened(const double z[9], DW<double> c[9]) {
  const double a = z[0], d = z[1], f = z[2], br = z[3], bi = z[4], cr = z[5], ci = z[6], er = z[7], ei = z[8];
  c[0] = sum3_exact(d * f, -(er * er), -(ei * ei));
  c[1] = sum3_plain(a * f, -(cr * cr), -(ci * ci));
  c[2] = sum3_exact(a * d, -(br * br), -(bi * bi));
  c[3] = sum3_exact(cr * er, ci * ei, -(br * f));
  c[4] = sum3_exact(ci * er, -(cr * ei), -(bi * f));
  c[5] = sum3_exact(br * er, -(bi * ei), -(cr * d));
  c[6] = sum3_exact(br * ei, bi * er, -(ci * d));
  c[7] = sum3_plain(cr * br, ci * bi, -(a * er));
  c[8] = sum3_plain(ci * br, -(cr * bi), -(a * ei));
}

// adjugate_comp_reroute: the FP64 recompute of one pixel, rounded to FP32:
// exact-product cofactors as above, then the compensated determinant, the
// one division and the scaling of the FP64 compensated form (plain for the
// plainly summed cofactors).
PX_HD int adjugate_comp_reroute(const float z[9], float x[9], float& det) {
  double zd[9], xd[9], dd;
#pragma unroll
  for (int k = 0; k < 9; ++k) zd[k] = (double)z[k];
  int st;
  {
    DW<double> c[9];
    const double no_rerr[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // the bound is not used here
    double bound;
    cofactors_widened(zd, c);
    dd = det_comp(zd, c, no_rerr, bound);
    const double t = 1.0 / dd;
    scale_comp(c, t, xd);
    xd[1] = c[1].hi * t;  // the plainly summed cofactors: no low word
    xd[7] = c[7].hi * t;
    xd[8] = c[8].hi * t;
    st = classify(dd, t, zd[0], c[2].hi + c[2].lo);
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) x[k] = (float)xd[k];
  det = (float)dd;
  if (st == ST_OK) {
    st = classify(det, 1.0f / det, z[0], 1.0f);  // the minors were checked in FP64
    if (st == ST_OK) st = ST_REROUTED;
  }
  return st;
}

PX_HD int adjugate_comp(const float z[9], float x[9], float& det, float* bound_out = nullptr) {
  if (adjugate_comp_try(z, x, det, bound_out)) return ST_OK;
  return adjugate_comp_reroute(z, x, det);
}

// ---------------------------------------------------------------------------
// Multilook front end (Introduction, Eq. (ZN), read as the outer product):
// Z = (1/N) sum_l S(l) S(l)^H for single-look vectors S = (S_HH, S_HV, S_VV).
// One look's contribution to the nine packed components, accumulated in
// FP64 (for FP32 looks every product is exact in FP64):
//   a += |S_HH|^2, d += |S_HV|^2, f += |S_VV|^2,
//   b += S_HH conj(S_HV), c += S_HH conj(S_VV), e += S_HV conj(S_VV).
// s = (Re S_HH, Im S_HH, Re S_HV, Im S_HV, Re S_VV, Im S_VV).
// look_accumulate forms each component's two-product sum first and adds it
// (three operations, a short dependency chain from look to look);
// look_accumulate_chained adds each real product with one FMA (two
// operations, twice the chain).  The first suits the per-pixel multilook
// (few looks per lane, latency-bound), the second the boxcar (many looks
// per row sum, bound by VALU issue).  Both round once per addition.
// ---------------------------------------------------------------------------
template <class T>
PX_HD void look_accumulate(const T s[6], double acc[9]) {
  const double hr = s[0], hi = s[1], vr = s[2], vi = s[3], wr = s[4], wi = s[5];
  acc[0] += hr * hr + hi * hi;
  acc[1] += vr * vr + vi * vi;
  acc[2] += wr * wr + wi * wi;
  acc[3] += hr * vr + hi * vi;
  acc[4] += hi * vr - hr * vi;
  acc[5] += hr * wr + hi * wi;
  acc[6] += hi * wr - hr * wi;
  acc[7] += vr * wr + vi * wi;
  acc[8] += vi * wr - vr * wi;
}

// The first look of a sum: its contribution itself (equal to adding it to
// zero with look_accumulate_chained).
template <class T>
PX_HD void look_first(const T s[6], double acc[9]) {
  const double hr = s[0], hi = s[1], vr = s[2], vi = s[3], wr = s[4], wi = s[5];
  acc[0] = fma_(hi, hi, hr * hr);
  acc[1] = fma_(vi, vi, vr * vr);
  acc[2] = fma_(wi, wi, wr * wr);
  acc[3] = fma_(hi, vi, hr * vr);
  acc[4] = fma_(-hr, vi, hi * vr);
  acc[5] = fma_(hi, wi, hr * wr);
  acc[6] = fma_(-hr, wi, hi * wr);
  acc[7] = fma_(vi, wi, vr * wr);
  acc[8] = fma_(-vr, wi, vi * wr);
}

template <class T>
PX_HD void look_accumulate_chained(const T s[6], double acc[9]) {
  const double hr = s[0], hi = s[1], vr = s[2], vi = s[3], wr = s[4], wi = s[5];
  acc[0] = fma_(hi, hi, fma_(hr, hr, acc[0]));
  acc[1] = fma_(vi, vi, fma_(vr, vr, acc[1]));
  acc[2] = fma_(wi, wi, fma_(wr, wr, acc[2]));
  acc[3] = fma_(hi, vi, fma_(hr, vr, acc[3]));
  acc[4] = fma_(-hr, vi, fma_(hi, vr, acc[4]));
  acc[5] = fma_(hi, wi, fma_(hr, wr, acc[5]));
  acc[6] = fma_(-hr, wi, fma_(hi, wr, acc[6]));
  acc[7] = fma_(vi, wi, fma_(vr, wr, acc[7]));
  acc[8] = fma_(-vr, wi, fma_(vi, wr, acc[8]));
}

// ---------------------------------------------------------------------------
// Cholesky comparison form (Section 2.2 and Alg. 1): A = L L^H,
//   l00 = sqrt(a), v0 = 1/l00, l10 = conj(b) v0, l20 = conj(c) v0,
//   l11 = sqrt(d - |l10|^2), v1 = 1/l11,
//   l21 = (conj(e) - l20 conj(l10)) v1   (the conjugate of the printed
//                                          assignment, which solves A[1][2]
//                                          instead of A[2][1]),
//   l22 = sqrt(f - |l20|^2 - |l21|^2), v2 = 1/l22;
// T = L^{-1}: t10 = -l10 v0 v1, t20 = v2 v0 (l21 l10 v1 - l20), t21 = -l21 v1 v2;
// det = (l00 l11 l22)^2 and A^{-1} = T^H T (upper triangle).
// Status: non-finite input first, then not positive definite when a squared
// pivot is <= 0, then non-finite results.
// ---------------------------------------------------------------------------
template <class T>
PX_HD int cholesky_plain(const T z[9], T x[9], T& det) {
  const T a = z[0], d = z[1], f = z[2], br = z[3], bi = z[4], cr = z[5], ci = z[6], er = z[7], ei = z[8];
  const T p0 = a;
  const T l00 = sqrt_(p0), v0 = T(1) / l00;
  const T l10r = br * v0, l10i = -bi * v0;  // conj(b) v0
  const T l20r = cr * v0, l20i = -ci * v0;  // conj(c) v0
  const T p1 = d - (l10r * l10r + l10i * l10i);
  const T l11 = sqrt_(p1), v1 = T(1) / l11;
  // l20 conj(l10)
  const T mr = l20r * l10r + l20i * l10i;
  const T mi = l20i * l10r - l20r * l10i;
  const T l21r = (er - mr) * v1, l21i = (-ei - mi) * v1;
  const T p2 = f - (l20r * l20r + l20i * l20i) - (l21r * l21r + l21i * l21i);
  const T l22 = sqrt_(p2), v2 = T(1) / l22;
  const T t10s = -v0 * v1;
  const T t10r = l10r * t10s, t10i = l10i * t10s;
  // l21 l10 v1 - l20
  const T wr = (l21r * l10r - l21i * l10i) * v1 - l20r;
  const T wi = (l21r * l10i + l21i * l10r) * v1 - l20i;
  const T t20s = v2 * v0;
  const T t20r = wr * t20s, t20i = wi * t20s;
  const T t21s = -v1 * v2;
  const T t21r = l21r * t21s, t21i = l21i * t21s;
  const T g = l00 * l11 * l22;
  det = g * g;
  x[0] = v0 * v0 + (t10r * t10r + t10i * t10i) + (t20r * t20r + t20i * t20i);
  x[1] = v1 * v1 + (t21r * t21r + t21i * t21i);
  x[2] = v2 * v2;
  // b_i = conj(t10) t11 + conj(t20) t21
  x[3] = t10r * v1 + (t20r * t21r + t20i * t21i);
  x[4] = -t10i * v1 + (t20r * t21i - t20i * t21r);
  // c_i = conj(t20) t22, e_i = conj(t21) t22
  x[5] = t20r * v2;
  x[6] = -t20i * v2;
  x[7] = t21r * v2;
  x[8] = -t21i * v2;
  bool finite_in = true;
#pragma unroll
  for (int k = 0; k < 9; ++k) finite_in = finite_in && finite_(z[k]);
  if (!finite_in) return ST_NONFINITE;
  if (p0 <= T(0) || p1 <= T(0) || p2 <= T(0)) return ST_NOT_PD;
  if (!(finite_(det) && finite_(v0) && finite_(v1) && finite_(v2) && finite_(p0 + p1 + p2)))
    return ST_NONFINITE;
  return ST_OK;
}

PX_HD int cholesky_wide(const float z[9], float x[9], float& det) {
  double zd[9], xd[9], dd;
#pragma unroll
  for (int k = 0; k < 9; ++k) zd[k] = (double)z[k];
  int st = cholesky_plain(zd, xd, dd);
#pragma unroll
  for (int k = 0; k < 9; ++k) x[k] = (float)xd[k];
  det = (float)dd;
  if (st == ST_OK && !(finite_(det) && det > 0.0f && finite_(1.0f / det))) st = ST_NONFINITE;
  return st;
}

// FP32 Cholesky with an FP64 recompute of pixels whose FP32 pivots fail.
PX_HD int cholesky_fallback(const float z[9], float x[9], float& det) {
  int st = cholesky_plain(z, x, det);
  if (st == ST_OK) return ST_OK;
  st = cholesky_wide(z, x, det);
  return st == ST_OK ? ST_REROUTED : st;
}

// ---------------------------------------------------------------------------
// Wishart term for one pixel: l = N (ln det S + tr(S^{-1} Z)), with S^{-1}
// from Alg. 2 (adjugate over det) and
//   tr(adj(S) Z) = a_c z_a + d_c z_d + f_c z_f
//                  + 2 (Re b_c Re z_b + Im b_c Im z_b + ... for c and e),
// since the off-diagonal pairs of a product of Hermitian matrices add to
// twice a real part.
// Gradient with respect to the packed real parameters of S:
//   M = N (P - P Z P), P = S^{-1} recomputed from the adjugate,
//   grad = g (M00, M11, M22, 2Re M01, 2Im M01, 2Re M02, 2Im M02, 2Re M12, 2Im M12)
// (dl = tr(M dS) for Hermitian M and dS; g is the upstream gradient).
// ---------------------------------------------------------------------------
template <class T> struct Cx { T r, i; };
template <class T> PX_HD Cx<T> cmul(Cx<T> a, Cx<T> b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
template <class T> PX_HD Cx<T> cadd(Cx<T> a, Cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <class T> PX_HD Cx<T> cconj(Cx<T> a) { return {a.r, -a.i}; }
template <class T> PX_HD Cx<T> rmul(T s, Cx<T> a) { return {s * a.r, s * a.i}; }

// Entry (i, j) of a packed Hermitian matrix (diagonal real, upper stored).
template <class T>
PX_HD Cx<T> herm(const T* v, int i, int j) {
  if (i == j) return {v[i], T(0)};
  const int k = (i + j == 1) ? 3 : (i + j == 2) ? 5 : 7;  // (0,1) -> b, (0,2) -> c, (1,2) -> e
  return i < j ? Cx<T>{v[k], v[k + 1]} : Cx<T>{v[k], -v[k + 1]};
}

// Products of entries of packed Hermitian matrices with the indices fixed at
// compile time, so that the real diagonal entries cost real arithmetic only
// (a product with a literal zero imaginary part would otherwise be kept:
// IEEE arithmetic may not drop it).
template <int I, int J, class T>
PX_HD Cx<T> he(const T* v) {
  if constexpr (I == J) {
    return {v[I], T(0)};
  } else {
    constexpr int k = (I + J == 1) ? 3 : (I + J == 2) ? 5 : 7;
    if constexpr (I < J) return {v[k], v[k + 1]};
    else return {v[k], -v[k + 1]};
  }
}

// acc (+)= A_IK B_KJ; FIRST: acc is set, not added to.
template <int I, int K, int J, bool FIRST, class T>
PX_HD void mac(Cx<T>& acc, const T* A, const T* B) {
  const Cx<T> a = he<I, K>(A), b = he<K, J>(B);
  if constexpr (I == K && K == J) {
    acc.r = FIRST ? a.r * b.r : fma_(a.r, b.r, acc.r);
    if (FIRST) acc.i = T(0);
  } else if constexpr (I == K) {
    acc.r = FIRST ? a.r * b.r : fma_(a.r, b.r, acc.r);
    acc.i = FIRST ? a.r * b.i : fma_(a.r, b.i, acc.i);
  } else if constexpr (K == J) {
    acc.r = FIRST ? a.r * b.r : fma_(a.r, b.r, acc.r);
    acc.i = FIRST ? a.i * b.r : fma_(a.i, b.r, acc.i);
  } else {
    acc.r = fma_(-a.i, b.i, FIRST ? a.r * b.r : fma_(a.r, b.r, acc.r));
    acc.i = fma_(a.i, b.r, FIRST ? a.r * b.i : fma_(a.r, b.i, acc.i));
  }
}

// Row I of the full product A B of packed Hermitian A, B.
template <int I, class T>
PX_HD void mat_row(const T* A, const T* B, Cx<T> (&row)[3]) {
  mac<I, 0, 0, true>(row[0], A, B);
  mac<I, 1, 0, false>(row[0], A, B);
  mac<I, 2, 0, false>(row[0], A, B);
  mac<I, 0, 1, true>(row[1], A, B);
  mac<I, 1, 1, false>(row[1], A, B);
  mac<I, 2, 1, false>(row[1], A, B);
  mac<I, 0, 2, true>(row[2], A, B);
  mac<I, 1, 2, false>(row[2], A, B);
  mac<I, 2, 2, false>(row[2], A, B);
}

// acc (+)= P_IK W_KJ for packed Hermitian P and a full complex W.
template <int I, int K, int J, bool FIRST, class T>
PX_HD void pw(Cx<T>& acc, const T* P, const Cx<T> (&W)[3][3]) {
  const Cx<T> a = he<I, K>(P), b = W[K][J];
  if constexpr (I == K) {
    acc.r = FIRST ? a.r * b.r : fma_(a.r, b.r, acc.r);
    acc.i = FIRST ? a.r * b.i : fma_(a.r, b.i, acc.i);
  } else {
    acc.r = fma_(-a.i, b.i, FIRST ? a.r * b.r : fma_(a.r, b.r, acc.r));
    acc.i = fma_(a.i, b.r, FIRST ? a.r * b.i : fma_(a.r, b.i, acc.i));
  }
}

// Entry (I, J), I != J, of P W.
template <int I, int J, class T>
PX_HD Cx<T> herm_w(const T* P, const Cx<T> (&W)[3][3]) {
  Cx<T> q;
  pw<I, 0, J, true>(q, P, W);
  pw<I, 1, J, false>(q, P, W);
  pw<I, 2, J, false>(q, P, W);
  return q;
}

// Real part of the diagonal entry (I, I) of P W (the entry of P Z P there is
// real; its imaginary part is not formed).
template <int I, class T>
PX_HD T herm_w_diag(const T* P, const Cx<T> (&W)[3][3]) {
  T q = P[I] * W[I][I].r;
  if constexpr (I != 0) { const Cx<T> a = he<I, 0>(P); q = fma_(-a.i, W[0][I].i, fma_(a.r, W[0][I].r, q)); }
  if constexpr (I != 1) { const Cx<T> a = he<I, 1>(P); q = fma_(-a.i, W[1][I].i, fma_(a.r, W[1][I].r, q)); }
  if constexpr (I != 2) { const Cx<T> a = he<I, 2>(P); q = fma_(-a.i, W[2][I].i, fma_(a.r, W[2][I].r, q)); }
  return q;
}

// A-priori bound on the rounding error of the plain determinant of
// Eq. (detr) with the cofactors of Eq. (adjoint_elements): each cofactor
// component is a sum of three products, evaluated with at most three
// roundings (fused or not), so |c^_i - c_i| <= gamma_3 S_i with S_i the sum
// of its products' magnitudes; the five-term sum of x_i c^_i adds at most
// gamma_5 sum |x_i c^_i|.  Together, with gamma_n = n u / (1 - n u):
//   |det^ - det| <= gamma_8 sum_i |x_i| (|c^_i| + S_i),
// x = (a, Re b, Im b, Re c, Im c) and i over a_c, Re b_c, Im b_c, Re c_c,
// Im c_c; plus 64 eta (1 + sum |x_i|) for operations whose results are
// subnormal (eta the smallest normal number), as in det_comp.  Evaluated in
// the storage type, rounding up by (1 + 16u).
template <class T>
PX_HD T det_plain_bound(const T z[9], const T c[9]) {
  const T a = z[0], d = z[1], f = z[2], br = z[3], bi = z[4], cr = z[5], ci = z[6], er = z[7], ei = z[8];
  const T s0 = abs_(d * f) + (er * er + ei * ei);
  const T s3 = abs_(cr * er) + abs_(ci * ei) + abs_(br * f);
  const T s4 = abs_(ci * er) + abs_(cr * ei) + abs_(bi * f);
  const T s5 = abs_(br * er) + abs_(bi * ei) + abs_(cr * d);
  const T s6 = abs_(br * ei) + abs_(bi * er) + abs_(ci * d);
  const T sum = abs_(a) * (abs_(c[0]) + s0) + abs_(br) * (abs_(c[3]) + s3) + abs_(bi) * (abs_(c[4]) + s4) +
                abs_(cr) * (abs_(c[5]) + s5) + abs_(ci) * (abs_(c[6]) + s6);
  constexpr double u = Eps<T>::u;
  constexpr T g8 = (T)(8.0 * u / (1.0 - 8.0 * u) * (1.0 + 16.0 * u));
  constexpr T eta64 = (T)(64.0 * Eps<T>::eta);
  return fma_(g8, sum, eta64 * (T(1) + abs_(a) + abs_(br) + abs_(bi) + abs_(cr) + abs_(ci)));
}

// Relative determinant error bound of S above which a Wishart term is
// counted as of low accuracy.
constexpr double WISHART_LOW_REL = 1e-3;

// The Wishart term of one pixel and/or its packed gradient.  low (optional)
// is set when S is positive definite but its determinant may be off by more
// than WISHART_LOW_REL relative (det_plain_bound): the term and the gradient
// of such a pixel carry errors of that order or more.
template <class T>
PX_HD int wishart_pixel(const T s[9], const T z[9], T n_looks, bool want_ell, T& ell, bool want_grad, T grad[9],
                        T gscale, bool* low = nullptr) {
  T c[9];
  cofactors_plain(s, c);
  const T det = det_from_cofactors(s, c);
  const T t = T(1) / det;
  const int st = classify(det, t, s[0], c[2]);
  if (low) *low = st == ST_OK && det_plain_bound(s, c) > (T)WISHART_LOW_REL * det;
  if (want_ell) {
    const T tr = c[0] * z[0] + c[1] * z[1] + c[2] * z[2] +
                 T(2) * (c[3] * z[3] + c[4] * z[4] + c[5] * z[5] + c[6] * z[6] + c[7] * z[7] + c[8] * z[8]);
    ell = n_looks * (log_(det) + tr * t);
  }
  if (want_grad) {
    T P[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) P[k] = t * c[k];
    // W = Z P, all nine entries
    Cx<T> W[3][3];
    mat_row<0>(z, P, W[0]);
    mat_row<1>(z, P, W[1]);
    mat_row<2>(z, P, W[2]);
    // Q = P W on the upper triangle; grad = g N (P - Q), off-diagonals doubled
    const T gs = gscale * n_looks, gs2 = T(2) * gs;
    grad[0] = gs * (P[0] - herm_w_diag<0>(P, W));
    grad[1] = gs * (P[1] - herm_w_diag<1>(P, W));
    grad[2] = gs * (P[2] - herm_w_diag<2>(P, W));
    const Cx<T> q01 = herm_w<0, 1>(P, W), q02 = herm_w<0, 2>(P, W), q12 = herm_w<1, 2>(P, W);
    grad[3] = gs2 * (P[3] - q01.r);
    grad[4] = gs2 * (P[4] - q01.i);
    grad[5] = gs2 * (P[5] - q02.r);
    grad[6] = gs2 * (P[6] - q02.i);
    grad[7] = gs2 * (P[7] - q12.r);
    grad[8] = gs2 * (P[8] - q12.i);
  }
  return st;
}

}  // namespace px
