// CPU oracle for the 3x3 Hermitian inverse, determinant and Wishart
// log-likelihood.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and
// the benchmark's CPU-baseline leg load it; the GPU library never does, and
// the two share no code.
//
// Every routine is plain per-pixel scalar code, templated on the real type R
// (double for the FP64 oracle, __float128 for the reference of FP64 checks).
// Build: g++ -O2 -std=c++17 -fPIC -shared -fopenmp -ffp-contract=off
//        oracle.cpp -lquadmath
//
// Input planes (upper triangle of A, Section 2.1 "Preliminaries and
// Notation"): 0:a 1:d 2:f 3:Re b 4:Im b 5:Re c 6:Im c 7:Re e 8:Im e, plane k
// at base + k*pitch.  Inputs are double; FP32 data are widened exactly.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <quadmath.h>

namespace {

inline double sqrt_(double x) { return std::sqrt(x); }
inline __float128 sqrt_(__float128 x) { return sqrtq(x); }
inline double log_(double x) { return std::log(x); }
inline __float128 log_(__float128 x) { return logq(x); }
inline double fabs_(double x) { return std::fabs(x); }
inline __float128 fabs_(__float128 x) { return fabsq(x); }

template <class R>
struct Cx {
  R re, im;
};
template <class R> inline Cx<R> cx(R re, R im) { return Cx<R>{re, im}; }
template <class R> inline Cx<R> operator+(Cx<R> x, Cx<R> y) { return {x.re + y.re, x.im + y.im}; }
template <class R> inline Cx<R> operator-(Cx<R> x, Cx<R> y) { return {x.re - y.re, x.im - y.im}; }
template <class R> inline Cx<R> operator*(Cx<R> x, Cx<R> y) {
  return {x.re * y.re - x.im * y.im, x.re * y.im + x.im * y.re};
}
template <class R> inline Cx<R> scale(Cx<R> x, R s) { return {x.re * s, x.im * s}; }
template <class R> inline Cx<R> conj(Cx<R> x) { return {x.re, -x.im}; }
template <class R> inline R abs2(Cx<R> x) { return x.re * x.re + x.im * x.im; }
template <class R> inline Cx<R> div(Cx<R> x, Cx<R> y) {
  R den = abs2(y);
  Cx<R> p = x * conj(y);
  return {p.re / den, p.im / den};
}

// Full Hermitian matrix from the packed upper triangle (Section 2.1).
template <class R>
void unpack(const double* z, int64_t pitch, int64_t i, Cx<R> A[3][3]) {
  R a = (R)z[0 * pitch + i], d = (R)z[1 * pitch + i], f = (R)z[2 * pitch + i];
  Cx<R> b = cx<R>((R)z[3 * pitch + i], (R)z[4 * pitch + i]);
  Cx<R> c = cx<R>((R)z[5 * pitch + i], (R)z[6 * pitch + i]);
  Cx<R> e = cx<R>((R)z[7 * pitch + i], (R)z[8 * pitch + i]);
  A[0][0] = cx<R>(a, 0); A[0][1] = b;       A[0][2] = c;
  A[1][0] = conj(b);     A[1][1] = cx<R>(d, 0); A[1][2] = e;
  A[2][0] = conj(c);     A[2][1] = conj(e); A[2][2] = cx<R>(f, 0);
}

// Upper triangle of a full matrix into the 9 packed components.
template <class R>
void pack(Cx<R> X[3][3], R out[9]) {
  out[0] = X[0][0].re; out[1] = X[1][1].re; out[2] = X[2][2].re;
  out[3] = X[0][1].re; out[4] = X[0][1].im;
  out[5] = X[0][2].re; out[6] = X[0][2].im;
  out[7] = X[1][2].re; out[8] = X[1][2].im;
}

// Brute-force inverse and determinant: complex Gaussian elimination of
// [A | I] with partial pivoting (largest modulus; ties to the lowest row),
// then back substitution for each column of the identity.
// det = (-1)^swaps * product of pivots.  This is the plain definition
// A X = I, independent of the paper's adjugate identities (Eqs. inv_adjoint,
// det) and of its Cholesky relations.  Returns false on a zero pivot.
template <class R>
bool gauss_elim(const Cx<R> A[3][3], Cx<R> X[3][3], Cx<R>& det) {
  Cx<R> M[3][6];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 6; ++c)
      M[r][c] = c < 3 ? A[r][c] : cx<R>(r == c - 3 ? (R)1 : (R)0, (R)0);
  det = cx<R>((R)1, (R)0);
  bool ok = true;
  for (int k = 0; k < 3; ++k) {
    int p = k;
    R best = abs2(M[k][k]);
    for (int r = k + 1; r < 3; ++r)
      if (abs2(M[r][k]) > best) { best = abs2(M[r][k]); p = r; }
    if (p != k) {
      for (int c = 0; c < 6; ++c) { Cx<R> t = M[k][c]; M[k][c] = M[p][c]; M[p][c] = t; }
      det = cx<R>(-det.re, -det.im);
    }
    Cx<R> piv = M[k][k];
    det = det * piv;
    if (piv.re == 0 && piv.im == 0) { ok = false; continue; }
    for (int r = k + 1; r < 3; ++r) {
      Cx<R> fct = div(M[r][k], piv);
      for (int c = k; c < 6; ++c) M[r][c] = M[r][c] - fct * M[k][c];
    }
  }
  for (int j = 0; j < 3; ++j)
    for (int r = 2; r >= 0; --r) {
      Cx<R> s = M[r][3 + j];
      for (int c = r + 1; c < 3; ++c) s = s - M[r][c] * X[c][j];
      X[r][j] = div(s, M[r][r]);
    }
  return ok;
}

// Cholesky form (Section 2.2 relations and Alg. 1), with l21 taken as the
// solution of the conjugated relation: A[2][1] = conj(e) = l20 conj(l10) +
// l21 l11, i.e. l21 = (conj(e) - l20 conj(l10)) / l11.  (The relation as
// printed, and the assignment that follows it, yield conj(l21): the
// determinant survives but the inverse does not.)  L^{-1} entries follow
// Alg. 1's second step; det = (l00 l11 l22)^2; A^{-1} = (L^{-1})^H L^{-1}.
template <class R>
void cholesky_inv_det(const Cx<R> A[3][3], R out[9], R& det, R piv2[3]) {
  R a = A[0][0].re, d = A[1][1].re, f = A[2][2].re;
  Cx<R> b = A[0][1], c = A[0][2], e = A[1][2];
  piv2[0] = a;
  R l00 = sqrt_(a), v0 = (R)1 / l00;
  Cx<R> l10 = scale(conj(b), v0), l20 = scale(conj(c), v0);
  piv2[1] = d - abs2(l10);
  R l11 = sqrt_(piv2[1]), v1 = (R)1 / l11;
  Cx<R> l21 = scale(conj(e) - l20 * conj(l10), v1);
  piv2[2] = f - abs2(l20) - abs2(l21);
  R l22 = sqrt_(piv2[2]), v2 = (R)1 / l22;
  // T = L^{-1}
  R t00 = v0, t11 = v1, t22 = v2;
  Cx<R> t10 = scale(l10, -v0 * v1);
  Cx<R> t20 = scale(scale(l21 * l10, v1) - l20, v2 * v0);
  Cx<R> t21 = scale(l21, -v1 * v2);
  R g = l00 * l11 * l22;
  det = g * g;
  // A^{-1} = T^H T, upper triangle
  out[0] = t00 * t00 + abs2(t10) + abs2(t20);
  out[1] = t11 * t11 + abs2(t21);
  out[2] = t22 * t22;
  Cx<R> bi = scale(conj(t10), t11) + conj(t20) * t21;
  Cx<R> ci = scale(conj(t20), t22);
  Cx<R> ei = scale(conj(t21), t22);
  out[3] = bi.re; out[4] = bi.im;
  out[5] = ci.re; out[6] = ci.im;
  out[7] = ei.re; out[8] = ei.im;
}

// Checks of the brute-force result that the definition fixes: the
// determinant of a Hermitian matrix is real, and so is the inverse
// Hermitian.  Reported as |Im det|/|Re det| and ||X - X^H||_F / ||X||_F.
template <class R>
void ge_checks(Cx<R> X[3][3], Cx<R> det, double chk[2]) {
  chk[0] = (double)(fabs_(det.im) / fabs_(det.re));
  R num = 0, den = 0;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      num += abs2(X[r][c] - conj(X[c][r]));
      den += abs2(X[r][c]);
    }
  chk[1] = (double)sqrt_(num / den);
}

inline void split(__float128 x, double& hi, double& lo) {
  hi = (double)x;
  lo = (double)(x - (__float128)hi);
}

// Wishart per-pixel term l = N (ln det S + tr(S^{-1} Z)) and its gradient
// M = N (S^{-1} - S^{-1} Z S^{-1}) with respect to the packed real
// parameters of S: (M00, M11, M22, 2Re M01, 2Im M01, 2Re M02, 2Im M02,
// 2Re M12, 2Im M12), from dl = tr(M dS) for Hermitian M and dS.
// S^{-1} and det S come from the brute-force elimination.
template <class R>
bool wishart(const Cx<R> S[3][3], const Cx<R> Z[3][3], R n_looks, R& ell, R g[9]) {
  Cx<R> P[3][3], det;
  if (!gauss_elim(S, P, det)) return false;
  R tr = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) tr += (P[i][j] * Z[j][i]).re;
  ell = n_looks * (log_(det.re) + tr);
  Cx<R> PZ[3][3], PZP[3][3], M[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Cx<R> s = cx<R>(0, 0);
      for (int k = 0; k < 3; ++k) s = s + P[i][k] * Z[k][j];
      PZ[i][j] = s;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Cx<R> s = cx<R>(0, 0);
      for (int k = 0; k < 3; ++k) s = s + PZ[i][k] * P[k][j];
      PZP[i][j] = s;
      M[i][j] = scale(P[i][j] - s, n_looks);
    }
  g[0] = M[0][0].re; g[1] = M[1][1].re; g[2] = M[2][2].re;
  g[3] = 2 * M[0][1].re; g[4] = 2 * M[0][1].im;
  g[5] = 2 * M[0][2].re; g[6] = 2 * M[0][2].im;
  g[7] = 2 * M[1][2].re; g[8] = 2 * M[1][2].im;
  return true;
}

// Multilook covariance (Introduction, Eq. (ZN), read as the outer product
// S S^H): Z = (1/N) sum_l S(l) S(l)^H from N single-look scattering vectors
// S = (S_HH, S_HV, S_VV).  Look planes: 6l + 2i + 0/1 = Re/Im of S_i of look
// l.  Also returns, per packed component, (1/N) sum_l |S_i(l)| |S_j(l)|,
// which bounds the sum of the magnitudes of the terms.
template <class R>
void multilook(const double* looks, int64_t lp, int64_t i, int nl, R z[9], double mag[9]) {
  Cx<R> acc[3][3];
  R m[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) { acc[r][c] = cx<R>(0, 0); m[r][c] = 0; }
  for (int l = 0; l < nl; ++l) {
    Cx<R> S[3];
    R a[3];
    for (int k = 0; k < 3; ++k) {
      S[k] = cx<R>((R)looks[(6 * l + 2 * k) * lp + i], (R)looks[(6 * l + 2 * k + 1) * lp + i]);
      a[k] = sqrt_(abs2(S[k]));
    }
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        acc[r][c] = acc[r][c] + S[r] * conj(S[c]);
        m[r][c] += a[r] * a[c];
      }
  }
  const R inv_n = (R)1 / (R)nl;
  Cx<R> Z[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Z[r][c] = scale(acc[r][c], inv_n);
  pack(Z, z);
  const int ii[9] = {0, 1, 2, 0, 0, 0, 0, 1, 1}, jj[9] = {0, 1, 2, 1, 1, 2, 2, 2, 2};
  for (int k = 0; k < 9; ++k) mag[k] = (double)(m[ii[k]][jj[k]] * inv_n);
}

inline bool finite_input(const double* z, int64_t pitch, int64_t i) {
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(z[k * pitch + i])) return false;
  return true;
}

}  // namespace

extern "C" {

// FP64 brute force.  inv: 9 planes (pitch ip), det: n values, chk: 2 planes
// of n (nullable).  Returns the number of pixels with a zero pivot.
int64_t oracle_ge_f64(int64_t n, const double* z, int64_t zp, double* inv, int64_t ip,
                      double* det, double* chk, int threads) {
  int64_t bad = 0;
#pragma omp parallel for num_threads(threads) schedule(static) reduction(+ : bad)
  for (int64_t i = 0; i < n; ++i) {
    Cx<double> A[3][3], X[3][3], dt;
    unpack(z, zp, i, A);
    if (!gauss_elim(A, X, dt)) ++bad;
    double o[9];
    pack(X, o);
    for (int k = 0; k < 9; ++k) inv[k * ip + i] = o[k];
    det[i] = dt.re;
    if (chk) {
      double c[2];
      ge_checks(X, dt, c);
      chk[i] = c[0];
      chk[n + i] = c[1];
    }
  }
  return bad;
}

// __float128 brute force; results split into double hi + lo parts.
int64_t oracle_ge_f128(int64_t n, const double* z, int64_t zp, double* inv_hi, double* inv_lo,
                       int64_t ip, double* det_hi, double* det_lo, double* chk, int threads) {
  int64_t bad = 0;
#pragma omp parallel for num_threads(threads) schedule(static) reduction(+ : bad)
  for (int64_t i = 0; i < n; ++i) {
    Cx<__float128> A[3][3], X[3][3], dt;
    unpack(z, zp, i, A);
    if (!gauss_elim(A, X, dt)) ++bad;
    __float128 o[9];
    pack(X, o);
    for (int k = 0; k < 9; ++k) split(o[k], inv_hi[k * ip + i], inv_lo[k * ip + i]);
    split(dt.re, det_hi[i], det_lo[i]);
    if (chk) {
      double c[2];
      ge_checks(X, dt, c);
      chk[i] = c[0];
      chk[n + i] = c[1];
    }
  }
  return bad;
}

// FP64 Cholesky form.  piv2: 3 planes of n squared pivots (nullable).
int64_t oracle_chol_f64(int64_t n, const double* z, int64_t zp, double* inv, int64_t ip,
                        double* det, double* piv2, int threads) {
#pragma omp parallel for num_threads(threads) schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    Cx<double> A[3][3];
    unpack(z, zp, i, A);
    double o[9], dt, p2[3];
    cholesky_inv_det(A, o, dt, p2);
    for (int k = 0; k < 9; ++k) inv[k * ip + i] = o[k];
    det[i] = dt;
    if (piv2)
      for (int k = 0; k < 3; ++k) piv2[k * n + i] = p2[k];
  }
  return 0;
}

int64_t oracle_chol_f128(int64_t n, const double* z, int64_t zp, double* inv_hi, double* inv_lo,
                         int64_t ip, double* det_hi, double* det_lo, int threads) {
#pragma omp parallel for num_threads(threads) schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    Cx<__float128> A[3][3];
    unpack(z, zp, i, A);
    __float128 o[9], dt, p2[3];
    cholesky_inv_det(A, o, dt, p2);
    for (int k = 0; k < 9; ++k) split(o[k], inv_hi[k * ip + i], inv_lo[k * ip + i]);
    split(dt, det_hi[i], det_lo[i]);
  }
  return 0;
}

// Positive-definiteness class of each stored matrix, decided by the signs of
// the squared Cholesky pivots in __float128 (Section 3.1 asks only for
// det != 0; a Hermitian matrix is positive definite iff all pivots are > 0).
// 0 = positive definite, 2 = not positive definite, 3 = non-finite input.
int64_t oracle_pd_class(int64_t n, const double* z, int64_t zp, uint8_t* cls, int threads) {
  int64_t not_pd = 0;
#pragma omp parallel for num_threads(threads) schedule(static) reduction(+ : not_pd)
  for (int64_t i = 0; i < n; ++i) {
    if (!finite_input(z, zp, i)) { cls[i] = 3; ++not_pd; continue; }
    Cx<__float128> A[3][3];
    unpack(z, zp, i, A);
    __float128 o[9], dt, p2[3];
    // pivots are evaluated in order and stop at the first non-positive one
    p2[1] = p2[2] = 1;
    if (A[0][0].re <= 0) { cls[i] = 2; ++not_pd; continue; }
    cholesky_inv_det(A, o, dt, p2);
    bool pd = p2[0] > 0 && p2[1] > 0 && p2[2] > 0;
    cls[i] = pd ? 0 : 2;
    if (!pd) ++not_pd;
  }
  return not_pd;
}

// Wishart term and gradient, FP64.  ell: n values; grad: 9 planes (pitch gp).
int64_t oracle_wishart_f64(int64_t n, const double* s, int64_t sp, const double* z, int64_t zp,
                           double n_looks, double* ell, double* grad, int64_t gp, int threads) {
  int64_t bad = 0;
#pragma omp parallel for num_threads(threads) schedule(static) reduction(+ : bad)
  for (int64_t i = 0; i < n; ++i) {
    Cx<double> S[3][3], Z[3][3];
    unpack(s, sp, i, S);
    unpack(z, zp, i, Z);
    double l = 0, g[9] = {0};
    if (!wishart(S, Z, n_looks, l, g)) ++bad;
    ell[i] = l;
    if (grad)
      for (int k = 0; k < 9; ++k) grad[k * gp + i] = g[k];
  }
  return bad;
}

int64_t oracle_wishart_f128(int64_t n, const double* s, int64_t sp, const double* z, int64_t zp,
                            double n_looks, double* ell_hi, double* ell_lo, double* grad_hi,
                            double* grad_lo, int64_t gp, int threads) {
  int64_t bad = 0;
#pragma omp parallel for num_threads(threads) schedule(static) reduction(+ : bad)
  for (int64_t i = 0; i < n; ++i) {
    Cx<__float128> S[3][3], Z[3][3];
    unpack(s, sp, i, S);
    unpack(z, zp, i, Z);
    __float128 l = 0, g[9] = {0};
    if (!wishart(S, Z, (__float128)n_looks, l, g)) ++bad;
    split(l, ell_hi[i], ell_lo[i]);
    if (grad_hi)
      for (int k = 0; k < 9; ++k) split(g[k], grad_hi[k * gp + i], grad_lo[k * gp + i]);
  }
  return bad;
}

// Multilook in __float128: Z (hi, lo) planes (pitch zp) and magnitudes (pitch zp).
int64_t oracle_multilook_f128(int64_t n, const double* looks, int64_t lp, int nl, double* z_hi, double* z_lo,
                              int64_t zp, double* mag, int threads) {
#pragma omp parallel for num_threads(threads) schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    __float128 z[9];
    double m[9];
    multilook(looks, lp, i, nl, z, m);
    for (int k = 0; k < 9; ++k) {
      split(z[k], z_hi[k * zp + i], z_lo[k * zp + i]);
      if (mag) mag[k * zp + i] = m[k];
    }
  }
  return 0;
}

}  // extern "C"
