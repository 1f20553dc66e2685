// Host build of the kernels' per-pixel compensated arithmetic (pixel.hpp),
// for tests: the reroute bound is validated on the CPU and device results
// are compared bitwise against these host results.  The compensated functions use
// explicit FMAs only, so with contraction off the host and device evaluate
// identical operation sequences.
// Build: g++ -O2 -std=c++17 -fPIC -shared -fopenmp -ffp-contract=off
#include <cstdint>

#include "../../paper_1807_08084_amd/csrc/pixel.hpp"

extern "C" {

int64_t host_adjugate_comp_f32(int64_t n, const float* z, int64_t zp, float* inv, float* det, uint8_t* st,
                               float* bound, int threads) {
  int64_t rerouted = 0;
#pragma omp parallel for num_threads(threads) schedule(static) reduction(+ : rerouted)
  for (int64_t i = 0; i < n; ++i) {
    float zz[9], xx[9], d, b;
    for (int k = 0; k < 9; ++k) zz[k] = z[k * zp + i];
    const int s = px::adjugate_comp(zz, xx, d, &b);
    for (int k = 0; k < 9; ++k) inv[k * n + i] = xx[k];
    det[i] = d;
    st[i] = (uint8_t)s;
    bound[i] = b;
    rerouted += s == px::ST_REROUTED;
  }
  return rerouted;
}

int64_t host_adjugate_comp_f64(int64_t n, const double* z, int64_t zp, double* inv, double* det, uint8_t* st,
                               int threads) {
  int64_t bad = 0;
#pragma omp parallel for num_threads(threads) schedule(static) reduction(+ : bad)
  for (int64_t i = 0; i < n; ++i) {
    double zz[9], xx[9], d;
    for (int k = 0; k < 9; ++k) zz[k] = z[k * zp + i];
    const int s = px::adjugate_comp(zz, xx, d);
    for (int k = 0; k < 9; ++k) inv[k * n + i] = xx[k];
    det[i] = d;
    st[i] = (uint8_t)s;
    bad += s != px::ST_OK;
  }
  return bad;
}

// Plain determinant (Eq. detr with the plain cofactors) and its a-priori
// rounding bound, as the Wishart term evaluates them.
void host_det_plain_bound_f32(int64_t n, const float* z, int64_t zp, float* det, float* bound, int threads) {
#pragma omp parallel for num_threads(threads) schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    float zz[9], c[9];
    for (int k = 0; k < 9; ++k) zz[k] = z[k * zp + i];
    px::cofactors_plain(zz, c);
    det[i] = px::det_from_cofactors(zz, c);
    bound[i] = px::det_plain_bound(zz, c);
  }
}

// The error-free additions of the compensated cofactors, element-wise:
// TwoSum (kind 0) or FastTwoSum (kind 1).
void host_sum_pair_f32(int64_t n, const float* a, const float* b, float* s, float* e, int kind) {
  for (int64_t i = 0; i < n; ++i) {
    if (kind) px::fast_two_sum(a[i], b[i], s[i], e[i]);
    else px::two_sum(a[i], b[i], s[i], e[i]);
  }
}

// The three diagonal cofactors in the ordered form, hi + lo, and the order
// flag.
void host_diag_cofactors_f32(int64_t n, const float* z, int64_t zp, float* hi, float* lo, uint8_t* ordered) {
  for (int64_t i = 0; i < n; ++i) {
    float zz[9], rerr[9];
    for (int k = 0; k < 9; ++k) zz[k] = z[k * zp + i];
    px::DW<float> c[9];
    bool ord = true;
    px::cofactors_comp(zz, c, rerr, &ord);
    for (int k = 0; k < 3; ++k) { hi[k * n + i] = c[k].hi; lo[k * n + i] = c[k].lo; }
    ordered[i] = ord ? 1 : 0;
  }
}

}  // extern "C"
