// Nonlocal-means filtering of a PolSAR covariance image with stochastic
// distances between Wishart laws, the consumer the Introduction motivates:
// every pixel compares its covariance with each pixel of a (2r+1)^2 search
// window, which needs the inverse (symmetrized Kullback-Leibler distance) or
// the determinant (Bhattacharyya distance) of every covariance, and the
// filtered covariance is the weighted mean
//     out_p = sum_q w_pq Z_q / sum_q w_pq,   w_pq = exp(-d(Z_p, Z_q) / h).
// Distances between complex Wishart laws of N looks (Frery, Nascimento and
// Cintra, IEEE Trans. Geosci. Remote Sens. 52(2), 2014; the Sigma-free
// terms cancel):
//   KL: d = N/2 (tr(Z_p^-1 Z_q) + tr(Z_q^-1 Z_p)) - 3N
//   B:  d = N (ln det((Z_p + Z_q)/2) - (ln det Z_p + ln det Z_q)/2)
// with tr(AB) = a_A a_B + d_A d_B + f_A f_B + 2 (Re/Im products of b, c, e)
// for Hermitian A, B, and det of the pair mean by the row-0 real-part
// expansion (Eq. detr).  Windows are clipped at the image border.
//
// Blocks cover TW x TH output pixels.  For window row offset dy the block's
// lanes need the band of TH input rows y0 + dy .. y0 + dy + TH - 1, each
// TW + 2r columns wide (covariance and inverse or log2 det, structure of
// arrays in LDS).  Consecutive bands share TH - 1 rows, so the band is a
// ring of TH row slots: the first dy stages TH rows, every later dy stages
// only its new bottom row into the slot of the row no lane needs any more,
// and each input row is read from memory once per block (TH + 2r rows per
// TH output rows).  Then every lane sweeps its 2r+1 horizontal neighbours
// in each of its rows of the band: a block of LH x TW lanes covers
// TH = RPL * LH rows, each lane RPL of them (taller tiles re-read less of
// the 2r-row halo that neighbouring tiles share).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/polsar.h"
#include "common.hpp"

namespace {
using polsar_dev::xcd_tile;

constexpr int TW = 64, LH = 4, MAX_R = 16;

struct NlmArgs {
  const void* z;
  int64_t zp;
  const void* aux;  // KL: 9 inverse planes; B: det plane
  int64_t ap;
  void* out;
  int64_t op;
  void* wsum;
  int64_t H, W;
  int r;
  double n_looks, h;
};

template <class T> __device__ __forceinline__ T exp2_(T x);
// FP32: the hardware's base-2 exponential (within 1 ulp; results below the
// normal range flush, which only drops weights under 2^-126 of the largest)
template <> __device__ __forceinline__ float exp2_(float x) { return __builtin_amdgcn_exp2f(x); }
template <> __device__ __forceinline__ double exp2_(double x) { return exp2(x); }
template <class T> __device__ __forceinline__ T log2_(T x);
// (log2f, not the bare hardware logarithm: determinants of images with tiny
// entries can be subnormal, which log2f scales first)
template <> __device__ __forceinline__ float log2_(float x) { return log2f(x); }
template <> __device__ __forceinline__ double log2_(double x) { return log2(x); }

// DIST 0: symmetrized Kullback-Leibler (F = 18 staged values per pixel:
// Z and Z^-1); DIST 1: Bhattacharyya (F = 10: Z and log2 det Z).  The
// block's LH x TW lanes own a tile of TH = RPL * LH rows: lane (tx, ty)
// computes the outputs of rows ty + m LH, m < RPL.
template <class T, int DIST, int RPL>
__global__ __launch_bounds__(TW * LH) void k_nlm(NlmArgs a) {
  constexpr int TH = RPL * LH;
  constexpr int F = DIST == 0 ? 18 : 10;
  // the band, F x TH rows x BW columns; a compile-time row length keeps
  // every band access at a fixed offset from one address per lane
  constexpr int BW = TW + 2 * MAX_R;
  __shared__ T band[F * TH * BW];
  const T* __restrict__ Z = (const T*)a.z;
  const T* __restrict__ A = (const T*)a.aux;
  const int tx = threadIdx.x % TW, ty = threadIdx.x / TW;
  const unsigned t = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int64_t x0 = (int64_t)(t % gridDim.x) * TW, y0 = (int64_t)(t / gridDim.x) * TH;
  const int64_t px = x0 + tx;
  const int r = a.r, bw = TW + 2 * r;
  const T N = (T)a.n_looks;
  const T log2e = (T)1.4426950408889634;
  // this lane's pixels: Z_p with the off-diagonal doubled (for tr(Q^-1 P)),
  // and Z_p^-1 with the off-diagonal doubled, or log2 det Z_p
  bool valid[RPL];
  T zp2[RPL][9], ip2[RPL][9], lp[RPL], acc[RPL][9], wsum[RPL];
#pragma unroll
  for (int m = 0; m < RPL; ++m) {
    const int64_t py = y0 + ty + m * LH;
    valid[m] = px < a.W && py < a.H;
    lp[m] = T(0);
    wsum[m] = T(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) { zp2[m][k] = T(0); ip2[m][k] = T(0); acc[m][k] = T(0); }
    if (valid[m]) {
      const int64_t i = py * a.W + px;
#pragma unroll
      for (int k = 0; k < 9; ++k) zp2[m][k] = Z[k * a.zp + i] * (k < 3 ? T(1) : T(2));
      if (DIST == 0) {
#pragma unroll
        for (int k = 0; k < 9; ++k) ip2[m][k] = A[k * a.ap + i] * (k < 3 ? T(1) : T(2));
      } else {
        lp[m] = log2_(A[i]);
      }
    }
  }
  // w = exp2(alpha * s + beta): KL s = t1 + t2; B s = log2 det(Zp + Zq) - (lp + lq)/2
  const T alpha = DIST == 0 ? -N * log2e / (T(2) * (T)a.h) : -N / (T)a.h;
  const T beta = DIST == 0 ? T(3) * N * log2e / (T)a.h : T(3) * N / (T)a.h;
  // input row j of the block (global row y0 - r + j) lives in ring slot j % TH
  auto stage = [&](int j, int col) {
    const int64_t gy = y0 - r + j, gx = x0 - r + col;
    const int slot = j % TH;
    if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) {
      const int64_t i = gy * a.W + gx;
#pragma unroll
      for (int k = 0; k < 9; ++k) band[(k * TH + slot) * BW + col] = Z[k * a.zp + i];
      if (DIST == 0) {
#pragma unroll
        for (int k = 0; k < 9; ++k) band[((9 + k) * TH + slot) * BW + col] = A[k * a.ap + i];
      } else {
        band[(9 * TH + slot) * BW + col] = log2_(A[i]);
      }
    }
  };
  const int lo = px >= r ? -r : (int)-px;
  const int hi = a.W - 1 - px >= r ? r : (int)(a.W - 1 - px);
  for (int dy = -r; dy <= r; ++dy) {
    __syncthreads();  // every lane is done with the slot about to be refilled
    if (dy == -r) {
      for (int idx = threadIdx.x; idx < TH * bw; idx += TW * LH) stage(idx / bw, idx % bw);  // the first band
    } else {
      for (int col = threadIdx.x; col < bw; col += TW * LH) stage(TH - 1 + dy + r, col);  // its new bottom row
    }
    __syncthreads();
    // which of this lane's rows have their row y + dy inside the image (the
    // others read no band row: an unstaged slot holds stale values)
    bool use[RPL];
    int sl[RPL];
#pragma unroll
    for (int m = 0; m < RPL; ++m) {
      const int64_t qy = y0 + ty + m * LH + dy;
      use[m] = valid[m] && qy >= 0 && qy < a.H;
      sl[m] = (ty + m * LH + dy + r) % TH;  // this lane's input row y0 + ty + m LH + dy
    }
    for (int dx = lo; dx <= hi; ++dx) {
      const int c = tx + dx + r;
#pragma unroll
      for (int m = 0; m < RPL; ++m) {
        if (!use[m]) continue;
        T q[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) q[k] = band[(k * TH + sl[m]) * BW + c];
        T s;
        if (DIST == 0) {
          // tr(Zp^-1 Zq) + tr(Zq^-1 Zp) as one chain of 18 FMAs
          T tt = ip2[m][0] * q[0];
          tt = fma(band[(9 * TH + sl[m]) * BW + c], zp2[m][0], tt);
#pragma unroll
          for (int k = 1; k < 9; ++k) {
            tt = fma(ip2[m][k], q[k], tt);
            tt = fma(band[((9 + k) * TH + sl[m]) * BW + c], zp2[m][k], tt);
          }
          s = tt;
        } else {
          // det(Z_p + Z_q): the off-diagonal of zp2 is doubled, halve it back
          T mm[9];
#pragma unroll
          for (int k = 0; k < 9; ++k) mm[k] = zp2[m][k] * (k < 3 ? T(1) : T(0.5)) + q[k];
          T cf[9];
          px::cofactors_plain(mm, cf);
          s = log2_(px::det_from_cofactors(mm, cf)) - T(0.5) * (lp[m] + band[(9 * TH + sl[m]) * BW + c]);
        }
        const T w = exp2_(alpha * s + beta);
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[m][k] += w * q[k];
        wsum[m] += w;
      }
    }
  }
#pragma unroll
  for (int m = 0; m < RPL; ++m) {
    if (!valid[m]) continue;
    const int64_t i = (y0 + ty + m * LH) * a.W + px;
    const T inv = T(1) / wsum[m];
#pragma unroll
    for (int k = 0; k < 9; ++k) ((T*)a.out)[k * a.op + i] = acc[m][k] * inv;
    if (a.wsum) ((T*)a.wsum)[i] = wsum[m];
  }
}

// Rows per lane.  One for every form: two (8-row tiles, 30 staged rows per 8
// output rows instead of 26 per 4 at r = 11) were measured on the 4096^2
// FP32 image with r = 11.  KL: 250 instead of 321 B fetched from HBM per
// pixel, but its 55 KB band leaves two blocks per CU and it ran 42% slower
// (14.7 against 10.3 ms).  Bhattacharyya: 1.5% faster, but 64 instead of 47 B
// fetched per pixel.
constexpr int NLM_RPL = 1;

}  // namespace

extern "C" int polsar_nlm_wishart(int dtype, int distance, int64_t height, int64_t width, int radius,
                                  double n_looks, double h, const void* z, int64_t z_pitch, const void* aux,
                                  int64_t aux_pitch, void* out, int64_t out_pitch, void* wsum, void* stream) {
  if (dtype != POLSAR_F32 && dtype != POLSAR_F64) return POLSAR_E_ARG;
  if (distance != POLSAR_DIST_KL && distance != POLSAR_DIST_BHATTACHARYYA) return POLSAR_E_ARG;
  if (height < 0 || width < 0 || radius < 0 || radius > MAX_R || !(n_looks > 0.0) || !(h > 0.0))
    return POLSAR_E_ARG;
  // one block row of the grid per tile row (LH NLM_RPL output rows),
  // at most 65535 of them
  const bool kl = distance == POLSAR_DIST_KL;
  const int th = LH * NLM_RPL;
  if (width > (1 << 20) || height > (int64_t)th * 65535) return POLSAR_E_ARG;
  const int64_t n = height * width;
  const size_t es = dtype == POLSAR_F64 ? 8 : 4;
  const int aux_planes = distance == POLSAR_DIST_KL ? 9 : 1;
  if (n == 0) return POLSAR_OK;
  if (!z || !aux || !out) return POLSAR_E_ARG;
  if (z_pitch < n || out_pitch < n || (aux_planes > 1 && aux_pitch < n)) return POLSAR_E_ARG;
  if ((uintptr_t)z % es || (uintptr_t)aux % es || (uintptr_t)out % es || (wsum && (uintptr_t)wsum % es))
    return POLSAR_E_ALIGN;
  auto lo_hi = [&](const void* p, int planes, int64_t pitch) {
    const uintptr_t lo = (uintptr_t)p;
    return std::make_pair(lo, lo + (uintptr_t)(((planes - 1) * pitch + n) * (int64_t)es));
  };
  auto ov = [](std::pair<uintptr_t, uintptr_t> x, std::pair<uintptr_t, uintptr_t> y) {
    return x.first < y.second && y.first < x.second;
  };
  const auto ro = lo_hi(out, 9, out_pitch);
  if (ov(ro, lo_hi(z, 9, z_pitch)) || ov(ro, lo_hi(aux, aux_planes, aux_pitch))) return POLSAR_E_ALIAS;
  if (wsum) {
    const auto rw = lo_hi(wsum, 1, n);
    if (ov(rw, ro) || ov(rw, lo_hi(z, 9, z_pitch)) || ov(rw, lo_hi(aux, aux_planes, aux_pitch)))
      return POLSAR_E_ALIAS;
  }
  NlmArgs a{z, z_pitch, aux, aux_pitch, out, out_pitch, wsum, height, width, radius, n_looks, h};
  const dim3 grid((unsigned)((width + TW - 1) / TW), (unsigned)((height + th - 1) / th));
  hipStream_t s = (hipStream_t)stream;
  if (dtype == POLSAR_F32) {
    if (kl) hipLaunchKernelGGL((k_nlm<float, 0, NLM_RPL>), grid, dim3(TW * LH), 0, s, a);
    else hipLaunchKernelGGL((k_nlm<float, 1, NLM_RPL>), grid, dim3(TW * LH), 0, s, a);
  } else {
    if (kl) hipLaunchKernelGGL((k_nlm<double, 0, NLM_RPL>), grid, dim3(TW * LH), 0, s, a);
    else hipLaunchKernelGGL((k_nlm<double, 1, NLM_RPL>), grid, dim3(TW * LH), 0, s, a);
  }
  return hipGetLastError() == hipSuccess ? POLSAR_OK : POLSAR_E_HIP;
}
