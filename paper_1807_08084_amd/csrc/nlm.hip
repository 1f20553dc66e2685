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
// Blocks cover (TW CPL) x TH output pixels.  For window row offset dy the
// block's lanes need the band of TH input rows y0 + dy .. y0 + dy + TH - 1,
// each TW CPL + 2r columns wide (covariance and inverse or log2 det,
// structure of arrays in LDS).  Consecutive bands share TH - 1 rows, so the
// band is a ring of TH row slots: the first dy stages TH rows, every later dy
// stages only its new bottom row into the slot of the row no lane needs any
// more, and each input row is read from memory once per block (TH + 2r rows
// per TH output rows).  Then every lane sweeps the horizontal neighbours of
// its CPL adjacent outputs in its row of the band.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/polsar.h"
#include "common.hpp"

namespace {
using polsar_dev::xcd_tile;

constexpr int TW = 64, LH = 4, TH = LH, MAX_R = 16;

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
// block's LH x TW lanes own a tile of LH rows and TW * CPL columns: lane
// (tx, ty) computes the outputs of columns CPL tx + j, j < CPL, of row ty.
// With CPL = 2 each neighbour column read from LDS serves both of the lane's
// outputs (2r + 2 reads of 18 values for 2 (2r + 1) pairs); the band then
// keeps even and odd columns in two halves of its row, so that the lanes'
// reads, two columns apart, fall on consecutive words.
template <class T, int DIST, int CPL>
__global__ __launch_bounds__(TW * LH) void k_nlm(NlmArgs a) {
  constexpr int F = DIST == 0 ? 18 : 10;
  // the band, F x TH rows x BW columns; a compile-time row length keeps
  // every band access at a fixed offset from one address per lane
  constexpr int BW = TW * CPL + 2 * MAX_R;
  constexpr int HALF = BW / 2;  // CPL 2: odd columns from here (BW is even)
  static_assert(CPL == 1 || (CPL == 2 && BW % 2 == 0), "one or two columns per lane");
  __shared__ T band[F * TH * BW];
  auto at = [](int col) { return CPL == 2 ? ((col & 1) ? HALF + (col >> 1) : (col >> 1)) : col; };
  const T* __restrict__ Z = (const T*)a.z;
  const T* __restrict__ A = (const T*)a.aux;
  const int tx = threadIdx.x % TW, ty = threadIdx.x / TW;
  const unsigned t = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int64_t x0 = (int64_t)(t % gridDim.x) * (TW * CPL), y0 = (int64_t)(t / gridDim.x) * TH;
  const int64_t py = y0 + ty;
  const int r = a.r, bw = TW * CPL + 2 * r;
  const T N = (T)a.n_looks;
  const T log2e = (T)1.4426950408889634;
  // this lane's pixels: Z_p with the off-diagonal doubled (for tr(Q^-1 P)),
  // and Z_p^-1 with the off-diagonal doubled, or log2 det Z_p; each one's
  // window of staged columns [d0, d1] (clipped at the image's sides)
  bool valid[CPL];
  int d0[CPL], d1[CPL];
  T zp2[CPL][9], ip2[CPL][9], lp[CPL], acc[CPL][9], wsum[CPL];
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int64_t px = x0 + CPL * tx + j;
    valid[j] = px < a.W && py < a.H;
    lp[j] = T(0);
    wsum[j] = T(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) { zp2[j][k] = T(0); ip2[j][k] = T(0); acc[j][k] = T(0); }
    // staged column of neighbour dx: CPL tx + j + dx + r
    const int lo = px >= r ? -r : (int)-px;
    const int hi = a.W - 1 - px >= r ? r : (int)(a.W - 1 - px);
    d0[j] = j + lo + r;
    d1[j] = j + hi + r;
    if (valid[j]) {
      const int64_t i = py * a.W + px;
#pragma unroll
      for (int k = 0; k < 9; ++k) zp2[j][k] = Z[k * a.zp + i] * (k < 3 ? T(1) : T(2));
      if (DIST == 0) {
#pragma unroll
        for (int k = 0; k < 9; ++k) ip2[j][k] = A[k * a.ap + i] * (k < 3 ? T(1) : T(2));
      } else {
        lp[j] = log2_(A[i]);
      }
    }
  }
  // the columns this lane reads: the union of its outputs' windows
  int dlo = 1 << 30, dhi = -1;
#pragma unroll
  for (int j = 0; j < CPL; ++j)
    if (valid[j]) {
      dlo = d0[j] < dlo ? d0[j] : dlo;
      dhi = d1[j] > dhi ? d1[j] : dhi;
    }
  // w = exp2(alpha * s + beta): KL s = t1 + t2; B s = log2 det(Zp + Zq) - (lp + lq)/2
  const T alpha = DIST == 0 ? -N * log2e / (T(2) * (T)a.h) : -N / (T)a.h;
  const T beta = DIST == 0 ? T(3) * N * log2e / (T)a.h : T(3) * N / (T)a.h;
  // input row i of the block (global row y0 - r + i) lives in ring slot i % TH
  auto stage = [&](int i, int col) {
    const int64_t gy = y0 - r + i, gx = x0 - r + col;
    const int slot = i % TH;
    if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) {
      const int64_t g = gy * a.W + gx;
      const int c = at(col);
#pragma unroll
      for (int k = 0; k < 9; ++k) band[(k * TH + slot) * BW + c] = Z[k * a.zp + g];
      if (DIST == 0) {
#pragma unroll
        for (int k = 0; k < 9; ++k) band[((9 + k) * TH + slot) * BW + c] = A[k * a.ap + g];
      } else {
        band[(9 * TH + slot) * BW + c] = log2_(A[g]);
      }
    }
  };
  for (int dy = -r; dy <= r; ++dy) {
    __syncthreads();  // every lane is done with the slot about to be refilled
    if (dy == -r) {
      for (int idx = threadIdx.x; idx < TH * bw; idx += TW * LH) stage(idx / bw, idx % bw);  // the first band
    } else {
      for (int col = threadIdx.x; col < bw; col += TW * LH) stage(TH - 1 + dy + r, col);  // its new bottom row
    }
    __syncthreads();
    // rows y + dy outside the image are not read (an unstaged slot holds
    // stale values)
    const int64_t qy = py + dy;
    if (qy < 0 || qy >= a.H || dhi < 0) continue;
    const int sl = (ty + dy + r) % TH;  // this lane's input row y0 + ty + dy
    for (int d = dlo; d <= dhi; ++d) {
      const int c = at(CPL * tx + d);
      T q[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) q[k] = band[(k * TH + sl) * BW + c];
      T qi[DIST == 0 ? 9 : 1];
      if (DIST == 0) {
#pragma unroll
        for (int k = 0; k < 9; ++k) qi[k] = band[((9 + k) * TH + sl) * BW + c];
      } else {
        qi[0] = band[(9 * TH + sl) * BW + c];
      }
#pragma unroll
      for (int j = 0; j < CPL; ++j) {
        if (!valid[j] || d < d0[j] || d > d1[j]) continue;
        T s;
        if (DIST == 0) {
          // tr(Zp^-1 Zq) + tr(Zq^-1 Zp) as one chain of 18 FMAs
          T tt = ip2[j][0] * q[0];
          tt = fma(qi[0], zp2[j][0], tt);
#pragma unroll
          for (int k = 1; k < 9; ++k) {
            tt = fma(ip2[j][k], q[k], tt);
            tt = fma(qi[k], zp2[j][k], tt);
          }
          s = tt;
        } else {
          // det(Z_p + Z_q): the off-diagonal of zp2 is doubled, halve it back
          T mm[9];
#pragma unroll
          for (int k = 0; k < 9; ++k) mm[k] = zp2[j][k] * (k < 3 ? T(1) : T(0.5)) + q[k];
          T cf[9];
          px::cofactors_plain(mm, cf);
          s = log2_(px::det_from_cofactors(mm, cf)) - T(0.5) * (lp[j] + qi[0]);
        }
        const T w = exp2_(alpha * s + beta);
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[j][k] += w * q[k];
        wsum[j] += w;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    if (!valid[j]) continue;
    const int64_t i = py * a.W + x0 + CPL * tx + j;
    const T inv = T(1) / wsum[j];
#pragma unroll
    for (int k = 0; k < 9; ++k) ((T*)a.out)[k * a.op + i] = acc[j][k] * inv;
    if (a.wsum) ((T*)a.wsum)[i] = wsum[j];
  }
}

// Columns per lane: two in FP32 (on the 4096^2 image at r = 11, KL 10.2 ->
// 9.0 ms, its pairs having been bound by their 18 LDS reads, Bhattacharyya
// 9.7 -> 9.2 ms); one in FP64, whose KL band would take 92 KB of LDS.
template <class T, int DIST> constexpr int nlm_cpl() { return sizeof(T) == 4 ? 2 : 1; }

}  // namespace

extern "C" int polsar_nlm_wishart(int dtype, int distance, int64_t height, int64_t width, int radius,
                                  double n_looks, double h, const void* z, int64_t z_pitch, const void* aux,
                                  int64_t aux_pitch, void* out, int64_t out_pitch, void* wsum, void* stream) {
  if (dtype != POLSAR_F32 && dtype != POLSAR_F64) return POLSAR_E_ARG;
  if (distance != POLSAR_DIST_KL && distance != POLSAR_DIST_BHATTACHARYYA) return POLSAR_E_ARG;
  if (height < 0 || width < 0 || radius < 0 || radius > MAX_R || !(n_looks > 0.0) || !(h > 0.0))
    return POLSAR_E_ARG;
  // one block row of the grid per tile row (LH output rows), at most 65535
  // of them
  const bool kl = distance == POLSAR_DIST_KL;
  if (width > (1 << 20) || height > (int64_t)LH * 65535) return POLSAR_E_ARG;
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
  const int tw = TW * (dtype == POLSAR_F32 ? (kl ? nlm_cpl<float, 0>() : nlm_cpl<float, 1>())
                                           : (kl ? nlm_cpl<double, 0>() : nlm_cpl<double, 1>()));
  const dim3 grid((unsigned)((width + tw - 1) / tw), (unsigned)((height + LH - 1) / LH));
  hipStream_t s = (hipStream_t)stream;
  if (dtype == POLSAR_F32) {
    if (kl) hipLaunchKernelGGL((k_nlm<float, 0, nlm_cpl<float, 0>()>), grid, dim3(TW * LH), 0, s, a);
    else hipLaunchKernelGGL((k_nlm<float, 1, nlm_cpl<float, 1>()>), grid, dim3(TW * LH), 0, s, a);
  } else {
    if (kl) hipLaunchKernelGGL((k_nlm<double, 0, nlm_cpl<double, 0>()>), grid, dim3(TW * LH), 0, s, a);
    else hipLaunchKernelGGL((k_nlm<double, 1, nlm_cpl<double, 1>()>), grid, dim3(TW * LH), 0, s, a);
  }
  return hipGetLastError() == hipSuccess ? POLSAR_OK : POLSAR_E_HIP;
}
