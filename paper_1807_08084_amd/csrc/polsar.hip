// HIP kernels and C ABI for gfx950: per-pixel 3x3 Hermitian inverse and
// determinant (Alg. 2; Alg. 1 for comparison) and the Wishart term.
//
// Every op is bandwidth-bound streaming over structure-of-arrays planes:
// one lane owns V consecutive pixels (V = 16 or 8 bytes / element size, so
// each plane access is one 128- or 64-bit global load or store), U such
// vectors per tile per lane, and a tile is block*U vectors.  A lane issues
// all of its 9*U (or 18*U) loads before any arithmetic, then all of its
// stores.  Pixels are independent; lanes share only the fixed-order
// reductions of the Wishart sum, the status counters, and the wave's LDS
// queue of FP32 pixels recomputed in FP64.  This file also holds the fused
// multilook (per-pixel looks, and the spatial boxcar form), block-diagonal
// and out-of-core streaming entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/polsar.h"
#include "common.hpp"

namespace {
using namespace polsar_dev;

struct InvDetArgs {
  const void* z;
  int64_t zp;
  void* inv;
  int64_t ip;
  void* det;
  uint8_t* status;
  unsigned long long* counters;
  int64_t n;      // pixels
  int64_t nvec;   // full vectors: n / V
  int64_t tiles;  // ceil(nvec / (block * U)), at least 1
};

// Stores of one pixel-vector's results.
template <class T, int V, bool NT>
__device__ __forceinline__ void store_vec(const InvDetArgs& a, const T (&out)[9][V], const T (&dt)[V],
                                          const int (&st)[V], int64_t v) {
  const int64_t e = v * V;
  if (a.inv) {
    T* inv = (T*)a.inv;
#pragma unroll
    for (int k = 0; k < 9; ++k) store_v<T, V, NT>(inv + k * a.ip + e, out[k]);
  }
  if (a.det) store_v<T, V, NT>((T*)a.det + e, dt);
  if (a.status) store_status<V>(a.status + e, st);
}

// Largest dynamic LDS a launch asks for.
constexpr size_t MAX_DYN_LDS = 64 << 10;

// One pixel-vector of the inverse/determinant with the per-pixel function
// inline (every form but the FP32 compensated one of k_inv_det); the load
// is done by the caller.
template <class T, int OP, int V, bool NT>
__device__ __forceinline__ void inv_det_vec(const InvDetArgs& a, const T (&in)[9][V], int64_t v,
                                            unsigned& c0, unsigned& c1, unsigned& c2) {
  T out[9][V], dt[V];
  int st[V];
#pragma unroll
  for (int l = 0; l < V; ++l) {
    T zz[9], xx[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) zz[k] = in[k][l];
    st[l] = run_pixel<T, OP>(zz, xx, dt[l]);
#pragma unroll
    for (int k = 0; k < 9; ++k) out[k][l] = xx[k];
    tally(st[l], c0, c1, c2);
  }
  store_vec<T, V, NT>(a, out, dt, st, v);
}

template <class T, int OP, int V, int U, bool NT>
__global__ __launch_bounds__(256) void k_inv_det(InvDetArgs a) {
  const T* __restrict__ z = (const T*)a.z;
  const int B = blockDim.x;
  unsigned c0 = 0, c1 = 0, c2 = 0;
  for (int64_t tile = blockIdx.x; tile < a.tiles; tile += gridDim.x) {
    const int64_t v0 = tile * (int64_t)(B * U) + threadIdx.x;
    if constexpr (OP == ADJ_COMP && std::is_same<T, float>::value) {
      // all U vectors through the FP32 step and one shared FP64 queue
      extern __shared__ __align__(16) float polsar_dyn_lds[];
      const int w = threadIdx.x >> 6, nw = B >> 6;
      float* q = polsar_dyn_lds + (size_t)w * 64 * U * V * QUEUE_WORDS;
      uint8_t* qs = (uint8_t*)(polsar_dyn_lds + (size_t)nw * 64 * U * V * QUEUE_WORDS) + w * 64 * U * V;
      bool valid[U];
#pragma unroll
      for (int u = 0; u < U; ++u) valid[u] = v0 + (int64_t)u * B < a.nvec;
      auto load = [&](int u, float (&in)[9][V]) {
#pragma unroll
        for (int k = 0; k < 9; ++k) load_v<float, V, NT>(z + k * a.zp + (v0 + (int64_t)u * B) * V, in[k]);
      };
      float out[U][9][V], dt[U][V];
      int st[U][V];
      comp_f32_wave<U, V>(load, valid, out, dt, st, q, qs);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (!valid[u]) continue;
#pragma unroll
        for (int l = 0; l < V; ++l) tally(st[u][l], c0, c1, c2);
        store_vec<T, V, NT>(a, out[u], dt[u], st[u], v0 + (int64_t)u * B);
      }
    } else {
      T in[U][9][V];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t v = v0 + (int64_t)u * B;
        if (v < a.nvec) {
#pragma unroll
          for (int k = 0; k < 9; ++k) load_v<T, V, NT>(z + k * a.zp + v * V, in[u][k]);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t v = v0 + (int64_t)u * B;
        if (v < a.nvec) inv_det_vec<T, OP, V, NT>(a, in[u], v, c0, c1, c2);
      }
    }
    if (V > 1 && tile == a.tiles - 1) {
      // the n mod V pixels after the last full vector, one per lane
      const int64_t i = a.nvec * V + threadIdx.x;
      if (i < a.n) {
        T zz[9], xx[9], dt;
#pragma unroll
        for (int k = 0; k < 9; ++k) zz[k] = z[k * a.zp + i];
        const int st = run_pixel<T, OP>(zz, xx, dt);
        tally(st, c0, c1, c2);
        if (a.inv)
#pragma unroll
          for (int k = 0; k < 9; ++k) ((T*)a.inv)[k * a.ip + i] = xx[k];
        if (a.det) ((T*)a.det)[i] = dt;
        if (a.status) a.status[i] = (uint8_t)st;
      }
    }
  }
  if (a.counters) flush_counters(a.counters, c0, c1, c2);
}

// ------------------------------------------------------------------ multilook
struct MultilookArgs {
  const void* looks;
  int64_t lp;
  int n_looks;
  double inv_n;  // 1 / n_looks (FP64)
  void* z;  // optional output of the multilook covariance
  int64_t zp;
  InvDetArgs o;  // outputs (o.z unused), n, nvec, tiles
};

// Fused multilook front end + inverse/determinant: per lane V pixels, the N
// looks are streamed (6 planes each) into FP64 accumulators, scaled by 1/N
// (one FP64 multiply per component: exact for N a power of two, else within
// an FP64 rounding of the quotient, far below the storage rounding), Z is
// rounded to the storage type, optionally stored, and inverted exactly as
// k_inv_det inverts a stored Z (the FP32 compensated form through the
// wave's FP64 queue).
template <class T, int OP, int V, bool NT>
__global__ __launch_bounds__(256) void k_multilook(MultilookArgs a) {
  const T* __restrict__ S = (const T*)a.looks;
  const int B = blockDim.x;
  unsigned c0 = 0, c1 = 0, c2 = 0;
  const double inv_n = a.inv_n;
  for (int64_t tile = blockIdx.x; tile < a.o.tiles; tile += gridDim.x) {
    const int64_t v = tile * (int64_t)B + threadIdx.x;
    if (v < a.o.nvec) {
      double acc[V][9];
#pragma unroll
      for (int l = 0; l < V; ++l)
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[l][k] = 0.0;
#pragma unroll 2
      for (int look = 0; look < a.n_looks; ++look) {
        T in[6][V];
#pragma unroll
        for (int j = 0; j < 6; ++j) load_v<T, V, NT>(S + (int64_t)(6 * look + j) * a.lp + v * V, in[j]);
#pragma unroll
        for (int l = 0; l < V; ++l) {
          const T s6[6] = {in[0][l], in[1][l], in[2][l], in[3][l], in[4][l], in[5][l]};
          px::look_accumulate(s6, acc[l]);
        }
      }
      T zz[9][V];
#pragma unroll
      for (int l = 0; l < V; ++l)
#pragma unroll
        for (int k = 0; k < 9; ++k) zz[k][l] = (T)(acc[l][k] * inv_n);
      if (a.z) {
#pragma unroll
        for (int k = 0; k < 9; ++k) store_v<T, V, NT>((T*)a.z + k * a.zp + v * V, zz[k]);
      }
      if constexpr (OP == ADJ_COMP && std::is_same<T, float>::value) {
        extern __shared__ __align__(16) float polsar_dyn_lds[];
        const int w = threadIdx.x >> 6, nw = B >> 6;
        float* q = polsar_dyn_lds + (size_t)w * 64 * V * QUEUE_WORDS;
        uint8_t* qs = (uint8_t*)(polsar_dyn_lds + (size_t)nw * 64 * V * QUEUE_WORDS) + w * 64 * V;
        const bool valid[1] = {true};
        auto load = [&](int, float (&in)[9][V]) {
#pragma unroll
          for (int k = 0; k < 9; ++k)
#pragma unroll
            for (int l = 0; l < V; ++l) in[k][l] = zz[k][l];
        };
        float out[1][9][V], dt[1][V];
        int st[1][V];
        comp_f32_wave<1, V>(load, valid, out, dt, st, q, qs);
#pragma unroll
        for (int l = 0; l < V; ++l) tally(st[0][l], c0, c1, c2);
        store_vec<T, V, NT>(a.o, out[0], dt[0], st[0], v);
      } else {
        inv_det_vec<T, OP, V, NT>(a.o, zz, v, c0, c1, c2);
      }
    }
    if (V > 1 && tile == a.o.tiles - 1) {
      const int64_t i = a.o.nvec * V + threadIdx.x;
      if (i < a.o.n) {
        double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int look = 0; look < a.n_looks; ++look) {
          T s6[6];
#pragma unroll
          for (int j = 0; j < 6; ++j) s6[j] = S[(int64_t)(6 * look + j) * a.lp + i];
          px::look_accumulate(s6, acc);
        }
        T zz[9], xx[9], dt;
#pragma unroll
        for (int k = 0; k < 9; ++k) zz[k] = (T)(acc[k] * inv_n);
        if (a.z)
#pragma unroll
          for (int k = 0; k < 9; ++k) ((T*)a.z)[k * a.zp + i] = zz[k];
        const int st = run_pixel<T, OP>(zz, xx, dt);
        tally(st, c0, c1, c2);
        if (a.o.inv)
#pragma unroll
          for (int k = 0; k < 9; ++k) ((T*)a.o.inv)[k * a.o.ip + i] = xx[k];
        if (a.o.det) ((T*)a.o.det)[i] = dt;
        if (a.o.status) a.o.status[i] = (uint8_t)st;
      }
    }
  }
  if (a.o.counters) flush_counters(a.o.counters, c0, c1, c2);
}

// ------------------------------------------------------------------ boxcar multilook
// Spatial multilook fused with the inverse: Eq. (ZN) with the looks of pixel
// (y, x) taken from its (2R+1) x (2R+1) neighbourhood in a single-look
// image, clipped at the border,
//   Z(y, x) = (1/|W|) sum_{(y', x') in W(y, x)} S(y', x') S(y', x')^H.
// A block (one wave) owns BOX_TW output columns of a strip of box_strip(R)
// rows and walks down it one input row at a time: the row's single-look
// pixels (with an R-pixel halo each side, zeros outside the image, which add
// nothing) are staged in LDS in FP64, double-buffered, while the next row is
// being loaded; each lane forms the sum of its K = 2R+1 horizontal
// neighbours' outer products in FP64 (exact products for FP32 input) and
// adds K consecutive row sums for its output.  Each output is scaled by the
// reciprocal of the clipped window size (within an FP64 ulp of the
// quotient), rounded to the storage type (optionally stored) and inverted
// with the per-pixel function of the per-call kernel.
//
// The vertical sums, without subtraction (so every window keeps the error
// bound of a plain sum of its own terms), two ways:
// * K <= 5 (k_boxcar_shift): the last K row sums sit in registers, oldest
//   first, shifted down one slot per row, and the K of a window are added
//   in ascending row order.
// * K = 7 (k_boxcar_grouped): rows are taken in groups of K, row j of a
//   group going to slot j (the loop over a group is unrolled, so slot
//   indices are compile-time constants and nothing is shifted).  The window
//   that ends at row j of a group is the previous group's rows j+1 .. K-1
//   plus this group's rows 0 .. j: a running prefix sum of this group plus
//   the previous group's suffix sum from row j+1, which the slots hold once
//   a group ends and its suffix sums are formed in place (the scheme of van
//   Herk, and of Gil and Werman, for running maxima, with + for max): about
//   three additions of nine components per output for any K, instead of
//   K-1 plus the shift (7x7 on a 4096^2 image: 44.6-45.3 against 41.6
//   Gpx/s).  The group's K inlined inverses need more registers than the
//   shifted ring's one: at K = 3 and 5 they spilled and ran 25-35% slower.
constexpr int BOX_TW = 64, BOX_MAX_R = 3;
// Strip height: each strip re-forms the row sums of its 2R halo rows, so
// wide windows take taller strips (7x7: 64 rows 4% faster than 32); 3x3
// keeps 32 (64 rows, half the blocks, 5% slower).
constexpr int box_strip(int R) { return R >= 2 ? 64 : 32; }

struct BoxArgs {
  const void* s;
  int64_t sp;
  void* z;
  int64_t zp;
  void* inv;
  int64_t ip;
  void* det;
  uint8_t* status;
  unsigned long long* counters;
  int64_t H, W;
  int64_t nbx;  // blocks across the image
};

// The block's strip and this lane's column.
template <int R>
struct BoxStrip {
  int64_t x0, ys, y_first, y_last, gx, cols;
  __device__ BoxStrip(const BoxArgs& a) {
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t bx = t % a.nbx, by = t / a.nbx;
    x0 = bx * BOX_TW;
    ys = by * box_strip(R);
    const int64_t ye = ys + box_strip(R) < a.H ? ys + box_strip(R) : a.H;
    y_first = ys - R;  // rows staged (outside the image: zeros)
    y_last = ye - 1 + R;
    gx = x0 + threadIdx.x;
    cols = (gx + R < a.W ? gx + R : a.W - 1) - (gx - R > 0 ? gx - R : 0) + 1;
  }
};

// The staged pixels of input row y this lane loads.  Pixels outside the
// image load pixel 0 instead (every load is in bounds and unconditional, so
// the loads stay in flight while the current row is summed) and are staged
// as zeros, which add nothing.
template <class T, int R, int P>
__device__ __forceinline__ void box_load_row(const BoxArgs& a, int64_t x0, int64_t y, T (&v)[P][6], bool (&ok)[P]) {
  constexpr int SW = BOX_TW + 2 * R;
  const T* __restrict__ S = (const T*)a.s;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int col = threadIdx.x + p * BOX_TW;
    const int64_t x = x0 - R + col;
    ok[p] = col < SW && y >= 0 && y < a.H && x >= 0 && x < a.W;
    const int64_t i = ok[p] ? y * a.W + x : 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) v[p][k] = S[k * a.sp + i];
  }
}

// Stage the loaded row in an LDS row buffer, in FP64.
template <class T, int R, int P>
__device__ __forceinline__ void box_stage(double (*row)[BOX_TW + 2 * R], const T (&v)[P][6], const bool (&ok)[P]) {
  constexpr int SW = BOX_TW + 2 * R;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int col = threadIdx.x + p * BOX_TW;
    if (col < SW)
#pragma unroll
      for (int k = 0; k < 6; ++k) row[k][col] = ok[p] ? (double)v[p][k] : 0.0;
  }
}

// This lane's row sum of the staged row: its K horizontal neighbours.
template <int R>
__device__ __forceinline__ void box_row_sum(double (*row)[BOX_TW + 2 * R], double (&sum)[9]) {
  double s6[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) s6[k] = row[k][threadIdx.x];
  px::look_first(s6, sum);
#pragma unroll
  for (int dx = 1; dx < 2 * R + 1; ++dx) {
#pragma unroll
    for (int k = 0; k < 6; ++k) s6[k] = row[k][threadIdx.x + dx];
    px::look_accumulate_chained(s6, sum);
  }
}

// Output row yo of this lane from its window sum: Z, inverse, det, status.
template <class T, int OP, int R>
__device__ __forceinline__ void box_output(const BoxArgs& a, const BoxStrip<R>& b, int64_t yo, const double (&w)[9],
                                           unsigned& c0, unsigned& c1, unsigned& c2) {
  const int64_t rows = (yo + R < a.H ? yo + R : a.H - 1) - (yo - R > 0 ? yo - R : 0) + 1;
  const double rcp = 1.0 / (double)(rows * b.cols);
  T zz[9], xx[9], dt;
#pragma unroll
  for (int c = 0; c < 9; ++c) zz[c] = (T)(w[c] * rcp);
  const int64_t i = yo * a.W + b.gx;
  if (a.z)
#pragma unroll
    for (int c = 0; c < 9; ++c) ((T*)a.z)[c * a.zp + i] = zz[c];
  const int st_px = run_pixel<T, OP>(zz, xx, dt);
  tally(st_px, c0, c1, c2);
  if (a.inv)
#pragma unroll
    for (int c = 0; c < 9; ++c) ((T*)a.inv)[c * a.ip + i] = xx[c];
  if (a.det) ((T*)a.det)[i] = dt;
  if (a.status) a.status[i] = (uint8_t)st_px;
}

template <class T, int OP, int R>
__global__ __launch_bounds__(BOX_TW) void k_boxcar_shift(BoxArgs a) {
  constexpr int K = 2 * R + 1, SW = BOX_TW + 2 * R;
  constexpr int P = (SW + BOX_TW - 1) / BOX_TW;  // staged pixels per lane and row
  __shared__ double row[2][6][SW];
  const BoxStrip<R> b(a);
  double ring[K][9];  // row sums of rows y - 2R .. y, oldest first
#pragma unroll
  for (int m = 0; m < K; ++m)
#pragma unroll
    for (int c = 0; c < 9; ++c) ring[m][c] = 0.0;
  T pre[P][6];
  bool pok[P];
  unsigned c0 = 0, c1 = 0, c2 = 0;
  box_load_row<T, R, P>(a, b.x0, b.y_first, pre, pok);
#pragma unroll 1
  for (int64_t y = b.y_first; y <= b.y_last; ++y) {  // the same for every lane of the block
    const int buf = (int)((y - b.y_first) & 1);
    box_stage<T, R, P>(row[buf], pre, pok);
    __syncthreads();
    if (y + 1 <= b.y_last) box_load_row<T, R, P>(a, b.x0, y + 1, pre, pok);  // in flight while this row is summed
#pragma unroll
    for (int m = 0; m + 1 < K; ++m)
#pragma unroll
      for (int c = 0; c < 9; ++c) ring[m][c] = ring[m + 1][c];
    box_row_sum<R>(row[buf], ring[K - 1]);
    // output row y - R, whose window rows y - 2R .. y the ring now holds
    const int64_t yo = y - R;
    if (yo >= b.ys && b.gx < a.W) {
      double w[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) w[c] = ring[0][c];
#pragma unroll
      for (int m = 1; m < K; ++m)
#pragma unroll
        for (int c = 0; c < 9; ++c) w[c] += ring[m][c];
      box_output<T, OP, R>(a, b, yo, w, c0, c1, c2);
    }
  }
  if (a.counters) flush_counters(a.counters, c0, c1, c2);
}

template <class T, int OP, int R>
__global__ __launch_bounds__(BOX_TW) void k_boxcar_grouped(BoxArgs a) {
  constexpr int K = 2 * R + 1, SW = BOX_TW + 2 * R;
  constexpr int P = (SW + BOX_TW - 1) / BOX_TW;
  __shared__ double row[2][6][SW];
  const BoxStrip<R> b(a);
  // slot j: the row sum of row j of the current group, or, once the group is
  // done, the sum of its rows j .. K-1
  double ring[K][9];
#pragma unroll
  for (int m = 0; m < K; ++m)
#pragma unroll
    for (int c = 0; c < 9; ++c) ring[m][c] = 0.0;
  T pre[P][6];
  bool pok[P];
  unsigned c0 = 0, c1 = 0, c2 = 0;
  box_load_row<T, R, P>(a, b.x0, b.y_first, pre, pok);
#pragma unroll 1
  for (int64_t y0 = b.y_first; y0 <= b.y_last; y0 += K) {  // the same for every lane of the block
    double run[9];  // prefix sum of the group's row sums
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int64_t y = y0 + j;
      if (y > b.y_last) break;
      const int buf = (int)((y - b.y_first) & 1);
      box_stage<T, R, P>(row[buf], pre, pok);
      __syncthreads();
      if (y + 1 <= b.y_last) box_load_row<T, R, P>(a, b.x0, y + 1, pre, pok);
      box_row_sum<R>(row[buf], ring[j]);
#pragma unroll
      for (int c = 0; c < 9; ++c) run[c] = j == 0 ? ring[0][c] : run[c] + ring[j][c];
      // output row y - R: window rows y - 2R .. y
      const int64_t yo = y - R;
      if (yo >= b.ys && b.gx < a.W) {
        double w[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) w[c] = j + 1 < K ? ring[j + 1 < K ? j + 1 : 0][c] + run[c] : run[c];
        box_output<T, OP, R>(a, b, yo, w, c0, c1, c2);
      }
    }
    // the group's suffix sums, for the next group's windows
#pragma unroll
    for (int j = K - 2; j >= 0; --j)
#pragma unroll
      for (int c = 0; c < 9; ++c) ring[j][c] += ring[j + 1][c];
  }
  if (a.counters) flush_counters(a.counters, c0, c1, c2);
}

// ------------------------------------------------------------------ block diagonal
// Pixels whose matrix is block diagonal with K Hermitian 3x3 blocks (several
// frequency bands): each block is inverted on its own, the determinant is the
// product of the block determinants, the status the worst block status.
struct BlockArgs {
  int k;            // blocks per pixel
  void* bdet;       // optional per-block determinants: K planes, pitch bp
  int64_t bp;
  InvDetArgs o;     // z: 9K planes (block b at planes 9b..9b+8), inv likewise
};

template <class T, int OP, int V, bool NT>
__global__ __launch_bounds__(256) void k_blockdiag(BlockArgs a) {
  const T* __restrict__ Z = (const T*)a.o.z;
  const int B = blockDim.x;
  unsigned c0 = 0, c1 = 0, c2 = 0;
  for (int64_t tile = blockIdx.x; tile < a.o.tiles; tile += gridDim.x) {
    const int64_t v = tile * (int64_t)B + threadIdx.x;
    if (v < a.o.nvec) {
      T prod[V];
      int worst[V];
#pragma unroll
      for (int l = 0; l < V; ++l) { prod[l] = T(1); worst[l] = 0; }
      for (int b = 0; b < a.k; ++b) {
        T in[9][V], out[9][V], dt[V];
#pragma unroll
        for (int k = 0; k < 9; ++k) load_v<T, V, NT>(Z + (int64_t)(9 * b + k) * a.o.zp + v * V, in[k]);
#pragma unroll
        for (int l = 0; l < V; ++l) {
          T zz[9], xx[9];
#pragma unroll
          for (int k = 0; k < 9; ++k) zz[k] = in[k][l];
          const int st = run_pixel<T, OP>(zz, xx, dt[l]);
#pragma unroll
          for (int k = 0; k < 9; ++k) out[k][l] = xx[k];
          prod[l] *= dt[l];
          worst[l] = st > worst[l] ? st : worst[l];
        }
        if (a.o.inv)
#pragma unroll
          for (int k = 0; k < 9; ++k) store_v<T, V, NT>((T*)a.o.inv + (int64_t)(9 * b + k) * a.o.ip + v * V, out[k]);
        if (a.bdet) store_v<T, V, NT>((T*)a.bdet + (int64_t)b * a.bp + v * V, dt);
      }
#pragma unroll
      for (int l = 0; l < V; ++l) tally(worst[l], c0, c1, c2);
      if (a.o.det) store_v<T, V, NT>((T*)a.o.det + v * V, prod);
      if (a.o.status) store_status<V>(a.o.status + v * V, worst);
    }
    if (V > 1 && tile == a.o.tiles - 1) {
      const int64_t i = a.o.nvec * V + threadIdx.x;
      if (i < a.o.n) {
        T prod = T(1);
        int worst = 0;
        for (int b = 0; b < a.k; ++b) {
          T zz[9], xx[9], dt;
#pragma unroll
          for (int k = 0; k < 9; ++k) zz[k] = Z[(int64_t)(9 * b + k) * a.o.zp + i];
          const int st = run_pixel<T, OP>(zz, xx, dt);
          prod *= dt;
          worst = st > worst ? st : worst;
          if (a.o.inv)
#pragma unroll
            for (int k = 0; k < 9; ++k) ((T*)a.o.inv)[(int64_t)(9 * b + k) * a.o.ip + i] = xx[k];
          if (a.bdet) ((T*)a.bdet)[(int64_t)b * a.bp + i] = dt;
        }
        tally(worst, c0, c1, c2);
        if (a.o.det) ((T*)a.o.det)[i] = prod;
        if (a.o.status) a.o.status[i] = (uint8_t)worst;
      }
    }
  }
  if (a.o.counters) flush_counters(a.o.counters, c0, c1, c2);
}

// ------------------------------------------------------------------ Wishart
struct WishartArgs {
  const void* s;
  int64_t sp;
  const void* z;
  int64_t zp;
  double n_looks;
  void* ell;
  double* partial;  // one FP64 partial sum per tile (forward)
  const double* grad_loss;
  void* grad;
  int64_t gp;
  unsigned long long* counters;
  int64_t n, nvec, tiles;
  int fwd, bwd;
};

template <class T, int V, bool NT>
__device__ __forceinline__ double wishart_vec(const WishartArgs& a, const T (&s)[9][V], const T (&z)[9][V],
                                              int64_t v, T gscale, unsigned& c0, unsigned& c1, unsigned& c2) {
  T ell[V], g[9][V];
  double acc = 0.0;
#pragma unroll
  for (int l = 0; l < V; ++l) {
    T ss[9], zz[9], gg[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) { ss[k] = s[k][l]; zz[k] = z[k][l]; }
    bool low = false;
    const int st = px::wishart_pixel<T>(ss, zz, (T)a.n_looks, a.fwd, ell[l], a.bwd, gg, gscale,
                                        a.counters ? &low : nullptr);
    tally(st, c0, c1, c2);
    c1 += low;
    if (a.fwd) acc += (double)ell[l];
    if (a.bwd)
#pragma unroll
      for (int k = 0; k < 9; ++k) g[k][l] = gg[k];
  }
  const int64_t e = v * V;
  if (a.fwd && a.ell) store_v<T, V, NT>((T*)a.ell + e, ell);
  if (a.bwd) {
    T* gp = (T*)a.grad;
#pragma unroll
    for (int k = 0; k < 9; ++k) store_v<T, V, NT>(gp + k * a.gp + e, g[k]);
  }
  return acc;
}

template <class T, int V, int U, bool NT>
__global__ __launch_bounds__(256) void k_wishart(WishartArgs a) {
  const T* __restrict__ S = (const T*)a.s;
  const T* __restrict__ Z = (const T*)a.z;
  const int B = blockDim.x;
  const T gscale = a.bwd ? (a.grad_loss ? (T)*a.grad_loss : T(1)) : T(1);
  unsigned c0 = 0, c1 = 0, c2 = 0;
  for (int64_t tile = blockIdx.x; tile < a.tiles; tile += gridDim.x) {
    const int64_t v0 = tile * (int64_t)(B * U) + threadIdx.x;
    T s[U][9][V], z[U][9][V];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t v = v0 + (int64_t)u * B;
      if (v < a.nvec) {
#pragma unroll
        for (int k = 0; k < 9; ++k) load_v<T, V, NT>(S + k * a.sp + v * V, s[u][k]);
#pragma unroll
        for (int k = 0; k < 9; ++k) load_v<T, V, NT>(Z + k * a.zp + v * V, z[u][k]);
      }
    }
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t v = v0 + (int64_t)u * B;
      if (v < a.nvec) acc += wishart_vec<T, V, NT>(a, s[u], z[u], v, gscale, c0, c1, c2);
    }
    if (V > 1 && tile == a.tiles - 1) {
      const int64_t i = a.nvec * V + threadIdx.x;
      if (i < a.n) {
        T ss[9], zz[9], gg[9], el;
#pragma unroll
        for (int k = 0; k < 9; ++k) { ss[k] = S[k * a.sp + i]; zz[k] = Z[k * a.zp + i]; }
        bool low = false;
        const int st = px::wishart_pixel<T>(ss, zz, (T)a.n_looks, a.fwd, el, a.bwd, gg, gscale,
                                            a.counters ? &low : nullptr);
        tally(st, c0, c1, c2);
        c1 += low;
        if (a.fwd) {
          acc += (double)el;
          if (a.ell) ((T*)a.ell)[i] = el;
        }
        if (a.bwd)
#pragma unroll
          for (int k = 0; k < 9; ++k) ((T*)a.grad)[k * a.gp + i] = gg[k];
      }
    }
    if (a.fwd) {
      const double bs = block_sum(acc);
      if (threadIdx.x == 0) a.partial[tile] = bs;
    }
  }
  if (a.counters) flush_counters(a.counters, c0, c1, c2);
}

// Fixed-order sum of `count` partials into *out (one block of REDUCE_BLOCK
// lanes: the 16,384 partials of a 2048x2048 FP32 call take one round of
// sixteen loads per lane).
__global__ __launch_bounds__(REDUCE_BLOCK) void k_reduce(const double* __restrict__ partial, int64_t count,
                                                double* __restrict__ out) {
  const double s = strided_sum(partial, count);
  if (threadIdx.x == 0) *out = s;
}

// ------------------------------------------------------------------ copy probe
// Output plane k is input plane k mod NI when there are at least as many
// outputs as inputs; with fewer outputs it is the sum of the inputs j with
// j mod NO == k, so that every input plane is read (a plane no output used
// would not be loaded at all).
template <class T, int V, int NI, int NO, bool NT>
__global__ __launch_bounds__(256) void k_copy(const T* __restrict__ src, int64_t sp, T* __restrict__ dst,
                                              int64_t dp, int64_t nvec, int64_t n) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < nvec) {
    T in[NI][V];
#pragma unroll
    for (int k = 0; k < NI; ++k) load_v<T, V, NT>(src + k * sp + v * V, in[k]);
    if constexpr (NI > NO) {
#pragma unroll
      for (int j = NO; j < NI; ++j)
#pragma unroll
        for (int l = 0; l < V; ++l) in[j % NO][l] += in[j][l];
    }
#pragma unroll
    for (int k = 0; k < NO; ++k) store_v<T, V, NT>(dst + k * dp + v * V, in[k % NI]);
  }
  if (blockIdx.x == 0) {
    const int64_t i = nvec * V + threadIdx.x;
    if (i < n)
      for (int k = 0; k < NO; ++k) {
        T x = src[(k % NI) * sp + i];
        for (int j = k + NO; j < NI; j += NO) x += src[j * sp + i];
        dst[k * dp + i] = x;
      }
  }
}

// ------------------------------------------------------------------ host side
std::mutex g_mu;
std::map<std::tuple<int, int, int, int>, polsar_launch> g_cfg;

// Defaults from a sweep of all launch shapes on MI355X (4096x4096 image):
// one 128-lane tile per block, one 128-bit vector per lane per plane,
// non-temporal (streaming) loads and stores.
// The Wishart kernel in FP64 with 16-byte accesses needs all 256 VGPRs (one
// wave per SIMD); with 8-byte accesses it runs at three waves per SIMD and
// 20% faster.  blocks_per_cu caps the resident blocks: with 4-5 waves per CU
// the 19 concurrent plane streams of a 3x3 inverse reach ~82% of HBM peak,
// with more they contend.
// Images below this many pixels take the Wishart kernel's launch from op 5
// of the table instead of op 1: on 2048x2048 (2^22 pixels) 8-byte accesses
// in 128-lane blocks, at most 5 per CU, ran the FP32 fused forward+backward
// 9-16% faster than the 4096x4096 image's shape, which is 4% faster there.
constexpr int64_t WISHART_SMALL = int64_t(1) << 23;
// Images of at least this many pixels take the inverse kernel's launch from
// op 6 of the table instead of op 0.  On an 8192x8192 image whose pixels are
// a fifth recomputed in FP64 the FP32 compensated kernel with 8-byte
// accesses ran 15% below its best shape (16-byte accesses in 128-lane
// blocks, at most 8 per CU: four pixels per lane fill the wave's FP64 queue
// twice as well as two), which stays within 3-5% of the best on an
// 8192x8192 image with almost no recomputes; on 4096x4096 images 8-byte
// accesses are 2-5% faster.  The Cholesky forms and the FP32-I/O FP64
// adjugate take the joint best of both 8192x8192 images (1-2% over their
// op-0 shapes); the other forms keep their op-0 shapes.
constexpr int64_t INV_DET_LARGE = int64_t(1) << 25;

polsar_launch default_launch(int op, int dtype, int method, int prec) {
  const bool f64 = dtype == POLSAR_F64, chol = method == POLSAR_CHOLESKY;
  switch (op) {
    case 1:  // FP32: 8-byte accesses, at most 4 blocks per CU (4096^2: 0.774 of HBM against 0.763 with
             // 16-byte accesses and no cap; 8192^2: 0.738 against 0.684).  FP64 shapes with 256-lane blocks
             // reach 0.78 on 4096^2 but fall to 0.58 on 8192^2; 128 lanes, 4 per CU: 0.754 and 0.685
      return f64 ? polsar_launch{128, 1, 0, 1, 8, 4} : polsar_launch{256, 1, 0, 1, 8, 4};
    case 5:  // the Wishart kernel below WISHART_SMALL pixels: more, smaller tiles (FP64 on 2048^2: 5 blocks
             // per CU 0.757 of HBM, the Wishart tuner's pick in every bench run, against 0.689 with 4)
      return f64 ? polsar_launch{128, 1, 0, 1, 8, 5} : polsar_launch{128, 1, 0, 1, 8, 5};
    case 2:  // FP32 compensated: 8-byte accesses, at most 8 blocks of 256 lanes per CU (0.75 of HBM on the
             // four-look 4096x4096 image against 0.67 with 16-byte accesses and no cap)
      if (!f64 && !chol && prec == POLSAR_COMPENSATED) return polsar_launch{256, 1, 0, 1, 8, 8};
      return f64 ? polsar_launch{256, 1, 0, 1, 8, 4} : polsar_launch{128, 1, 0, 1, 16, 0};
    case 3:  // FP32: one block of 128 lanes per tile, 8-byte accesses (64-image batch: 0.72 of HBM, against
             // 0.67 for the best persistent grid, 2 blocks of 256 lanes per CU)
      return f64 ? polsar_launch{256, 1, 2, 1, 16, 6} : polsar_launch{128, 1, 0, 1, 8, 0};
    case 4:  // copy probe: few waves in flight stream best
      return polsar_launch{64, 1, 0, 1, 16, 5};
    case 6:  // the inverse kernel on images of at least INV_DET_LARGE pixels
      if (f64) break;
      if (!chol && prec == POLSAR_COMPENSATED) return polsar_launch{128, 1, 0, 1, 16, 8};
      if (!chol && prec == POLSAR_WIDE) return polsar_launch{64, 1, 0, 1, 16, 5};
      if (chol && prec == POLSAR_PLAIN) return polsar_launch{128, 1, 0, 1, 16, 3};
      if (chol && prec == POLSAR_COMPENSATED) return polsar_launch{128, 1, 0, 1, 16, 8};
      break;
    default:
      break;
  }
  // op 0: winners of the autotuner on 4096x4096 and 8192x8192 images of the
  // same recipe, taken together.  For FP32 compensated the 8-byte access
  // with three waves per SIMD also keeps pixels recomputed in FP64 cheap
  // (images with many of them run best with 16-byte access at the same
  // occupancy, which streams the rest slower).  The FP64 adjugate runs 11%
  // faster on 8192x8192 with 16-byte accesses and 6 single-wave blocks per
  // CU than with 12 waves of 8-byte accesses (1% slower on 4096x4096).
  if (!chol && prec == POLSAR_COMPENSATED) return f64 ? polsar_launch{64, 1, 0, 1, 16, 6} : polsar_launch{128, 1, 0, 1, 8, 8};
  if (chol && prec == POLSAR_PLAIN) return f64 ? polsar_launch{64, 1, 0, 1, 16, 5} : polsar_launch{256, 1, 0, 1, 8, 3};
  if (!chol && prec == POLSAR_PLAIN) return f64 ? polsar_launch{64, 1, 0, 1, 16, 6} : polsar_launch{64, 1, 0, 1, 16, 5};
  if (chol && prec == POLSAR_WIDE) return polsar_launch{64, 2, 0, 1, 16, 0};
  if (chol) return polsar_launch{64, 1, 0, 1, 16, 0};
  return polsar_launch{128, 1, 0, 1, 8, 0};  // adjugate, FP32 storage with FP64 arithmetic
}

// Dynamic LDS bytes for a launch: what the kernel needs, raised so that at
// most blocks_per_cu blocks fit in a compute unit's LDS.
int lds_per_cu() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 160 << 10;
  if (!cached[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess || v <= 0)
      v = 160 << 10;
    cached[dev] = v;
  }
  return cached[dev];
}

size_t launch_lds(const polsar_launch& c, size_t need) {
  if (c.blocks_per_cu <= 0) return need;
  size_t pad = (size_t)lds_per_cu() / (size_t)(c.blocks_per_cu + 1) + 1024;
  pad = std::min<size_t>(pad, MAX_DYN_LDS);
  return std::max(need, pad);
}

polsar_launch get_cfg(int op, int dtype, int method, int prec) {
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_cfg.find(std::make_tuple(op, dtype, method, prec));
  return it == g_cfg.end() ? default_launch(op, dtype, method, prec) : it->second;
}

bool valid_launch(const polsar_launch& c, int op) {
  if (c.block != 64 && c.block != 128 && c.block != 256) return false;
  if (c.unroll != 1 && c.unroll != 2 && !((op == 0 || op == 6) && c.unroll == 4)) return false;
  if ((op == 2 || op == 3 || op == 4) && c.unroll != 1) return false;
  if (op == 4 && c.grid_per_cu != 0) return false;
  if (c.grid_per_cu < 0 || c.grid_per_cu > 64) return false;
  if (c.nontemporal != 0 && c.nontemporal != 1) return false;
  if (c.vector_bytes != 16 && c.vector_bytes != 8) return false;
  if (c.blocks_per_cu < 0 || c.blocks_per_cu > 64) return false;
  return true;
}

int device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) cu = 256;
    cached[dev] = cu;
  }
  return cached[dev];
}

// Blocks of a launch over `tiles` tiles: the launch's persistent grid, or
// one block per tile, and at most COUNTER_GRID_PER_CU blocks per CU when the
// call asks for counters.  Pixels are independent and the Wishart partial
// sums are kept per tile, so results do not depend on the grid.
int64_t launch_grid(const polsar_launch& c, int64_t tiles, bool counters) {
  int gpc = c.grid_per_cu;
  if (counters && (gpc == 0 || gpc > COUNTER_GRID_PER_CU)) gpc = COUNTER_GRID_PER_CU;
  int64_t grid = tiles;
  if (gpc > 0) grid = std::min<int64_t>(grid, (int64_t)gpc * device_cus());
  return grid;
}

inline size_t esize(int dtype) { return dtype == POLSAR_F64 ? 8 : 4; }

// Byte range [lo, hi) spanned by `planes` planes of n elements at `pitch`.
struct Range {
  uintptr_t lo, hi;
};
Range span(const void* p, int planes, int64_t pitch, int64_t n, size_t es) {
  uintptr_t lo = (uintptr_t)p;
  return Range{lo, lo + (uintptr_t)(((planes - 1) * pitch + n) * (int64_t)es)};
}
bool overlap(Range a, Range b) { return a.lo < b.hi && b.lo < a.hi; }

int check_planes(const void* p, int64_t pitch, int64_t n, size_t es) {
  if (!p) return n == 0 ? POLSAR_OK : POLSAR_E_ARG;  // an empty batch may pass null planes
  if (pitch < n || pitch > ((int64_t)1 << 40)) return POLSAR_E_ARG;
  if ((uintptr_t)p % es) return POLSAR_E_ALIGN;
  return POLSAR_OK;
}

bool vec_ok(const void* p, int64_t pitch, size_t es) {
  return p == nullptr || (((uintptr_t)p % 16) == 0 && ((pitch * (int64_t)es) % 16) == 0);
}

int op_code(int method, int prec) {
  if (method == POLSAR_ADJUGATE) return prec == POLSAR_PLAIN ? ADJ_PLAIN : prec == POLSAR_COMPENSATED ? ADJ_COMP : ADJ_WIDE;
  return prec == POLSAR_PLAIN ? CHOL_PLAIN : prec == POLSAR_COMPENSATED ? CHOL_COMP : CHOL_WIDE;
}

// Launch helpers: pick the template instance for (V, U, NT).
template <class T, int OP, int V, int U>
hipError_t go_inv_det(const polsar_launch& c, int64_t grid, InvDetArgs& a, hipStream_t s) {
  const size_t lds =
      launch_lds(c, (OP == ADJ_COMP && std::is_same<T, float>::value) ? comp_queue_bytes(c.block, U * V) : 0);
  if (c.nontemporal)
    hipLaunchKernelGGL((k_inv_det<T, OP, V, U, true>), dim3((unsigned)grid), dim3(c.block), lds, s, a);
  else
    hipLaunchKernelGGL((k_inv_det<T, OP, V, U, false>), dim3((unsigned)grid), dim3(c.block), lds, s, a);
  return hipGetLastError();
}

// Vectors per lane per tile actually used: the compensated FP32 kernel
// takes at most two (four run out of registers), and one where the block's
// shared FP64 queue for two would pass MAX_DYN_LDS.
template <class T, int OP, int V>
int inv_det_unroll(const polsar_launch& c) {
  if constexpr (OP == ADJ_COMP && std::is_same<T, float>::value) {
    const int u = c.unroll > 2 ? 2 : c.unroll;
    return (u == 2 && comp_queue_bytes(c.block, 2 * V) > MAX_DYN_LDS) ? 1 : u;
  } else {
    return c.unroll;
  }
}

template <class T, int OP, int V>
hipError_t dispatch_inv_det_v(const polsar_launch& c, InvDetArgs& a, hipStream_t s) {
  a.nvec = a.n / V;
  const int unroll = inv_det_unroll<T, OP, V>(c);
  const int64_t per_tile = (int64_t)c.block * unroll;
  a.tiles = std::max<int64_t>(1, (a.nvec + per_tile - 1) / per_tile);
  const int64_t grid = launch_grid(c, a.tiles, a.counters != nullptr);
  if (unroll == 1) return go_inv_det<T, OP, V, 1>(c, grid, a, s);
  if constexpr (OP == ADJ_COMP && std::is_same<T, float>::value) {
    return go_inv_det<T, OP, V, 2>(c, grid, a, s);
  } else {
    if (unroll == 2) return go_inv_det<T, OP, V, 2>(c, grid, a, s);
    return go_inv_det<T, OP, V, 4>(c, grid, a, s);
  }
}

// Access width: 16 bytes per lane per plane (V = 16 / sizeof(T) pixels),
// 8 bytes when the launch asks for it, one element when the planes are not
// 16-byte aligned.
template <class T, int OP>
hipError_t dispatch_inv_det(const polsar_launch& c, bool vec, InvDetArgs& a, hipStream_t s) {
  constexpr int VW = 16 / sizeof(T);
  if (!vec) return dispatch_inv_det_v<T, OP, 1>(c, a, s);
  if (c.vector_bytes == 8) return dispatch_inv_det_v<T, OP, VW / 2>(c, a, s);
  return dispatch_inv_det_v<T, OP, VW>(c, a, s);
}

hipError_t launch_inv_det(int dtype, int op, const polsar_launch& c, bool vec, InvDetArgs& a, hipStream_t s) {
  if (dtype == POLSAR_F32) {
    switch (op) {
      case ADJ_PLAIN: return dispatch_inv_det<float, ADJ_PLAIN>(c, vec, a, s);
      case ADJ_COMP: return dispatch_inv_det<float, ADJ_COMP>(c, vec, a, s);
      case ADJ_WIDE: return dispatch_inv_det<float, ADJ_WIDE>(c, vec, a, s);
      case CHOL_PLAIN: return dispatch_inv_det<float, CHOL_PLAIN>(c, vec, a, s);
      case CHOL_COMP: return dispatch_inv_det<float, CHOL_COMP>(c, vec, a, s);
      default: return dispatch_inv_det<float, CHOL_WIDE>(c, vec, a, s);
    }
  }
  switch (op) {
    case ADJ_PLAIN: return dispatch_inv_det<double, ADJ_PLAIN>(c, vec, a, s);
    case ADJ_COMP: return dispatch_inv_det<double, ADJ_COMP>(c, vec, a, s);
    default: return dispatch_inv_det<double, CHOL_PLAIN>(c, vec, a, s);
  }
}

// Validates polsar_inv_det arguments; fills `a` and `vec` on success.
// Valid (dtype, method, precision) combination?
int check_mode(int dtype, int method, int prec) {
  if (dtype != POLSAR_F32 && dtype != POLSAR_F64) return POLSAR_E_ARG;
  if (method != POLSAR_ADJUGATE && method != POLSAR_CHOLESKY) return POLSAR_E_ARG;
  if (prec != POLSAR_PLAIN && prec != POLSAR_COMPENSATED && prec != POLSAR_WIDE) return POLSAR_E_ARG;
  if (dtype == POLSAR_F64 && prec == POLSAR_WIDE) return POLSAR_E_UNSUPPORTED;
  if (dtype == POLSAR_F64 && method == POLSAR_CHOLESKY && prec != POLSAR_PLAIN) return POLSAR_E_UNSUPPORTED;
  return POLSAR_OK;
}

int prepare_inv_det(int dtype, int method, int prec, int64_t n, const void* z, int64_t zp, void* inv,
                    int64_t ip, void* det, uint8_t* status, unsigned long long* counters, InvDetArgs& a,
                    bool& vec) {
  int r0 = check_mode(dtype, method, prec);
  if (r0) return r0;
  if (n < 0) return POLSAR_E_ARG;
  const size_t es = esize(dtype);
  int r = check_planes(z, zp, n, es);
  if (r) return r;
  if (inv && (r = check_planes(inv, ip, n, es))) return r;
  if (det && ((uintptr_t)det % es)) return POLSAR_E_ALIGN;
  if (counters && ((uintptr_t)counters % 8)) return POLSAR_E_ALIGN;
  if (!inv && !det && !status && !counters) return POLSAR_E_ARG;
  if (n > 0) {
    const Range rz = span(z, 9, zp, n, es);
    if (inv) {
      const Range ri = span(inv, 9, ip, n, es);
      if (!(inv == z && ip == zp) && overlap(ri, rz)) return POLSAR_E_ALIAS;
    }
    if (det) {
      const Range rd = span(det, 1, n, n, es);
      if (overlap(rd, rz) || (inv && overlap(rd, span(inv, 9, ip, n, es)))) return POLSAR_E_ALIAS;
    }
    if (status) {
      const Range rs = span(status, 1, n, n, 1);
      if (overlap(rs, rz) || (inv && overlap(rs, span(inv, 9, ip, n, es))) || (det && overlap(rs, span(det, 1, n, n, es))))
        return POLSAR_E_ALIAS;
    }
  }
  a = InvDetArgs{z, zp, inv, ip, det, status, counters, n, 0, 0};
  const int VW = (int)(16 / es);
  vec = vec_ok(z, zp, es) && vec_ok(inv, ip, es) && vec_ok(det, 0, es) &&
        (status == nullptr || ((uintptr_t)status % VW) == 0);
  return POLSAR_OK;
}

// ---- multilook launch
template <class T, int OP, int V>
hipError_t dispatch_multilook_v(const polsar_launch& c, MultilookArgs& a, hipStream_t s) {
  a.o.nvec = a.o.n / V;
  a.o.tiles = std::max<int64_t>(1, (a.o.nvec + c.block - 1) / c.block);
  const int64_t grid = launch_grid(c, a.o.tiles, a.o.counters != nullptr);
  const size_t lds =
      launch_lds(c, (OP == ADJ_COMP && std::is_same<T, float>::value) ? comp_queue_bytes(c.block, V) : 0);
  if (c.nontemporal)
    hipLaunchKernelGGL((k_multilook<T, OP, V, true>), dim3((unsigned)grid), dim3(c.block), lds, s, a);
  else
    hipLaunchKernelGGL((k_multilook<T, OP, V, false>), dim3((unsigned)grid), dim3(c.block), lds, s, a);
  return hipGetLastError();
}

template <class T, int OP>
hipError_t dispatch_multilook(const polsar_launch& c, bool vec, MultilookArgs& a, hipStream_t s) {
  constexpr int VW = 16 / sizeof(T);
  if (!vec) return dispatch_multilook_v<T, OP, 1>(c, a, s);
  if (c.vector_bytes == 8) return dispatch_multilook_v<T, OP, VW / 2>(c, a, s);
  return dispatch_multilook_v<T, OP, VW>(c, a, s);
}

hipError_t launch_multilook(int dtype, int op, const polsar_launch& c, bool vec, MultilookArgs& a, hipStream_t s) {
  if (dtype == POLSAR_F32) {
    switch (op) {
      case ADJ_PLAIN: return dispatch_multilook<float, ADJ_PLAIN>(c, vec, a, s);
      case ADJ_COMP: return dispatch_multilook<float, ADJ_COMP>(c, vec, a, s);
      case ADJ_WIDE: return dispatch_multilook<float, ADJ_WIDE>(c, vec, a, s);
      case CHOL_PLAIN: return dispatch_multilook<float, CHOL_PLAIN>(c, vec, a, s);
      case CHOL_COMP: return dispatch_multilook<float, CHOL_COMP>(c, vec, a, s);
      default: return dispatch_multilook<float, CHOL_WIDE>(c, vec, a, s);
    }
  }
  switch (op) {
    case ADJ_PLAIN: return dispatch_multilook<double, ADJ_PLAIN>(c, vec, a, s);
    case ADJ_COMP: return dispatch_multilook<double, ADJ_COMP>(c, vec, a, s);
    default: return dispatch_multilook<double, CHOL_PLAIN>(c, vec, a, s);
  }
}

// ---- boxcar launch: one block (one wave) per BOX_TW columns x box_strip(R) rows,
// a 1-D grid; the radius is a template parameter (the ring of row sums is
// indexed at compile time)
template <class T, int OP, int R>
hipError_t go_boxcar_r(BoxArgs& a, hipStream_t s) {
  a.nbx = (a.W + BOX_TW - 1) / BOX_TW;
  const int64_t nby = (a.H + box_strip(R) - 1) / box_strip(R);
  if constexpr (R <= 2)
    hipLaunchKernelGGL((k_boxcar_shift<T, OP, R>), dim3((unsigned)(a.nbx * nby)), dim3(BOX_TW), 0, s, a);
  else
    hipLaunchKernelGGL((k_boxcar_grouped<T, OP, R>), dim3((unsigned)(a.nbx * nby)), dim3(BOX_TW), 0, s, a);
  return hipGetLastError();
}

template <class T, int OP>
hipError_t go_boxcar(BoxArgs& a, int r, hipStream_t s) {
  switch (r) {
    case 0: return go_boxcar_r<T, OP, 0>(a, s);
    case 1: return go_boxcar_r<T, OP, 1>(a, s);
    case 2: return go_boxcar_r<T, OP, 2>(a, s);
    default: return go_boxcar_r<T, OP, 3>(a, s);
  }
}

hipError_t launch_boxcar(int dtype, int op, BoxArgs& a, int r, hipStream_t s) {
  if (dtype == POLSAR_F32) {
    switch (op) {
      case ADJ_PLAIN: return go_boxcar<float, ADJ_PLAIN>(a, r, s);
      case ADJ_COMP: return go_boxcar<float, ADJ_COMP>(a, r, s);
      case ADJ_WIDE: return go_boxcar<float, ADJ_WIDE>(a, r, s);
      case CHOL_PLAIN: return go_boxcar<float, CHOL_PLAIN>(a, r, s);
      case CHOL_COMP: return go_boxcar<float, CHOL_COMP>(a, r, s);
      default: return go_boxcar<float, CHOL_WIDE>(a, r, s);
    }
  }
  switch (op) {
    case ADJ_PLAIN: return go_boxcar<double, ADJ_PLAIN>(a, r, s);
    case ADJ_COMP: return go_boxcar<double, ADJ_COMP>(a, r, s);
    default: return go_boxcar<double, CHOL_PLAIN>(a, r, s);
  }
}

// ---- block-diagonal launch
template <class T, int OP, int V>
hipError_t dispatch_block_v(const polsar_launch& c, BlockArgs& a, hipStream_t s) {
  a.o.nvec = a.o.n / V;
  a.o.tiles = std::max<int64_t>(1, (a.o.nvec + c.block - 1) / c.block);
  const int64_t grid = launch_grid(c, a.o.tiles, a.o.counters != nullptr);
  const size_t lds = launch_lds(c, 0);
  if (c.nontemporal)
    hipLaunchKernelGGL((k_blockdiag<T, OP, V, true>), dim3((unsigned)grid), dim3(c.block), lds, s, a);
  else
    hipLaunchKernelGGL((k_blockdiag<T, OP, V, false>), dim3((unsigned)grid), dim3(c.block), lds, s, a);
  return hipGetLastError();
}

template <class T, int OP>
hipError_t dispatch_block(const polsar_launch& c, bool vec, BlockArgs& a, hipStream_t s) {
  constexpr int VW = 16 / sizeof(T);
  return vec ? dispatch_block_v<T, OP, VW>(c, a, s) : dispatch_block_v<T, OP, 1>(c, a, s);
}

hipError_t launch_block(int dtype, int op, const polsar_launch& c, bool vec, BlockArgs& a, hipStream_t s) {
  if (dtype == POLSAR_F32) {
    switch (op) {
      case ADJ_PLAIN: return dispatch_block<float, ADJ_PLAIN>(c, vec, a, s);
      case ADJ_COMP: return dispatch_block<float, ADJ_COMP>(c, vec, a, s);
      case ADJ_WIDE: return dispatch_block<float, ADJ_WIDE>(c, vec, a, s);
      case CHOL_PLAIN: return dispatch_block<float, CHOL_PLAIN>(c, vec, a, s);
      case CHOL_COMP: return dispatch_block<float, CHOL_COMP>(c, vec, a, s);
      default: return dispatch_block<float, CHOL_WIDE>(c, vec, a, s);
    }
  }
  switch (op) {
    case ADJ_PLAIN: return dispatch_block<double, ADJ_PLAIN>(c, vec, a, s);
    case ADJ_COMP: return dispatch_block<double, ADJ_COMP>(c, vec, a, s);
    default: return dispatch_block<double, CHOL_PLAIN>(c, vec, a, s);
  }
}

// ---- Wishart launch
template <class T, int V, int U>
hipError_t go_wishart(const polsar_launch& c, int64_t grid, WishartArgs& a, hipStream_t s) {
  const size_t lds = launch_lds(c, 0);
  if (c.nontemporal)
    hipLaunchKernelGGL((k_wishart<T, V, U, true>), dim3((unsigned)grid), dim3(c.block), lds, s, a);
  else
    hipLaunchKernelGGL((k_wishart<T, V, U, false>), dim3((unsigned)grid), dim3(c.block), lds, s, a);
  return hipGetLastError();
}

// Pixels per access of a Wishart launch, and its tiles (one partial sum each).
int wishart_vector(const polsar_launch& c, bool vec, size_t es) {
  const int vw = (int)(16 / es);
  return !vec ? 1 : (c.vector_bytes == 8 ? vw / 2 : vw);
}
int64_t wishart_tiles(const polsar_launch& c, int v, int64_t n) {
  const int64_t per_tile = (int64_t)c.block * c.unroll;
  return std::max<int64_t>(1, (n / v + per_tile - 1) / per_tile);
}

template <class T, int V>
hipError_t dispatch_wishart_v(const polsar_launch& c, WishartArgs& a, hipStream_t s) {
  a.nvec = a.n / V;
  a.tiles = wishart_tiles(c, V, a.n);
  const int64_t grid = launch_grid(c, a.tiles, a.counters != nullptr);
  return c.unroll == 1 ? go_wishart<T, V, 1>(c, grid, a, s) : go_wishart<T, V, 2>(c, grid, a, s);
}

template <class T>
hipError_t dispatch_wishart(const polsar_launch& c, bool vec, WishartArgs& a, hipStream_t s) {
  constexpr int VW = 16 / sizeof(T);
  if (!vec) return dispatch_wishart_v<T, 1>(c, a, s);
  if (c.vector_bytes == 8) return dispatch_wishart_v<T, VW / 2>(c, a, s);
  return dispatch_wishart_v<T, VW>(c, a, s);
}

// Wishart partial sums (one per tile) of any launch shape: the smallest
// tile is 64 lanes x 1 vector of one element.
int64_t max_wishart_partials(int64_t n) { return std::max<int64_t>(1, (n + 63) / 64); }

}  // namespace

// LDS bytes of a launch with this shape (shared with the batch kernel).
size_t polsar_launch_lds_bytes(const polsar_launch& c, size_t need) { return launch_lds(c, need); }

// ============================================================== C ABI
struct polsar_batch;  // defined in batch.hip

extern "C" {

const char* polsar_version(void) { return "polsar-mi355x 0.1 (gfx950)"; }

int64_t polsar_recommended_pitch(int dtype, int64_t n) {
  if ((dtype != POLSAR_F32 && dtype != POLSAR_F64) || n < 0) return -1;
  const int64_t es = (int64_t)esize(dtype);
  const int64_t blk = (64 << 10) / es, half = (32 << 10) / es;
  return (n + blk - 1) / blk * blk + half;
}

const char* polsar_status_string(int status) {
  switch (status) {
    case POLSAR_OK: return "ok";
    case POLSAR_E_ARG: return "invalid argument";
    case POLSAR_E_ALIGN: return "misaligned pointer";
    case POLSAR_E_UNSUPPORTED: return "unsupported combination";
    case POLSAR_E_HIP: return "HIP runtime error";
    case POLSAR_E_WORKSPACE: return "workspace missing or too small";
    case POLSAR_E_ALIAS: return "outputs overlap inputs";
    default: return "unknown status";
  }
}

int polsar_device_compute_units(int* cus) {
  if (!cus) return POLSAR_E_ARG;
  *cus = device_cus();
  return POLSAR_OK;
}

int polsar_wishart_launch_op(int64_t n) { return n < WISHART_SMALL ? 5 : 1; }

int polsar_inv_det_launch_op(int64_t n) { return n >= INV_DET_LARGE ? 6 : 0; }

int polsar_get_launch(int op, int dtype, int method, int precision, polsar_launch* out) {
  if (!out || op < 0 || op > 6) return POLSAR_E_ARG;
  *out = get_cfg(op, dtype, method, precision);
  return POLSAR_OK;
}

int polsar_set_launch(int op, int dtype, int method, int precision, const polsar_launch* cfg) {
  if (!cfg || op < 0 || op > 6 || !valid_launch(*cfg, op)) return POLSAR_E_ARG;
  std::lock_guard<std::mutex> g(g_mu);
  g_cfg[std::make_tuple(op, dtype, method, precision)] = *cfg;
  return POLSAR_OK;
}

int polsar_inv_det(int dtype, int method, int precision, int64_t n, const void* z, int64_t z_pitch, void* inv,
                   int64_t inv_pitch, void* det, uint8_t* status, unsigned long long* counters, void* stream) {
  InvDetArgs a;
  bool vec = false;
  int r = prepare_inv_det(dtype, method, precision, n, z, z_pitch, inv, inv_pitch, det, status, counters, a, vec);
  if (r) return r;
  if (n == 0) return POLSAR_OK;
  const polsar_launch c = get_cfg(polsar_inv_det_launch_op(n), dtype, method, precision);
  if (launch_inv_det(dtype, op_code(method, precision), c, vec, a, (hipStream_t)stream) != hipSuccess)
    return POLSAR_E_HIP;
  return POLSAR_OK;
}

int polsar_multilook_inv_det(int dtype, int method, int precision, int64_t n, int n_looks, const void* looks,
                             int64_t looks_pitch, void* z, int64_t z_pitch, void* inv, int64_t inv_pitch,
                             void* det, uint8_t* status, unsigned long long* counters, void* stream) {
  int r = check_mode(dtype, method, precision);
  if (r) return r;
  if (n < 0 || n_looks < 1 || n_looks > 4096) return POLSAR_E_ARG;
  const size_t es = esize(dtype);
  if ((r = check_planes(looks, looks_pitch, n, es))) return r;
  if (z && (r = check_planes(z, z_pitch, n, es))) return r;
  if (inv && (r = check_planes(inv, inv_pitch, n, es))) return r;
  if (det && ((uintptr_t)det % es)) return POLSAR_E_ALIGN;
  if (counters && ((uintptr_t)counters % 8)) return POLSAR_E_ALIGN;
  if (!z && !inv && !det && !status && !counters) return POLSAR_E_ARG;
  if (n > 0) {
    const Range rl = span(looks, 6 * n_looks, looks_pitch, n, es);
    const Range rz = z ? span(z, 9, z_pitch, n, es) : Range{0, 0};
    const Range ri = inv ? span(inv, 9, inv_pitch, n, es) : Range{0, 0};
    const Range rd = det ? span(det, 1, n, n, es) : Range{0, 0};
    const Range rs = status ? span(status, 1, n, n, 1) : Range{0, 0};
    const Range all[5] = {rl, rz, ri, rd, rs};
    for (int p = 0; p < 5; ++p)
      for (int q = p + 1; q < 5; ++q)
        if (all[p].hi > all[p].lo && all[q].hi > all[q].lo && overlap(all[p], all[q])) return POLSAR_E_ALIAS;
  }
  if (n == 0) return POLSAR_OK;
  MultilookArgs a{looks, looks_pitch, n_looks, 1.0 / n_looks, z, z_pitch,
                  InvDetArgs{nullptr, 0, inv, inv_pitch, det, status, counters, n, 0, 0}};
  const bool vec = vec_ok(looks, looks_pitch, es) && vec_ok(z, z_pitch, es) && vec_ok(inv, inv_pitch, es) && vec_ok(det, 0, es) &&
        (status == nullptr || ((uintptr_t)status % (16 / es)) == 0);
  const polsar_launch c = get_cfg(2, dtype, method, precision);
  if (launch_multilook(dtype, op_code(method, precision), c, vec, a, (hipStream_t)stream) != hipSuccess)
    return POLSAR_E_HIP;
  return POLSAR_OK;
}

int polsar_boxcar_inv_det(int dtype, int method, int precision, int64_t height, int64_t width, int radius,
                          const void* s, int64_t s_pitch, void* z, int64_t z_pitch, void* inv, int64_t inv_pitch,
                          void* det, uint8_t* status, unsigned long long* counters, void* stream) {
  int r = check_mode(dtype, method, precision);
  if (r) return r;
  if (height < 0 || width < 0 || radius < 0 || radius > BOX_MAX_R) return POLSAR_E_ARG;
  if (height > ((int64_t)1 << 24) || width > ((int64_t)1 << 24)) return POLSAR_E_ARG;
  const int64_t n = height * width;
  // one block per 64 columns of a strip of 32 or 64 rows: at most ~2^21
  // blocks, a 1-D grid
  if (n > ((int64_t)1 << 32)) return POLSAR_E_ARG;
  const size_t es = esize(dtype);
  if ((r = check_planes(s, s_pitch, n, es))) return r;
  if (z && (r = check_planes(z, z_pitch, n, es))) return r;
  if (inv && (r = check_planes(inv, inv_pitch, n, es))) return r;
  if (det && ((uintptr_t)det % es)) return POLSAR_E_ALIGN;
  if (counters && ((uintptr_t)counters % 8)) return POLSAR_E_ALIGN;
  if (!z && !inv && !det && !status && !counters) return POLSAR_E_ARG;
  if (n > 0) {
    const Range rl = span(s, 6, s_pitch, n, es);
    const Range rz = z ? span(z, 9, z_pitch, n, es) : Range{0, 0};
    const Range ri = inv ? span(inv, 9, inv_pitch, n, es) : Range{0, 0};
    const Range rd = det ? span(det, 1, n, n, es) : Range{0, 0};
    const Range rs = status ? span(status, 1, n, n, 1) : Range{0, 0};
    const Range all[5] = {rl, rz, ri, rd, rs};
    for (int p = 0; p < 5; ++p)
      for (int q = p + 1; q < 5; ++q)
        if (all[p].hi > all[p].lo && all[q].hi > all[q].lo && overlap(all[p], all[q])) return POLSAR_E_ALIAS;
  }
  if (n == 0) return POLSAR_OK;
  BoxArgs a{s, s_pitch, z, z_pitch, inv, inv_pitch, det, status, counters, height, width, 0};
  if (launch_boxcar(dtype, op_code(method, precision), a, radius, (hipStream_t)stream) != hipSuccess)
    return POLSAR_E_HIP;
  return POLSAR_OK;
}

int polsar_blockdiag_inv_det(int dtype, int method, int precision, int64_t n, int n_blocks, const void* z,
                             int64_t z_pitch, void* inv, int64_t inv_pitch, void* det, void* block_det,
                             int64_t block_det_pitch, uint8_t* status, unsigned long long* counters, void* stream) {
  int r = check_mode(dtype, method, precision);
  if (r) return r;
  if (n < 0 || n_blocks < 1 || n_blocks > 1024) return POLSAR_E_ARG;
  const size_t es = esize(dtype);
  if ((r = check_planes(z, z_pitch, n, es))) return r;
  if (inv && (r = check_planes(inv, inv_pitch, n, es))) return r;
  if (block_det && (r = check_planes(block_det, block_det_pitch, n, es))) return r;
  if (det && ((uintptr_t)det % es)) return POLSAR_E_ALIGN;
  if (counters && ((uintptr_t)counters % 8)) return POLSAR_E_ALIGN;
  if (!inv && !det && !block_det && !status && !counters) return POLSAR_E_ARG;
  if (n > 0) {
    const int P = 9 * n_blocks;
    const Range rz = span(z, P, z_pitch, n, es);
    const Range ri = inv ? span(inv, P, inv_pitch, n, es) : Range{0, 0};
    const Range rd = det ? span(det, 1, n, n, es) : Range{0, 0};
    const Range rb = block_det ? span(block_det, n_blocks, block_det_pitch, n, es) : Range{0, 0};
    const Range rs = status ? span(status, 1, n, n, 1) : Range{0, 0};
    const Range all[5] = {rz, ri, rd, rb, rs};
    for (int p = 0; p < 5; ++p)
      for (int q = p + 1; q < 5; ++q) {
        if (p == 0 && q == 1 && inv == z && inv_pitch == z_pitch) continue;  // in place
        if (all[p].hi > all[p].lo && all[q].hi > all[q].lo && overlap(all[p], all[q])) return POLSAR_E_ALIAS;
      }
  }
  if (n == 0) return POLSAR_OK;
  BlockArgs a{n_blocks, block_det, block_det_pitch, InvDetArgs{z, z_pitch, inv, inv_pitch, det, status, counters, n, 0, 0}};
  const bool vec = vec_ok(z, z_pitch, es) && vec_ok(inv, inv_pitch, es) && vec_ok(det, 0, es) &&
                   vec_ok(block_det, block_det_pitch, es) && (status == nullptr || ((uintptr_t)status % (16 / es)) == 0);
  const polsar_launch c = get_cfg(0, dtype, method, precision);
  if (launch_block(dtype, op_code(method, precision), c, vec, a, (hipStream_t)stream) != hipSuccess) return POLSAR_E_HIP;
  return POLSAR_OK;
}

size_t polsar_wishart_workspace_bytes(int dtype, int64_t n) {
  if (n < 0) return 0;
  (void)dtype;  // the partials are FP64 for either storage type
  return (size_t)max_wishart_partials(n) * sizeof(double);
}

}  // extern "C"

// polsar_wishart_loglik and its allocation-free variant: validation and
// launch with the per-tile partial sums at `ws` (ws_words words of 8 bytes):
// the caller's workspace (its size is checked against the largest tile count
// of any launch), or, when fixed_ws is given, the library's fixed scratch of
// ws_words words (checked against this launch's tile count), whose device
// address fixed_ws returns once every argument has passed validation.
int polsar_wishart_call(int dtype, int pass, int64_t n, const void* sigma, int64_t s_pitch, const void* z,
                        int64_t z_pitch, double n_looks, double* loss, void* ell, const double* grad_loss, void* grad,
                        int64_t g_pitch, double* ws, int64_t ws_words, int (*fixed_ws)(double**),
                        unsigned long long* counters, void* stream) {
  const bool ws_user = fixed_ws == nullptr;
  if (dtype != POLSAR_F32 && dtype != POLSAR_F64) return POLSAR_E_ARG;
  if (pass != POLSAR_FWD && pass != POLSAR_BWD && pass != POLSAR_FWD_BWD) return POLSAR_E_ARG;
  if (n < 0 || !(n_looks > 0.0)) return POLSAR_E_ARG;
  const bool fwd = pass & POLSAR_FWD, bwd = pass & POLSAR_BWD;
  const size_t es = esize(dtype);
  int r = check_planes(sigma, s_pitch, n, es);
  if (r) return r;
  if ((r = check_planes(z, z_pitch, n, es))) return r;
  if (fwd && !loss) return POLSAR_E_ARG;
  if (loss && ((uintptr_t)loss % 8)) return POLSAR_E_ALIGN;
  if (grad_loss && ((uintptr_t)grad_loss % 8)) return POLSAR_E_ALIGN;
  if (ell && ((uintptr_t)ell % es)) return POLSAR_E_ALIGN;
  if (counters && ((uintptr_t)counters % 8)) return POLSAR_E_ALIGN;
  if (bwd && (r = check_planes(grad, g_pitch, n, es))) return r;
  if (fwd && n > 0 && ws_user) {
    if (!ws || ws_words < max_wishart_partials(n)) return POLSAR_E_WORKSPACE;
    if ((uintptr_t)ws % 8) return POLSAR_E_ALIGN;
  }
  if (n > 0) {
    const Range rs = span(sigma, 9, s_pitch, n, es), rz = span(z, 9, z_pitch, n, es);
    if (bwd) {
      const Range rg = span(grad, 9, g_pitch, n, es);
      if (overlap(rg, rs) || overlap(rg, rz)) return POLSAR_E_ALIAS;
    }
    if (fwd && ell) {
      const Range re = span(ell, 1, n, n, es);
      if (overlap(re, rs) || overlap(re, rz) || (bwd && overlap(re, span(grad, 9, g_pitch, n, es))))
        return POLSAR_E_ALIAS;
    }
  }
  const bool vec = n > 0 && vec_ok(sigma, s_pitch, es) && vec_ok(z, z_pitch, es) &&
                   (!bwd || vec_ok(grad, g_pitch, es)) && (!(fwd && ell) || vec_ok(ell, 0, es));
  const polsar_launch c = get_cfg(polsar_wishart_launch_op(n), dtype, 0, 0);
  if (fwd && n > 0 && !ws_user) {
    if (wishart_tiles(c, wishart_vector(c, vec, es), n) > ws_words) return POLSAR_E_WORKSPACE;
    if ((r = fixed_ws(&ws))) return r;
  }
  hipStream_t s = (hipStream_t)stream;
  if (n == 0) {
    if (fwd) {
      // an empty sum is zero: reduce zero partials
      hipLaunchKernelGGL(k_reduce, dim3(1), dim3(REDUCE_BLOCK), 0, s, (const double*)nullptr, (int64_t)0, loss);
      if (hipGetLastError() != hipSuccess) return POLSAR_E_HIP;
    }
    return POLSAR_OK;
  }
  WishartArgs a{sigma, s_pitch, z, z_pitch, n_looks, fwd ? ell : nullptr, fwd ? ws : nullptr, grad_loss,
                bwd ? grad : nullptr, g_pitch, counters, n, 0, 0, fwd ? 1 : 0, bwd ? 1 : 0};
  hipError_t e = dtype == POLSAR_F32 ? dispatch_wishart<float>(c, vec, a, s) : dispatch_wishart<double>(c, vec, a, s);
  if (e != hipSuccess) return POLSAR_E_HIP;
  if (fwd) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(REDUCE_BLOCK), 0, s, (const double*)ws, a.tiles, loss);
    if (hipGetLastError() != hipSuccess) return POLSAR_E_HIP;
  }
  return POLSAR_OK;
}

extern "C" {

int polsar_wishart_loglik(int dtype, int pass, int64_t n, const void* sigma, int64_t s_pitch, const void* z,
                          int64_t z_pitch, double n_looks, double* loss, void* ell, const double* grad_loss,
                          void* grad, int64_t g_pitch, void* workspace, size_t ws_bytes,
                          unsigned long long* counters, void* stream) {
  return polsar_wishart_call(dtype, pass, n, sigma, s_pitch, z, z_pitch, n_looks, loss, ell, grad_loss, grad, g_pitch,
                      (double*)workspace, (int64_t)(ws_bytes / sizeof(double)), nullptr, counters, stream);
}

int polsar_autotune_inv_det(int dtype, int method, int precision, int64_t n, const void* z, int64_t z_pitch,
                            void* inv, int64_t inv_pitch, void* det, int reps, polsar_launch* best,
                            float* best_ms, void* stream) {
  InvDetArgs a;
  bool vec = false;
  int r = prepare_inv_det(dtype, method, precision, n, z, z_pitch, inv, inv_pitch, det, nullptr, nullptr, a, vec);
  if (r) return r;
  if (n == 0 || reps <= 0) return POLSAR_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return POLSAR_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return POLSAR_E_HIP;
  }
  const int op = op_code(method, precision);
  polsar_launch win{0, 0, 0, 0, 0, 0};
  float win_ms = 1e30f;
  int rc = POLSAR_OK;
  // mean time per call of `reps` back-to-back calls with launch c, after one
  // untimed call; negative on a HIP error
  auto time_cfg = [&](const polsar_launch& c) -> float {
    InvDetArgs aa = a;
    if (launch_inv_det(dtype, op, c, vec, aa, s) != hipSuccess) return -1.f;
    (void)hipEventRecord(e0, s);
    for (int i = 0; i < reps; ++i) {
      aa = a;
      (void)launch_inv_det(dtype, op, c, vec, aa, s);
    }
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) return -1.f;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return ms / reps;
  };
  // Stage 1, every candidate once: block x unroll x {one tile per block,
  // 8 blocks per CU persistent} x access width x resident-block cap, with
  // streaming accesses.  Stage 2: the six fastest again, in three
  // interleaved passes, ranked by their best pass (single timings of
  // neighbouring candidates differ by a few percent from run to run).
  std::vector<std::pair<float, polsar_launch>> all;
  for (int block : {64, 128, 256})
    for (int unroll : {1, 2})
      for (int gpc : {0, 8})
        for (int vb : {16, 8})
          for (int bpc : {0, 2, 3, 4, 5, 6, 8}) {
            const polsar_launch c{block, unroll, gpc, 1, vb, bpc};
            const float ms = time_cfg(c);
            if (ms < 0.f) { rc = POLSAR_E_HIP; goto done; }
            all.emplace_back(ms, c);
          }
  std::sort(all.begin(), all.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
  all.resize(std::min<size_t>(all.size(), 6));
  for (auto& e : all) e.first = 1e30f;
  for (int pass = 0; pass < 3; ++pass)
    for (auto& e : all) {
      const float ms = time_cfg(e.second);
      if (ms < 0.f) { rc = POLSAR_E_HIP; goto done; }
      e.first = std::min(e.first, ms);
    }
  for (const auto& e : all)
    if (e.first < win_ms) { win_ms = e.first; win = e.second; }
  {
    std::lock_guard<std::mutex> g(g_mu);
    g_cfg[std::make_tuple(polsar_inv_det_launch_op(n), dtype, method, precision)] = win;
  }
  if (best) *best = win;
  if (best_ms) *best_ms = win_ms;
done:
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

int polsar_stream_copy(int dtype, int64_t n, const void* src, int64_t src_pitch, int n_in, void* dst,
                       int64_t dst_pitch, int n_out, void* stream) {
  if (dtype != POLSAR_F32 && dtype != POLSAR_F64) return POLSAR_E_ARG;
  if (n < 0) return POLSAR_E_ARG;
  const size_t es = esize(dtype);
  int r = check_planes(src, src_pitch, n, es);
  if (r) return r;
  if ((r = check_planes(dst, dst_pitch, n, es))) return r;
  const bool shape_ok = (n_in == 9 && n_out == 10) || (n_in == 18 && n_out == 9) || (n_in == 18 && n_out == 19) ||
                        (n_in == 24 && n_out == 10) || (n_in == 27 && n_out == 28) || (n_in == 1 && n_out == 1);
  if (!shape_ok) return POLSAR_E_UNSUPPORTED;
  if (!vec_ok(src, src_pitch, es) || !vec_ok(dst, dst_pitch, es)) return POLSAR_E_ALIGN;
  if (n > 0 && overlap(span(src, n_in, src_pitch, n, es), span(dst, n_out, dst_pitch, n, es))) return POLSAR_E_ALIAS;
  if (n == 0) return POLSAR_OK;
  hipStream_t s = (hipStream_t)stream;
  // launch shape: op 4 of the table (block, access width, non-temporal,
  // resident-block cap); one vector per lane, one tile per block
  const polsar_launch c = get_cfg(4, dtype, 0, 0);
  const int VW = (int)(c.vector_bytes / es);
  const int64_t nvec = n / VW;
  const int64_t grid = std::max<int64_t>(1, (nvec + c.block - 1) / c.block);
  const size_t lds = launch_lds(c, 0);
#define POLSAR_COPY(T, V, NI, NO)                                                                              \
  do {                                                                                                        \
    if (c.nontemporal)                                                                                        \
      hipLaunchKernelGGL((k_copy<T, V, NI, NO, true>), dim3((unsigned)grid), dim3(c.block), lds, s,           \
                         (const T*)src, src_pitch, (T*)dst, dst_pitch, nvec, n);                              \
    else                                                                                                      \
      hipLaunchKernelGGL((k_copy<T, V, NI, NO, false>), dim3((unsigned)grid), dim3(c.block), lds, s,          \
                         (const T*)src, src_pitch, (T*)dst, dst_pitch, nvec, n);                              \
  } while (0)
#define POLSAR_COPY_V(T, V)                                                                                    \
  do {                                                                                                        \
    if (n_in == 9) POLSAR_COPY(T, V, 9, 10);                                                                  \
    else if (n_in == 18 && n_out == 9) POLSAR_COPY(T, V, 18, 9);                                              \
    else if (n_in == 18) POLSAR_COPY(T, V, 18, 19);                                                           \
    else if (n_in == 24) POLSAR_COPY(T, V, 24, 10);                                                           \
    else if (n_in == 27) POLSAR_COPY(T, V, 27, 28);                                                           \
    else POLSAR_COPY(T, V, 1, 1);                                                                             \
  } while (0)
  if (dtype == POLSAR_F32) {
    if (VW == 4) POLSAR_COPY_V(float, 4);
    else POLSAR_COPY_V(float, 2);
  } else {
    if (VW == 2) POLSAR_COPY_V(double, 2);
    else POLSAR_COPY_V(double, 1);
  }
#undef POLSAR_COPY_V
#undef POLSAR_COPY
  return hipGetLastError() == hipSuccess ? POLSAR_OK : POLSAR_E_HIP;
}


// ------------------------------------------------------------------ out-of-core streaming
// Host-resident images (larger than device memory, or simply on the host):
// the pixels are cut into chunks; chunk i uses device buffer set i % 2 and
// stream i % 2: one 2-D copy of its 9 input plane segments host -> device,
// the inverse kernel, and 2-D copies of the 9 inverse planes, the det and
// the status segments back.  Work on the two streams overlaps, so the copy
// of one chunk runs while the other is computed.
}  // extern "C"

struct polsar_streamer {
  int dtype, method, precision;
  int64_t chunk, pitch;  // device plane pitch (elements) of each buffer set
  void* dz[2];
  void* dout[2];  // 9 inverse planes + det plane
  uint8_t* dst[2];
  hipStream_t st[2];
};

namespace {
void streamer_release(polsar_streamer* s) {
  if (!s) return;
  for (int b = 0; b < 2; ++b) {
    if (s->st[b]) (void)hipStreamDestroy(s->st[b]);
    if (s->dz[b]) (void)hipFree(s->dz[b]);
    if (s->dout[b]) (void)hipFree(s->dout[b]);
    if (s->dst[b]) (void)hipFree(s->dst[b]);
  }
  delete s;
}
}  // namespace

extern "C" {

int polsar_streamer_create(int dtype, int method, int precision, int64_t chunk_pixels, polsar_streamer** out) {
  if (!out) return POLSAR_E_ARG;
  *out = nullptr;
  int r = check_mode(dtype, method, precision);
  if (r) return r;
  if (chunk_pixels < 1 || chunk_pixels > ((int64_t)1 << 34)) return POLSAR_E_ARG;
  polsar_streamer* s = new polsar_streamer();
  s->dtype = dtype;
  s->method = method;
  s->precision = precision;
  s->chunk = chunk_pixels;
  s->pitch = polsar_recommended_pitch(dtype, chunk_pixels);
  const size_t es = esize(dtype);
  for (int b = 0; b < 2; ++b) {
    if (hipMalloc(&s->dz[b], 9 * s->pitch * es) != hipSuccess || hipMalloc(&s->dout[b], 10 * s->pitch * es) != hipSuccess ||
        hipMalloc((void**)&s->dst[b], (size_t)chunk_pixels) != hipSuccess ||
        hipStreamCreateWithFlags(&s->st[b], hipStreamNonBlocking) != hipSuccess) {
      streamer_release(s);
      return POLSAR_E_HIP;
    }
  }
  *out = s;
  return POLSAR_OK;
}

int polsar_streamer_run(polsar_streamer* s, int64_t n, const void* z, int64_t z_pitch, void* inv, int64_t inv_pitch,
                        void* det, uint8_t* status, unsigned long long* counters) {
  if (!s) return POLSAR_E_ARG;
  if (n < 0) return POLSAR_E_ARG;
  const size_t es = esize(s->dtype);
  int r = check_planes(z, z_pitch, n, es);
  if (r) return r;
  if (inv && (r = check_planes(inv, inv_pitch, n, es))) return r;
  if (det && ((uintptr_t)det % es)) return POLSAR_E_ALIGN;
  if (!inv && !det && !status && !counters) return POLSAR_E_ARG;
  if (counters && ((uintptr_t)counters % 8)) return POLSAR_E_ALIGN;
  if (n > 0) {
    const Range rz = span(z, 9, z_pitch, n, es);
    if (inv && overlap(span(inv, 9, inv_pitch, n, es), rz)) return POLSAR_E_ALIAS;
    if (det && overlap(span(det, 1, n, n, es), rz)) return POLSAR_E_ALIAS;
  }
  const polsar_launch c = get_cfg(polsar_inv_det_launch_op(s->chunk), s->dtype, s->method, s->precision);
  const int op = op_code(s->method, s->precision);
  const size_t P = (size_t)s->pitch * es;
  hipError_t e = hipSuccess;
  for (int64_t off = 0, i = 0; off < n && e == hipSuccess; off += s->chunk, ++i) {
    const int b = (int)(i & 1);
    const int64_t m = std::min<int64_t>(s->chunk, n - off);
    hipStream_t st = s->st[b];
    const size_t w = (size_t)m * es;
    e = hipMemcpy2DAsync(s->dz[b], P, (const char*)z + off * es, (size_t)z_pitch * es, w, 9, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) break;
    InvDetArgs a{s->dz[b], s->pitch, inv ? s->dout[b] : nullptr, s->pitch,
                 det ? (char*)s->dout[b] + 9 * P : nullptr, status ? s->dst[b] : nullptr, counters, m, 0, 0};
    e = launch_inv_det(s->dtype, op, c, true, a, st);
    if (e != hipSuccess) break;
    if (inv) e = hipMemcpy2DAsync((char*)inv + off * es, (size_t)inv_pitch * es, s->dout[b], P, w, 9, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && det) e = hipMemcpyAsync((char*)det + off * es, (char*)s->dout[b] + 9 * P, w, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && status) e = hipMemcpyAsync(status + off, s->dst[b], (size_t)m, hipMemcpyDeviceToHost, st);
  }
  const hipError_t e0 = hipStreamSynchronize(s->st[0]);
  const hipError_t e1 = hipStreamSynchronize(s->st[1]);
  return (e == hipSuccess && e0 == hipSuccess && e1 == hipSuccess) ? POLSAR_OK : POLSAR_E_HIP;
}

void polsar_streamer_destroy(polsar_streamer* s) { streamer_release(s); }

}  // extern "C"
