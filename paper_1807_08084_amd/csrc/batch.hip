// Batched launch over many images of uneven sizes.
//
// The images' pixels are cut into tiles of `block` vectors (one vector per
// lane, V pixels per vector on the 128-bit path), numbered consecutively
// image after image.  The grid has one block per tile, so the hardware
// dispatcher hands tiles to compute units as they free up, or is a
// persistent grid (k blocks per compute unit) that strides over the global
// tile numbers.  A block finds the image of its first tile by binary search
// over the images' first tiles and moves forward from there.  Per tile it loads Z once and, as the batch asks, writes the
// inverse/determinant of Z (FP32 compensated: rejected pixels through the
// wave's FP64 queue, as in the per-call kernel), then loads S and writes the
// Wishart term and gradient of S against the same Z.  The descriptor table
// is a restrict argument (scalar loads) and the plane pointers read from it
// are typed global, so the accesses are global rather than flat ones.  Wishart partial sums are kept per tile and reduced per
// image in a fixed order by a second kernel, so the losses do not depend
// on the grid.  Both launches are captured in one HIP graph at creation;
// running the batch is one graph launch.
//
// The per-pixel functions are those of the per-call kernels, so every
// per-pixel output is bitwise equal to a per-image call; the per-image loss
// equals the per-call Wishart loss bitwise when both cut tiles alike (same
// block size and access width, unroll 1), and to rounding otherwise.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/polsar.h"
#include "common.hpp"

size_t polsar_launch_lds_bytes(const polsar_launch& c, size_t need);

namespace {
using namespace polsar_dev;

struct ImgDesc {
  const void* z;
  void* inv;
  void* det;
  uint8_t* status;
  const void* sigma;
  void* grad;
  void* ell;
  double* loss;
  int64_t n, zp, ip, sp, gp;
  double n_looks;
  int64_t tile0;   // first global tile of this image
  int64_t ntiles;  // tiles of this image
  int64_t nvec;    // full vectors on this image's path
  int vec;         // 1: 128-bit path, 0: one element per access
  int pad;
};

struct BatchArgs {
  const ImgDesc* img;
  int count;
  int64_t total_tiles;
  double* partial;  // one per global tile
  const double* grad_loss;
  unsigned long long* counters;
  int do_inv, do_fwd, do_bwd;
};

// This lane's vector of local tile lt of image d (the cut of the per-call
// kernels at unroll 1), plus the image's tail pixels in its last tile.
// Returns the lane's sum of Wishart terms.
template <class T, int OP, int V, bool NT>
__device__ __forceinline__ double batch_tile(const BatchArgs& a, const ImgDesc& d, int64_t lt, T gscale,
                                             unsigned& c0, unsigned& c1, unsigned& c2) {
  // descriptor plane pointers, typed global (see gptr)
  const gptr<const T> Z = to_global((const T*)d.z);
  const gptr<const T> S = to_global((const T*)d.sigma);
  const gptr<T> inv = to_global((T*)d.inv), det = to_global((T*)d.det);
  const gptr<T> ell = to_global((T*)d.ell), grad = to_global((T*)d.grad);
  const gptr<uint8_t> status = to_global(d.status);
  const int64_t v = lt * (int64_t)blockDim.x + threadIdx.x;
  const bool wish = a.do_fwd || a.do_bwd;
  double acc = 0.0;
  if (v < d.nvec) {
    T z[9][V];
#pragma unroll
    for (int k = 0; k < 9; ++k) gload_v<T, V, NT>(Z + k * d.zp + v * V, z[k]);
    const int64_t e = v * V;
    if (a.do_inv) {
      T out[9][V], dt[V];
      int st[V];
      if constexpr (OP == ADJ_COMP && std::is_same<T, float>::value) {
        // the FP32 step for the lane's V pixels, rejected pixels through the
        // wave's shared FP64 queue (as in the per-call kernel)
        extern __shared__ __align__(16) float polsar_dyn_lds[];
        const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
        float* q = polsar_dyn_lds + (size_t)w * 64 * V * QUEUE_WORDS;
        uint8_t* qs = (uint8_t*)(polsar_dyn_lds + (size_t)nw * 64 * V * QUEUE_WORDS) + w * 64 * V;
        const bool valid[1] = {true};
        auto load = [&](int, float (&in)[9][V]) {
#pragma unroll
          for (int k = 0; k < 9; ++k)
#pragma unroll
            for (int l = 0; l < V; ++l) in[k][l] = z[k][l];
        };
        float o1[1][9][V], d1[1][V];
        int s1[1][V];
        comp_f32_wave<1, V>(load, valid, o1, d1, s1, q, qs);
#pragma unroll
        for (int l = 0; l < V; ++l) {
#pragma unroll
          for (int k = 0; k < 9; ++k) out[k][l] = o1[0][k][l];
          dt[l] = d1[0][l];
          st[l] = s1[0][l];
          tally(st[l], c0, c1, c2);
        }
      } else {
#pragma unroll
        for (int l = 0; l < V; ++l) {
          T zz[9], xx[9];
#pragma unroll
          for (int k = 0; k < 9; ++k) zz[k] = z[k][l];
          st[l] = run_pixel<T, OP>(zz, xx, dt[l]);
#pragma unroll
          for (int k = 0; k < 9; ++k) out[k][l] = xx[k];
          tally(st[l], c0, c1, c2);
        }
      }
      if (inv)
#pragma unroll
        for (int k = 0; k < 9; ++k) gstore_v<T, V, NT>(inv + k * d.ip + e, out[k]);
      if (det) gstore_v<T, V, NT>(det + e, dt);
      if (status) gstore_status<V>(status + e, st);
    }
    if (wish) {
      // S is loaded after the inverse is stored, which keeps the registers
      // of S free while the inverse is worked on
      T s[9][V];
#pragma unroll
      for (int k = 0; k < 9; ++k) gload_v<T, V, NT>(S + k * d.sp + v * V, s[k]);
      T ellv[V], g[9][V];
#pragma unroll
      for (int l = 0; l < V; ++l) {
        T ss[9], zz[9], gg[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) { ss[k] = s[k][l]; zz[k] = z[k][l]; }
        px::wishart_pixel<T>(ss, zz, (T)d.n_looks, a.do_fwd, ellv[l], a.do_bwd, gg, gscale);
        if (a.do_fwd) acc += (double)ellv[l];
        if (a.do_bwd)
#pragma unroll
          for (int k = 0; k < 9; ++k) g[k][l] = gg[k];
      }
      if (a.do_fwd && ell) gstore_v<T, V, NT>(ell + e, ellv);
      if (a.do_bwd)
#pragma unroll
        for (int k = 0; k < 9; ++k) gstore_v<T, V, NT>(grad + k * d.gp + e, g[k]);
    }
  }
  if (V > 1 && lt == d.ntiles - 1) {
    const int64_t i = d.nvec * V + threadIdx.x;
    if (i < d.n) {
      T zz[9], ss[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) zz[k] = Z[k * d.zp + i];
      if (a.do_inv) {
        T xx[9], dt;
        const int st = run_pixel<T, OP>(zz, xx, dt);
        tally(st, c0, c1, c2);
        if (inv)
#pragma unroll
          for (int k = 0; k < 9; ++k) inv[k * d.ip + i] = xx[k];
        if (det) det[i] = dt;
        if (status) status[i] = (uint8_t)st;
      }
      if (wish) {
        T gg[9], el;
#pragma unroll
        for (int k = 0; k < 9; ++k) ss[k] = S[k * d.sp + i];
        px::wishart_pixel<T>(ss, zz, (T)d.n_looks, a.do_fwd, el, a.do_bwd, gg, gscale);
        if (a.do_fwd) {
          acc += (double)el;
          if (ell) ell[i] = el;
        }
        if (a.do_bwd)
#pragma unroll
          for (int k = 0; k < 9; ++k) grad[k * d.gp + i] = gg[k];
      }
    }
  }
  return acc;
}

template <class T, int OP, bool NT, int VW>
__global__ __launch_bounds__(256) void k_batch(BatchArgs a, const ImgDesc* __restrict__ img) {
  const T gscale = a.do_bwd ? (a.grad_loss ? (T)*a.grad_loss : T(1)) : T(1);
  unsigned c0 = 0, c1 = 0, c2 = 0;
  // image owning the block's first tile: last i with img[i].tile0 <= t, by
  // binary search; later tiles only move forward, by a short linear scan
  // (a dependent chain of descriptor loads per tile would stall the block)
  int cur = 0;
  {
    const int64_t t = blockIdx.x;
    int hi = a.count - 1;
    while (cur < hi) {
      const int mid = (cur + hi + 1) >> 1;
      if (img[mid].tile0 <= t) cur = mid; else hi = mid - 1;
    }
  }
  for (int64_t t = blockIdx.x; t < a.total_tiles; t += gridDim.x) {
    while (cur + 1 < a.count && img[cur + 1].tile0 <= t) ++cur;
    const ImgDesc& d = img[cur];
    const int64_t lt = t - d.tile0;
    const double acc = d.vec ? batch_tile<T, OP, VW, NT>(a, d, lt, gscale, c0, c1, c2)
                             : batch_tile<T, OP, 1, NT>(a, d, lt, gscale, c0, c1, c2);
    if (a.do_fwd) {
      const double bs = block_sum(acc);
      if (threadIdx.x == 0) a.partial[t] = bs;
    }
  }
  if (a.counters) flush_counters(a.counters, c0, c1, c2);
}

// One block per image: fixed-order sum of its tiles' partials into loss.
__global__ __launch_bounds__(REDUCE_BLOCK) void k_batch_reduce(const ImgDesc* __restrict__ img,
                                                                const double* __restrict__ partial) {
  const ImgDesc& d = img[blockIdx.x];
  const double s = strided_sum(partial + d.tile0, d.ntiles);
  if (threadIdx.x == 0 && d.loss) *d.loss = s;
}

int device_cus_b() {
  int dev = 0, cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) return 256;
  return cu;
}

}  // namespace

struct polsar_batch {
  int dtype, op, count;
  unsigned ops;
  int block, grid;
  int nt, half;  // half: 8-byte plane accesses instead of 16
  size_t lds;    // dynamic LDS per block (caps resident blocks)
  int64_t total_tiles;
  ImgDesc* d_img;
  double* d_partial;
  BatchArgs args;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

namespace {

hipError_t enqueue(const polsar_batch* b, hipStream_t s) {
  const int op = b->op;
#define POLSAR_BATCH(T, OPV)                                                                                   \
  do {                                                                                                        \
    constexpr int VW = 16 / sizeof(T);                                                                        \
    const dim3 g(b->grid), t(b->block);                                                                        \
    const size_t lds = b->lds;                                                                                 \
    if (b->half) {                                                                                            \
      if (b->nt) hipLaunchKernelGGL((k_batch<T, OPV, true, VW / 2>), g, t, lds, s, b->args, b->d_img);                  \
      else hipLaunchKernelGGL((k_batch<T, OPV, false, VW / 2>), g, t, lds, s, b->args, b->d_img);                       \
    } else {                                                                                                  \
      if (b->nt) hipLaunchKernelGGL((k_batch<T, OPV, true, VW>), g, t, lds, s, b->args, b->d_img);                      \
      else hipLaunchKernelGGL((k_batch<T, OPV, false, VW>), g, t, lds, s, b->args, b->d_img);                           \
    }                                                                                                         \
  } while (0)
  if (b->dtype == POLSAR_F32) {
    switch (op) {
      case ADJ_PLAIN: POLSAR_BATCH(float, ADJ_PLAIN); break;
      case ADJ_COMP: POLSAR_BATCH(float, ADJ_COMP); break;
      case ADJ_WIDE: POLSAR_BATCH(float, ADJ_WIDE); break;
      case CHOL_PLAIN: POLSAR_BATCH(float, CHOL_PLAIN); break;
      case CHOL_COMP: POLSAR_BATCH(float, CHOL_COMP); break;
      default: POLSAR_BATCH(float, CHOL_WIDE); break;
    }
  } else {
    switch (op) {
      case ADJ_PLAIN: POLSAR_BATCH(double, ADJ_PLAIN); break;
      case ADJ_COMP: POLSAR_BATCH(double, ADJ_COMP); break;
      default: POLSAR_BATCH(double, CHOL_PLAIN); break;
    }
  }
#undef POLSAR_BATCH
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (b->ops & POLSAR_OP_WISHART_FWD) {
    hipLaunchKernelGGL(k_batch_reduce, dim3(b->count), dim3(REDUCE_BLOCK), 0, s, (const ImgDesc*)b->d_img,
                       (const double*)b->d_partial);
    e = hipGetLastError();
  }
  return e;
}

void release(polsar_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_img) (void)hipFree(b->d_img);
  if (b->d_partial) (void)hipFree(b->d_partial);
  delete b;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Byte range [lo, hi) of some planes of one image.
struct Span {
  uintptr_t lo, hi;
  bool out;
};

// True when no output span overlaps another span (input or output).  Sorted
// by start, a span overlaps an earlier one of some kind exactly when it
// starts before the furthest end among the earlier spans of that kind.
bool disjoint_outputs(std::vector<Span>& v) {
  std::sort(v.begin(), v.end(), [](const Span& a, const Span& b) { return a.lo < b.lo; });
  uintptr_t end_in = 0, end_out = 0;
  for (const Span& x : v) {
    if (x.hi <= x.lo) continue;
    if (x.lo < end_out) return false;            // meets an earlier output
    if (x.out && x.lo < end_in) return false;    // an output meets an earlier input
    if (x.out) end_out = std::max(end_out, x.hi);
    else end_in = std::max(end_in, x.hi);
  }
  return true;
}

}  // namespace

extern "C" {

int polsar_batch_create(const polsar_image* imgs, int count, int dtype, int method, int precision, unsigned ops,
                        const double* grad_loss, unsigned long long* counters, int grid_per_cu,
                        polsar_batch** out) {
  if (!out) return POLSAR_E_ARG;
  *out = nullptr;
  if (!imgs || count <= 0 || count > (1 << 20)) return POLSAR_E_ARG;
  if (dtype != POLSAR_F32 && dtype != POLSAR_F64) return POLSAR_E_ARG;
  if (method != POLSAR_ADJUGATE && method != POLSAR_CHOLESKY) return POLSAR_E_ARG;
  if (precision != POLSAR_PLAIN && precision != POLSAR_COMPENSATED && precision != POLSAR_WIDE) return POLSAR_E_ARG;
  if (ops == 0 || (ops & ~7u)) return POLSAR_E_ARG;
  if (dtype == POLSAR_F64 && precision == POLSAR_WIDE) return POLSAR_E_UNSUPPORTED;
  if (dtype == POLSAR_F64 && method == POLSAR_CHOLESKY && precision != POLSAR_PLAIN) return POLSAR_E_UNSUPPORTED;
  if (grid_per_cu < 0 || grid_per_cu > 64) return POLSAR_E_ARG;
  if (grad_loss && !aligned(grad_loss, 8)) return POLSAR_E_ALIGN;
  if (counters && !aligned(counters, 8)) return POLSAR_E_ALIGN;
  const size_t es = dtype == POLSAR_F64 ? 8 : 4;
  // Launch shape: the batch entry of the launch table (op 3: block, blocks
  // per compute unit, access width, non-temporal); a tile is one vector per
  // lane of one block.
  polsar_launch use;
  polsar_get_launch(3, dtype, method, precision, &use);
  const int block = use.block;
  const bool half = use.vector_bytes == 8;
  const int VW = (int)((half ? 8 : 16) / es);
  std::vector<ImgDesc> h(count);
  std::vector<Span> spans;
  spans.reserve((size_t)count * 7);
  int64_t tiles = 0;
  for (int i = 0; i < count; ++i) {
    const polsar_image& m = imgs[i];
    if (m.n <= 0) return POLSAR_E_ARG;
    auto planes_ok = [&](const void* p, int64_t pitch) {
      return p && pitch >= m.n && aligned(p, es);
    };
    if (!planes_ok(m.z, m.z_pitch)) return POLSAR_E_ARG;
    bool vec = aligned(m.z, 16) && (m.z_pitch * (int64_t)es) % 16 == 0;
    if (ops & POLSAR_OP_INV_DET) {
      if (!m.inv && !m.det && !m.status) return POLSAR_E_ARG;
      if (m.inv && !planes_ok(m.inv, m.inv_pitch)) return POLSAR_E_ARG;
      if (m.det && !aligned(m.det, es)) return POLSAR_E_ALIGN;
      if (m.inv) vec = vec && aligned(m.inv, 16) && (m.inv_pitch * (int64_t)es) % 16 == 0;
      if (m.det) vec = vec && aligned(m.det, 16);
      if (m.status) vec = vec && aligned(m.status, VW);
    }
    if (ops & (POLSAR_OP_WISHART_FWD | POLSAR_OP_WISHART_BWD)) {
      if (!planes_ok(m.sigma, m.s_pitch) || !(m.n_looks > 0.0)) return POLSAR_E_ARG;
      vec = vec && aligned(m.sigma, 16) && (m.s_pitch * (int64_t)es) % 16 == 0;
    }
    if (ops & POLSAR_OP_WISHART_FWD) {
      if (!m.loss || !aligned(m.loss, 8)) return POLSAR_E_ARG;
      if (m.ell) vec = vec && aligned(m.ell, 16);
    }
    if (ops & POLSAR_OP_WISHART_BWD) {
      if (!planes_ok(m.grad, m.g_pitch)) return POLSAR_E_ARG;
      vec = vec && aligned(m.grad, 16) && (m.g_pitch * (int64_t)es) % 16 == 0;
    }
    {  // this image's byte ranges, checked against every image's below
      auto add = [&](const void* p, int planes, int64_t pitch, size_t e, bool is_out) {
        if (!p) return;
        const uintptr_t lo = (uintptr_t)p;
        spans.push_back(Span{lo, lo + (uintptr_t)(((planes - 1) * pitch + m.n) * (int64_t)e), is_out});
      };
      const bool wish = ops & (POLSAR_OP_WISHART_FWD | POLSAR_OP_WISHART_BWD);
      const bool inv_op = ops & POLSAR_OP_INV_DET;
      add(m.z, 9, m.z_pitch, es, false);
      if (wish) add(m.sigma, 9, m.s_pitch, es, false);
      if (inv_op) {
        add(m.inv, 9, m.inv_pitch, es, true);
        add(m.det, 1, m.n, es, true);
        add(m.status, 1, m.n, 1, true);
      }
      if (ops & POLSAR_OP_WISHART_BWD) add(m.grad, 9, m.g_pitch, es, true);
      if (ops & POLSAR_OP_WISHART_FWD) {
        add(m.ell, 1, m.n, es, true);
        if (m.loss) spans.push_back(Span{(uintptr_t)m.loss, (uintptr_t)m.loss + sizeof(double), true});
      }
    }
    ImgDesc& d = h[i];
    d.z = m.z;
    d.inv = (ops & POLSAR_OP_INV_DET) ? m.inv : nullptr;
    d.det = (ops & POLSAR_OP_INV_DET) ? m.det : nullptr;
    d.status = (ops & POLSAR_OP_INV_DET) ? m.status : nullptr;
    d.sigma = m.sigma;
    d.grad = m.grad;
    d.ell = (ops & POLSAR_OP_WISHART_FWD) ? m.ell : nullptr;
    d.loss = m.loss;
    d.n = m.n;
    d.zp = m.z_pitch;
    d.ip = m.inv_pitch;
    d.sp = m.s_pitch;
    d.gp = m.g_pitch;
    d.n_looks = m.n_looks;
    d.vec = vec ? 1 : 0;
    d.pad = 0;
    d.nvec = m.n / (vec ? VW : 1);  // VW: the batch's vector width (set above)
    d.ntiles = std::max<int64_t>(1, (d.nvec + block - 1) / block);
    d.tile0 = tiles;
    tiles += d.ntiles;
  }
  // One grid runs every image at once, so no output may overlap any input or
  // any other output of any image (inputs may be shared).
  if (!disjoint_outputs(spans)) return POLSAR_E_ALIAS;
  polsar_batch* b = new polsar_batch();
  b->dtype = dtype;
  b->count = count;
  b->ops = ops;
  b->op = method == POLSAR_ADJUGATE ? (precision == POLSAR_PLAIN ? ADJ_PLAIN : precision == POLSAR_COMPENSATED ? ADJ_COMP : ADJ_WIDE)
                                    : (precision == POLSAR_PLAIN ? CHOL_PLAIN : precision == POLSAR_COMPENSATED ? CHOL_COMP : CHOL_WIDE);
  b->block = block;
  b->nt = use.nontemporal;
  b->half = half ? 1 : 0;
  // the FP32 compensated inverse queues rejected pixels in LDS: 64*VW
  // entries per wave (the one-element path uses the front of that)
  const bool queued = b->op == ADJ_COMP && dtype == POLSAR_F32 && (ops & POLSAR_OP_INV_DET);
  b->lds = polsar_launch_lds_bytes(use, queued ? comp_queue_bytes(block, VW) : 0);
  b->total_tiles = tiles;
  // a persistent grid of gpc blocks per compute unit, or (gpc 0) one block
  // per tile, the hardware's dispatcher doing the balancing; with counters
  // at most COUNTER_GRID_PER_CU blocks per CU (one set of atomics per wave)
  int gpc = grid_per_cu > 0 ? grid_per_cu : use.grid_per_cu;
  if (counters && (gpc == 0 || gpc > COUNTER_GRID_PER_CU)) gpc = COUNTER_GRID_PER_CU;
  b->grid = (int)std::min<int64_t>(tiles, gpc > 0 ? (int64_t)gpc * device_cus_b() : (int64_t)INT32_MAX);
  if (hipMalloc((void**)&b->d_img, sizeof(ImgDesc) * count) != hipSuccess) { release(b); return POLSAR_E_HIP; }
  if (hipMalloc((void**)&b->d_partial, sizeof(double) * tiles) != hipSuccess) { release(b); return POLSAR_E_HIP; }
  if (hipMemcpy(b->d_img, h.data(), sizeof(ImgDesc) * count, hipMemcpyHostToDevice) != hipSuccess) {
    release(b);
    return POLSAR_E_HIP;
  }
  b->args = BatchArgs{b->d_img, count, tiles, b->d_partial, grad_loss, counters,
                      (ops & POLSAR_OP_INV_DET) ? 1 : 0, (ops & POLSAR_OP_WISHART_FWD) ? 1 : 0,
                      (ops & POLSAR_OP_WISHART_BWD) ? 1 : 0};
  // capture the kernels once
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) { release(b); return POLSAR_E_HIP; }
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t e1 = enqueue(b, cs);
    e = hipStreamEndCapture(cs, &b->graph);
    if (e == hipSuccess) e = e1;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) { release(b); return POLSAR_E_HIP; }
  *out = b;
  return POLSAR_OK;
}

int polsar_batch_run(polsar_batch* b, void* stream) {
  if (!b || !b->exec) return POLSAR_E_ARG;
  return hipGraphLaunch(b->exec, (hipStream_t)stream) == hipSuccess ? POLSAR_OK : POLSAR_E_HIP;
}

int polsar_batch_run_eager(polsar_batch* b, void* stream) {
  if (!b) return POLSAR_E_ARG;
  return enqueue(b, (hipStream_t)stream) == hipSuccess ? POLSAR_OK : POLSAR_E_HIP;
}

int64_t polsar_batch_tiles(const polsar_batch* b) { return b ? b->total_tiles : -1; }

void polsar_batch_destroy(polsar_batch* b) { release(b); }

}  // extern "C"
