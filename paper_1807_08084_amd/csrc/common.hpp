// Device helpers shared by the per-call kernels and the batched kernel:
// 128/64-bit plane access (through generic or global-space pointers), status
// bytes, counters, the op table mapping (method, precision) to the
// per-pixel function, the wave-shared FP64 queue of the FP32 compensated
// form, and a fixed-order block sum.
#pragma once

#include <hip/hip_runtime.h>

#include "pixel.hpp"

namespace polsar_dev {

// ------------------------------------------------------------------ vectors
template <class T, int V> struct VecOf { typedef T type __attribute__((ext_vector_type(V))); };

template <class T, int V, bool NT>
__device__ __forceinline__ void load_v(const T* __restrict__ p, T (&o)[V]) {
  if constexpr (V == 1) {
    o[0] = NT ? __builtin_nontemporal_load(p) : *p;
  } else {
    typedef typename VecOf<T, V>::type VT;
    const VT v = NT ? __builtin_nontemporal_load((const VT*)p) : *(const VT*)p;
#pragma unroll
    for (int l = 0; l < V; ++l) o[l] = v[l];
  }
}

template <class T, int V, bool NT>
__device__ __forceinline__ void store_v(T* __restrict__ p, const T (&o)[V]) {
  if constexpr (V == 1) {
    if (NT) __builtin_nontemporal_store(o[0], p); else *p = o[0];
  } else {
    typedef typename VecOf<T, V>::type VT;
    VT v;
#pragma unroll
    for (int l = 0; l < V; ++l) v[l] = o[l];
    if (NT) __builtin_nontemporal_store(v, (VT*)p); else *(VT*)p = v;
  }
}

// The same accesses through pointers typed in the global address space:
// plane pointers read from a descriptor in memory carry no address space, so
// the compiler would emit flat (generic) loads and stores for them; kernel
// arguments are known to be global already.
template <class T> using gptr = __attribute__((address_space(1))) T*;

template <class T> __device__ __forceinline__ gptr<T> to_global(T* p) { return (gptr<T>)p; }

template <class T, int V, bool NT>
__device__ __forceinline__ void gload_v(gptr<const T> p, T (&o)[V]) {
  if constexpr (V == 1) {
    o[0] = NT ? __builtin_nontemporal_load(p) : *p;
  } else {
    typedef typename VecOf<T, V>::type VT;
    const VT v = NT ? __builtin_nontemporal_load((gptr<const VT>)p) : *(gptr<const VT>)p;
#pragma unroll
    for (int l = 0; l < V; ++l) o[l] = v[l];
  }
}

template <class T, int V, bool NT>
__device__ __forceinline__ void gstore_v(gptr<T> p, const T (&o)[V]) {
  if constexpr (V == 1) {
    if (NT) __builtin_nontemporal_store(o[0], p); else *p = o[0];
  } else {
    typedef typename VecOf<T, V>::type VT;
    VT v;
#pragma unroll
    for (int l = 0; l < V; ++l) v[l] = o[l];
    if (NT) __builtin_nontemporal_store(v, (gptr<VT>)p); else *(gptr<VT>)p = v;
  }
}

template <int V>
__device__ __forceinline__ void gstore_status(gptr<uint8_t> p, const int (&st)[V]) {
  if constexpr (V == 4) {
    *(gptr<uint32_t>)p = (uint32_t)st[0] | ((uint32_t)st[1] << 8) | ((uint32_t)st[2] << 16) | ((uint32_t)st[3] << 24);
  } else if constexpr (V == 2) {
    *(gptr<uint16_t>)p = (uint16_t)(st[0] | (st[1] << 8));
  } else {
    *p = (uint8_t)st[0];
  }
}

template <int V>
__device__ __forceinline__ void store_status(uint8_t* p, const int (&st)[V]) {
  if constexpr (V == 4) {
    *(uint32_t*)p = (uint32_t)st[0] | ((uint32_t)st[1] << 8) | ((uint32_t)st[2] << 16) | ((uint32_t)st[3] << 24);
  } else if constexpr (V == 2) {
    *(uint16_t*)p = (uint16_t)(st[0] | (st[1] << 8));
  } else {
    *p = (uint8_t)st[0];
  }
}

// Add three per-lane counts to device counters: wave-level sum, one atomic
// per wave per counter.
__device__ __forceinline__ void flush_counters(unsigned long long* ctr, unsigned c0, unsigned c1, unsigned c2) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    c0 += __shfl_xor(c0, off, 64);
    c1 += __shfl_xor(c1, off, 64);
    c2 += __shfl_xor(c2, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (c0) atomicAdd(ctr + 0, (unsigned long long)c0);
    if (c1) atomicAdd(ctr + 1, (unsigned long long)c1);
    if (c2) atomicAdd(ctr + 2, (unsigned long long)c2);
  }
}

__device__ __forceinline__ void tally(int st, unsigned& c0, unsigned& c1, unsigned& c2) {
  c0 += st == px::ST_NOT_PD;
  c1 += st == px::ST_REROUTED;
  c2 += st == px::ST_NONFINITE;
}

// ------------------------------------------------------------------ ops
enum Op { ADJ_PLAIN = 0, ADJ_COMP = 1, ADJ_WIDE = 2, CHOL_PLAIN = 3, CHOL_COMP = 4, CHOL_WIDE = 5 };

template <class T, int OP>
__device__ __forceinline__ int run_pixel(const T (&z)[9], T (&x)[9], T& det) {
  if constexpr (OP == ADJ_PLAIN) return px::adjugate_plain(z, x, det);
  else if constexpr (OP == ADJ_COMP) return px::adjugate_comp(z, x, det);
  else if constexpr (OP == ADJ_WIDE) return px::adjugate_wide(z, x, det);
  else if constexpr (OP == CHOL_PLAIN) return px::cholesky_plain(z, x, det);
  else if constexpr (OP == CHOL_COMP) return px::cholesky_fallback(z, x, det);
  else return px::cholesky_wide(z, x, det);
}

// ------------------------------------------------------------------ FP32 compensated, shared FP64 queue
// Compensated FP32 for one lane's U*V pixels (U vectors of V) with the FP64
// recomputes gathered across the wave: every pixel first takes the FP32
// step, and a pixel the step rejects is queued in the wave's LDS region
// (its 9 inputs) right after its step, so its inputs need not stay in
// registers.  Then the wave's lanes take one queued pixel each through the
// FP64 step, and the results go back through LDS to the owning lanes,
// which store whole vectors.  A wave with nothing rejected skips the
// queue.  With a fraction p of pixels rejected the FP64 step runs
// ceil(U V p) times per wave instead of up to U V times; queueing all U
// vectors of a tile together fills the last round better than queueing
// each vector on its own.  (Letting the recomputing lanes store their
// pixels directly, over placeholders the owners' vector stores wrote,
// would free the owners earlier; measured, those scattered 4-byte stores
// made the kernel slower than the LDS round trip.)
// Queue: 64*U*V entries of QUEUE_WORDS floats (9 inputs, then 9 outputs +
// det), stored word-major (word k of entry e at q[k*64*U*V + e], so that
// each word of a pixel is one LDS access at an immediate offset from the
// same address and consecutive entries fall in consecutive banks), then
// 64*U*V status bytes.  valid[u] is false for vectors past the
// end of the image; those take no step and are not queued.  load(u, in)
// fills the 9 planes of vector u.  Every lane of the wave that is active at
// the call takes part (ballots); inactive lanes neither queue nor drain.
constexpr int QUEUE_WORDS = 10;

template <int U, int V, class Load>
__device__ __forceinline__ void comp_f32_wave(const Load& load, const bool (&valid)[U], float (&out)[U][9][V],
                                              float (&dt)[U][V], int (&st)[U][V], float* q, uint8_t* qs) {
  constexpr int E = 64 * U * V;  // entries: the stride between a pixel's words
  const int lane = threadIdx.x & 63;
  const unsigned long long below = lane == 0 ? 0ull : ((1ull << lane) - 1ull);
  unsigned long long mask[U][V];
  int total = 0;  // the wave's queued pixels
#pragma unroll
  for (int u = 0; u < U; ++u) {
    // vector u is fetched here (load(u, in)), after the steps of vector
    // u-1, which keeps the registers of two vectors' inputs free while the
    // first is worked on
    float in[9][V];
    if (valid[u]) load(u, in);
#pragma unroll
    for (int l = 0; l < V; ++l) {
      bool need = false;
      st[u][l] = px::ST_OK;
      if (valid[u]) {
        float zz[9], xx[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) zz[k] = in[k][l];
        need = !px::adjugate_comp_try(zz, xx, dt[u][l]);
#pragma unroll
        for (int k = 0; k < 9; ++k) out[u][k][l] = xx[k];
      }
      mask[u][l] = __ballot(need);
      if (need) {
        const int pos = total + __popcll(mask[u][l] & below);
#pragma unroll
        for (int k = 0; k < 9; ++k) q[k * E + pos] = in[k][l];
      }
      total += __popcll(mask[u][l]);
    }
  }
  if (total == 0) return;  // uniform across the active lanes
  // the active lanes share the queue: rank among them, stride = their count
  const unsigned long long active = __ballot(1);
  const int rank = __popcll(active & below), nact = __popcll(active);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int e = rank; e < total; e += nact) {
    float zz[9], xx[9], d;
#pragma unroll
    for (int k = 0; k < 9; ++k) zz[k] = q[k * E + e];
    const int sst = px::adjugate_comp_reroute(zz, xx, d);
#pragma unroll
    for (int k = 0; k < 9; ++k) q[k * E + e] = xx[k];
    q[9 * E + e] = d;
    qs[e] = (uint8_t)sst;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  int base = 0;
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int l = 0; l < V; ++l) {
      if ((mask[u][l] >> lane) & 1ull) {
        const int pos = base + __popcll(mask[u][l] & below);
#pragma unroll
        for (int k = 0; k < 9; ++k) out[u][k][l] = q[k * E + pos];
        dt[u][l] = q[9 * E + pos];
        st[u][l] = qs[pos];
      }
      base += __popcll(mask[u][l]);
    }
}

// LDS bytes of the FP32 compensated queue for one block, `slots` pixels per lane.
inline size_t comp_queue_bytes(int block, int slots) {
  const size_t entries = (size_t)block * slots;  // 64*slots per wave, block/64 waves
  return entries * (QUEUE_WORDS * sizeof(float) + 1);
}

// Most blocks per CU of a launch that asks for status counters.  Each wave
// adds its tallies to the caller's three counters with one atomic per
// counter when it ends; with one tile per block that puts hundreds of
// thousands of atomics on the same three addresses (6.1 ms against 0.88 ms
// for the FP32 compensated inverse of an 8192x8192 image), so such launches
// stride a grid of at most this many blocks per CU over the tiles instead.
constexpr int COUNTER_GRID_PER_CU = 16;

// Lanes of the fixed-order reduction kernels (the per-call Wishart loss and
// the batch's per-image losses use the same, so their orders agree).
constexpr int REDUCE_BLOCK = 1024;

// Deterministic block sum of one double per lane (blocks of up to 1024
// lanes); result valid in lane 0 of wave 0.  Order: fixed butterfly within
// each wave, then waves in order.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double wsum[16];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) wsum[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += wsum[i];
  }
  __syncthreads();
  return s;
}

// Tile of block b in a grid of g blocks.  The hardware deals the blocks of
// a grid out to MI355X's eight XCDs in turn (block b to XCD b mod 8), and
// each XCD has its own L2; this mapping gives the blocks of one XCD a
// contiguous run of tiles, so that neighbouring tiles, which read the same
// halo, meet in the same L2.  A bijection on [0, g): XCD k takes
// g / 8 + (k < g mod 8) tiles, starting where XCD k - 1's run ends.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned g) {
  constexpr unsigned NX = 8;
  const unsigned q = g / NX, r = g % NX, k = b % NX, j = b / NX;
  return k * q + (k < r ? k : r) + j;
}

// Fixed-order sum of p[0 .. count) by one block: lane t adds p[t],
// p[t + B], p[t + 2B], ... in ascending order (B = blockDim.x), then
// block_sum.  Loads are issued D at a time, so a lane waits for memory
// about count / (B D) times instead of count / B; the order of the
// additions, hence the result, is the same as one load at a time.
// Result valid in lane 0 of wave 0.
__device__ __forceinline__ double strided_sum(const double* __restrict__ p, int64_t count) {
  constexpr int D = 16;
  const int64_t B = blockDim.x;
  double s = 0.0;
  int64_t i = threadIdx.x;
  for (; i + (D - 1) * B < count; i += D * B) {
    double v[D];
#pragma unroll
    for (int j = 0; j < D; ++j) v[j] = p[i + j * B];
#pragma unroll
    for (int j = 0; j < D; ++j) s += v[j];
  }
  for (; i < count; i += B) s += p[i];
  return block_sum(s);
}

}  // namespace polsar_dev
