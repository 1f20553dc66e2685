// Device helpers shared by the per-call kernels and the batched kernel:
// 128-bit plane access, status bytes, counters, a fixed-order block sum and
// the op table mapping (method, precision) to the per-pixel function.
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

// Deterministic block sum of one double per lane; result valid in lane 0
// of wave 0.  Order: fixed butterfly within each wave, then waves in order.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double wsum[4];
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

}  // namespace polsar_dev
