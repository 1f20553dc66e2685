// Allocation-free variant of polsar_wishart_loglik: the forward pass keeps
// its per-tile partial sums in a fixed device array of this library instead
// of a caller workspace, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).  The kernels are those of
// polsar_wishart_loglik, at the same launch, so the results are the same
// bits.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/polsar.h"

// Shared with polsar.hip: validation and launch of the Wishart call with
// the per-tile partial sums at `ws` (ws_words 8-byte words).
int polsar_wishart_call(int dtype, int pass, int64_t n, const void* sigma, int64_t s_pitch, const void* z,
                        int64_t z_pitch, double n_looks, double* loss, void* ell, const double* grad_loss, void* grad,
                        int64_t g_pitch, double* ws, int64_t ws_words, int (*fixed_ws)(double**),
                        unsigned long long* counters, void* stream);

namespace {
// 8 MiB per GPU: up to 2^20 tile partials.
constexpr int64_t SCRATCH_WORDS = int64_t(1) << 20;
}  // namespace

// One copy per GPU, zero when the code object loads, held until the process
// ends.  Host code never passes this name to a kernel or a copy (on the host
// it is a stand-in, not a device address): it uses the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[SCRATCH_WORDS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_ptr[MAX_DEVICES] = {};

// Device address of the current device's scratch, looked up once per device
// (with that device current) on its first call.
int scratch_ptr(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return POLSAR_E_HIP;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return POLSAR_E_HIP;
    g_ptr[dev] = (double*)p;
  }
  *out = g_ptr[dev];
  return POLSAR_OK;
}
}  // namespace

extern "C" {

int polsar_wishart_loglik_noalloc(int dtype, int pass, int64_t n, const void* sigma, int64_t s_pitch,
                                  const void* z, int64_t z_pitch, double n_looks, double* loss, void* ell,
                                  const double* grad_loss, void* grad, int64_t g_pitch,
                                  unsigned long long* counters, void* stream) {
  return polsar_wishart_call(dtype, pass, n, sigma, s_pitch, z, z_pitch, n_looks, loss, ell, grad_loss, grad,
                             g_pitch, nullptr, SCRATCH_WORDS, scratch_ptr, counters, stream);
}

}  // extern "C"
