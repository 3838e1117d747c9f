// Allocation-free variant of sem_norm for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops): the partial sums of
// the reduction live in a fixed file-scope device array instead of the
// handle's buffer.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "internal.h"
#include "kernels.h"

namespace sem {
namespace {

// Partial sums of the two-stage reduction (kRedBlocks) and its result.  One
// copy per GPU, held until the process ends.
constexpr int kScratchDoubles = kRedBlocks + 8;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};   // device address of `scratch` per device

// Device address of the scratch array on the current device (resolved once
// per device), or null when the lookup fails.
double *scratch_ptr() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_ptr[dev] = static_cast<double *>(p);
  }
  return g_ptr[dev];
}

}  // namespace

bool noalloc_prepare() { return scratch_ptr() != nullptr; }

}  // namespace sem

extern "C" sem_status sem_norm_noalloc(sem_handle h, const double *x, double *out) {
  using namespace sem;
  if (!h || !x || !out) return SEM_EINVAL;
  hipStream_t s = nullptr;
  long n = 0;
  if (!handle_top(h, &s, &n)) return SEM_EINVAL;
  double *ptr = scratch_ptr();
  if (!ptr) {
    handle_error(h, "sem_norm_noalloc: hipGetSymbolAddress failed");
    return SEM_EHIP;
  }
  // every partial that the final stage reads is written by the first stage,
  // so nothing needs clearing between calls
  launch_dot(x, x, n, ptr, ptr + kRedBlocks, s);
  double v = 0.0;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(&v, ptr + kRedBlocks, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    handle_error(h, hipGetErrorString(e));
    return SEM_EHIP;
  }
  *out = std::sqrt(v);
  return SEM_OK;
}
