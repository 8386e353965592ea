// Screening entry point that allocates nothing: the sweep's panels live in a
// fixed device array of this library instead of a caller workspace, for
// callers that cannot allocate device memory.
#include <cstdio>
#include <mutex>

#include "gw_internal.hpp"

namespace gw {
namespace {

// One copy per GPU, resident until the process ends.  In host code the name
// only identifies the symbol; its device address comes from
// hipGetSymbolAddress (scratch_on_current_device).
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device
// with that device current.
int scratch_on_current_device(void** out) {
  int dev = -1;
  GW_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(GW_ERR_UNSUPPORTED, "gw_screen_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(GW_ERR_HIP, "gw_screen_noalloc: hipGetSymbolAddress returned no address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GW_OK;
}

}  // namespace
}  // namespace gw

using namespace gw;

extern "C" {

size_t gw_screen_noalloc_max_bytes(void) { return kScratchBytes; }

int gw_screen_noalloc(void* stream, int N, int n_omega, const double* P, const double* v, double* W, int* info) {
  if (N < 1 || n_omega < 1) return fail(GW_ERR_INVALID_ARG, "gw_screen_noalloc: N and n_omega must be >= 1");
  if (!P || !v || !W || !info) return fail(GW_ERR_INVALID_ARG, "gw_screen_noalloc: null pointer among P, v, W, info");
  if (P == W) return fail(GW_ERR_INVALID_ARG, "gw_screen_noalloc: W may not alias P");
  if ((long long)N * N > (1LL << 31)) return fail(GW_ERR_UNSUPPORTED, "gw_screen_noalloc: N too large");
  const size_t need = screen_workspace_bytes(N, n_omega);
  if (need > kScratchBytes) {
    char buf[200];
    snprintf(buf, sizeof buf,
             "gw_screen_noalloc: N=%d with %d frequencies needs %zu bytes of scratch, the fixed array holds %zu "
             "(use gw_screen with a workspace)",
             N, n_omega, need, kScratchBytes);
    return fail(GW_ERR_WORKSPACE, buf);
  }
  void* ptr = nullptr;
  int st = scratch_on_current_device(&ptr);
  if (st != GW_OK) return st;
  return screen_run(static_cast<hipStream_t>(stream), N, n_omega, reinterpret_cast<const double2*>(P), v,
                    reinterpret_cast<double2*>(W), info, ptr);
}

}  // extern "C"
