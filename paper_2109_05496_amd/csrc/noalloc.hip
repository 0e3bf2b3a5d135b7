// ctv_denoise_noalloc: ctv_denoise without a caller-supplied workspace, for
// callers that cannot allocate device memory (code under HIP-graph capture,
// tight serving loops). The workspace is one file-scope device array per GPU,
// of fixed size; the call allocates nothing and runs exactly the kernels of
// ctv_denoise on it, so results are bitwise those of ctv_denoise.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "ctv.h"
#include "ctv_host.hpp"

namespace ctv {

static_assert(CTV_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size must keep 256-byte alignment");

// Every GPU the library runs on holds its own copy until the process ends.
// Host code never uses this name as an address: it is a host-side stand-in.
// The device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[CTV_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// Device address of the current device's scratch array (resolved on the first
// call per device, with that device current).
static ctv_status scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(CTV_ERR_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(CTV_ERR_HIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CTV_OK;
}

}  // namespace ctv

using namespace ctv;

extern "C" ctv_status ctv_denoise_noalloc(const ctv_params* p, int32_t batch, int32_t m, int32_t n, const float* b,
                                          const float* lambda_host, const uint8_t* support, float* x, double* gap,
                                          ctv_stream_t stream) {
  // argument checks ahead of any HIP call (ctv_denoise repeats them)
  size_t need = 0;
  ctv_status st = ctv_workspace_size(p, batch, m, n, 0, &need, nullptr);
  if (st) return st;
  if (!b || !x || !lambda_host) return fail(CTV_ERR_INVALID_ARG, "b, x and lambda_host must be non-NULL");
  if (b == x) return fail(CTV_ERR_INVALID_ARG, "x must not alias b");
  for (int i = 0; i < batch; ++i) {
    st = validate_lambda(lambda_host[i]);
    if (st) return st;
  }
  if (need > (size_t)CTV_NOALLOC_SCRATCH_BYTES)
    return fail(CTV_ERR_WORKSPACE, "ctv_denoise_noalloc: the problem needs " + std::to_string(need) +
                                       " bytes of workspace, more than the fixed " +
                                       std::to_string((size_t)CTV_NOALLOC_SCRATCH_BYTES) +
                                       " (use ctv_denoise with a workspace)");
  void* ws = nullptr;
  st = scratch_of_current_device(&ws);
  if (st) return st;
  return ctv_denoise(p, batch, m, n, b, lambda_host, support, x, gap, nullptr, 0, nullptr, 0, nullptr, ws,
                     (size_t)CTV_NOALLOC_SCRATCH_BYTES, stream);
}
