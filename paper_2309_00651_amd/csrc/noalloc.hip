// hfx_apply_exchange_noalloc: K psi and E_x (as hfx_apply_exchange) with the
// workspace in a device array of this file instead of a caller's buffer, for
// callers that cannot allocate device memory (code under graph capture,
// serving loops, harnesses that forbid allocation).  Nothing here or in the
// launch sequence it runs calls hipMalloc, hipFree or another allocating
// routine, and no event is created.
//
// The array is file-scope device memory: each GPU the library runs on holds
// its own copy for the life of the process.  Host code may not use its name
// as an address (that is a host-side stand-in); the device address is looked
// up once per device with hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/hfx.h"
#include "tune.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;  // 256 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_lock;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device

}  // namespace

extern "C" hfx_status hfx_apply_exchange_noalloc(hfx_plan plan, const double* psi, void* kpsi,
                                                 double* ex, void* stream) {
  if (!plan || !psi || !kpsi) {
    hfx::set_error("null plan, psi or kpsi");
    return HFX_EINVAL;
  }
  const size_t need = hfx::apply_workspace_bytes(plan);
  if (need > kScratchBytes) {
    hfx::set_error("hfx_apply_exchange_noalloc: the plan's K psi calls need " +
                   std::to_string(need) + " workspace bytes, the static scratch holds " +
                   std::to_string(kScratchBytes) + " (use smaller batches: tiles=, rows=)");
    return HFX_ENOMEM;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    hfx::set_error("no usable HIP device");
    return HFX_EDEVICE;
  }
  if (dev != hfx::plan_device(plan)) {
    hfx::set_error("call with the plan's device current");
    return HFX_EINVAL;
  }
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> g(g_lock);
    if (!g_scratch[dev]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        hfx::set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        return HFX_EDEVICE;
      }
      g_scratch[dev] = p;
    }
    ptr = g_scratch[dev];
  }
  // Nothing in the scratch needs to start at zero: every pass writes the
  // pair grids, partial sums and staged orbitals it reads later in the call.
  return hfx::apply_into(plan, psi, kpsi, ex, ptr, stream);
}
