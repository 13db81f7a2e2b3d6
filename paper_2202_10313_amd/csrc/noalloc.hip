// The allocation-free advance, edg_advance_to_static (include/edge_lts.h):
// edg_advance_to with the B1 / B2 / B3 face traces of the advance held in a
// file-scope device array instead of the context's own trace buffers, for
// callers that cannot allocate device memory during the time loop.
//
// The array exists once per GPU (each device holds its own copy at its own
// address) from the first call on that device until the process ends.  In
// host code its name is only a stand-in: the device address is looked up
// once per device with hipGetSymbolAddress, with that device current, and
// that address is what reaches the kernels and the fill kernel.
#include <hip/hip_runtime.h>

#include <mutex>

#include "edge_lts.h"

namespace edg {
int advance_to_traces(edg_ctx* c, double t, void* base, size_t cap);
int ctx_device(const edg_ctx* c);
int ctx_fail(edg_ctx* c, int code, const char* msg);
}  // namespace edg

namespace {

__device__ __align__(256) unsigned char scratch[EDG_STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_lock;
void* g_scratch[MAX_DEVICES] = {};   // device address of `scratch` per device (null: not looked up yet)

// the device address of this device's array (the device must be current)
hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> guard(g_lock);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

extern "C" int edg_advance_to_static(edg_ctx* c, double t) {
  if (!c) return EDG_EINVAL;
  const int dev = edg::ctx_device(c);
  if (dev < 0 || dev >= MAX_DEVICES) return edg::ctx_fail(c, EDG_EINVAL, "device ordinal beyond the static scratch table");
  if (hipSetDevice(dev) != hipSuccess) return edg::ctx_fail(c, EDG_EHIP, "hipSetDevice failed");
  void* base = nullptr;
  const hipError_t e = scratch_address(dev, &base);
  if (e != hipSuccess) {
    static thread_local char msg[160];
    snprintf(msg, sizeof msg, "hipGetSymbolAddress of the static scratch: %s", hipGetErrorString(e));
    return edg::ctx_fail(c, EDG_EHIP, msg);
  }
  return edg::advance_to_traces(c, t, base, EDG_STATIC_SCRATCH_BYTES);
}
