// vc_noalloc.hip -- vc_pvc_device_noalloc: vc_pvc_device for callers that cannot allocate
// device memory. Its device buffers (instance table and state, worklist ring and tickets,
// per-workgroup stacks, control words) are carved, through the caller-workspace path of
// vc_host.cpp, from `scratch`: a fixed array of kScratchBytes in this library's code object,
// which each GPU the library runs on holds until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory: it is never passed to
// a kernel or a copy. noalloc_setup resolves its device address once per device (from
// vc_create, with the device current) and every use goes through that address.

#include <hip/hip_runtime.h>

#include <mutex>

#include "vc.h"
#include "vc_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mutex;
void* g_scratch[kMaxDevices] = {};  // the device address of `scratch` on each device

}  // namespace

namespace vc {

int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return VC_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (g_scratch[device]) return VC_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) {
    (void)hipGetLastError();
    return VC_ERR_DEVICE;
  }
  g_scratch[device] = ptr;
  return VC_OK;
}

}  // namespace vc

extern "C" int vc_pvc_device_noalloc(vc_ctx* ctx, const vc_graph* g, int32_t k,
                                     const vc_options* opts, int32_t* yes_out, int32_t* size_out,
                                     uint8_t* cover_dev, vc_stats* stats) {
  if (!ctx) return VC_ERR_INVALID_ARG;
  const int device = vc::context_device(ctx);
  void* ptr = nullptr;
  if (device >= 0 && device < kMaxDevices) {
    std::lock_guard<std::mutex> lock(g_mutex);
    ptr = g_scratch[device];
  }
  if (!ptr) return VC_ERR_DEVICE;  // vc_create resolves it; it cannot be missing here
  return vc::pvc_device_in(ctx, g, k, opts, ptr, kScratchBytes, yes_out, size_out, cover_dev,
                           stats);
}
