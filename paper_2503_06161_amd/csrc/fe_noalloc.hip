// Backward pass without caller-provided scratch, for callers that cannot
// allocate device memory.  Its scratch (per-Gaussian screen-space sums, the
// tiles' row offsets, the row index of each walked pair and the partial
// rows) lives in one file-scope device array per GPU; everything else is
// fe_render_backward.
#include "fe_common.h"

#include <mutex>

#pragma clang fp contract(off)

namespace {
constexpr size_t kStaticScratchBytes = FE_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
}  // namespace

// Each GPU the library runs on holds its own copy until the process ends.
// In host code this name is not a device address: the address is asked of
// the runtime once per device and kept in device_scratch[].
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex scratch_mutex;
void* device_scratch[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up once)
fe_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FE_ERR_HIP;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!device_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FE_ERR_HIP;
    device_scratch[dev] = p;
  }
  *out = device_scratch[dev];
  return FE_OK;
}
}  // namespace

extern "C" fe_status fe_render_backward_noalloc(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g,
                                                const fe_images* fwd, const void* state, size_t state_bytes,
                                                const float* d_rgb, const float* d_feat, const float* d_depth,
                                                const fe_grads* out, void* stream) {
  const fe_status v = fe_validate(cfg, cam, g ? g->n : -1);
  if (v != FE_OK) return v;
  if (fe_backward_scratch_bytes(cfg, cam, g->n) > kStaticScratchBytes) return FE_ERR_WORKSPACE_TOO_SMALL;
  void* mem = nullptr;
  const fe_status st = scratch_address(&mem);
  if (st != FE_OK) return st;
  return fe_render_backward(cfg, cam, g, fwd, state, state_bytes, d_rgb, d_feat, d_depth, out, mem,
                            kStaticScratchBytes, stream);
}
