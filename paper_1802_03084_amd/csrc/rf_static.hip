// rf_image_static: rf_image with its scratch in a fixed device array of the
// library, for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The row pass of the dense transform hands the column pass its
// row-transformed pairs through a scratch buffer (rf_image takes it as a
// workspace argument).  Here the scratch is the file-scope array below, one
// copy per GPU, held until the process ends.  Its device address is looked up
// once per device (hipGetSymbolAddress, with that device current) and only
// that address is ever passed to kernels: in host code the array's name is a
// host-side stand-in, not a device address.  Every band row of a pair is
// written by the row pass before the column pass reads it, so the scratch
// needs no clearing between calls; calls that overlap on one GPU share the
// array and race.
#include "rf_internal.h"

#include <mutex>

namespace {

constexpr size_t kStaticScratchBytes = (size_t)64 << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array (looked up on first use).
rf_status scratch_ptr(void **out) {
  int dev = 0;
  RF_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return RF_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    RF_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return RF_EHIP;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return RF_OK;
}

}  // namespace

extern "C" {

rf_status rf_image_static_max_bytes(size_t *bytes) {
  if (!bytes) return RF_EINVAL;
  *bytes = kStaticScratchBytes;
  return RF_OK;
}

rf_status rf_image_static(const rf_plan *p, const void *d_grid, int32_t nimg, float *d_img,
                          void *stream) {
  if (!p) return RF_EINVAL;
  if (nimg < 0) return RF_ERANGE;
  if (nimg == 0) return RF_OK;
  if (!d_grid || !d_img) return RF_EINVAL;
  if (image_ws_bytes(p, nimg) > kStaticScratchBytes) return RF_EWORKSPACE;
  void *ws = nullptr;
  const rf_status st = scratch_ptr(&ws);
  if (st != RF_OK) return st;
  return launch_image_dense(p, (const float2 *)d_grid, nimg, d_img, (float2 *)ws,
                            (hipStream_t)stream);
}

}  // extern "C"
