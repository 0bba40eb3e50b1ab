// hc_conv_masked_noalloc: the masked convolution (hc_conv_masked) for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc). Its scratch - the NTT-domain
// inputs X-hat and products Y-hat of one call - lives in one file-scope device
// array of HC_NOALLOC_SCRATCH_BYTES per device, whose device address is looked
// up once per device at set-up (hc_ctx_create calls noalloc_init with the
// context's device current). The entry point itself allocates nothing.
#include <mutex>

#include "hc_objects.h"

namespace {

constexpr size_t kScratchWords = HC_NOALLOC_SCRATCH_BYTES / sizeof(uint32_t);
// Host code must not take this name as a device address: the kernels get the
// address hipGetSymbolAddress returned for the device (g_scratch below).
static __device__ __align__(256) uint32_t scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

}  // namespace

// The scratch array's address on `device`, which must be the current device.
hc_status hc::noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(HC_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return HC_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "scratch array address");
  if (!p) return fail(HC_EDEVICE, "scratch array address is null");
  g_scratch[device] = p;
  return HC_OK;
}

extern "C" hc_status hc_conv_masked_noalloc(const hc_layer *ly, const uint32_t *ct_in, const uint32_t *mask,
                                            uint32_t *c0_ext, uint32_t *c1_out, uint32_t B, void *stream) {
  if (!ly || (B && (!ct_in || !mask || !c0_ext || !c1_out))) return hc::fail(HC_EINVAL, "null argument");
  if (B == 0) return HC_OK;
  const size_t need = hc::ws_bytes_for(ly, B, true);
  if (need > HC_NOALLOC_SCRATCH_BYTES)
    return hc::fail(HC_EINVAL, "hc_conv_masked_noalloc: this layer needs " + std::to_string(need) +
                                   " bytes of scratch for " + std::to_string(B) + " images, above the fixed " +
                                   std::to_string((size_t)HC_NOALLOC_SCRATCH_BYTES) +
                                   "; use fewer images per call, or hc_conv_masked with a workspace");
  const int dev = ly->ctx->device;
  hc::DeviceGuard dg(dev);
  void *p = nullptr;
  if (dev >= 0 && dev < kMaxDevices) {
    std::lock_guard<std::mutex> lk(g_mu);
    p = g_scratch[dev];
  }
  if (!p) {  // set-up did not run or failed on this device: look the address up now
    const hc_status s = hc::noalloc_init(dev);
    if (s != HC_OK) return s;
    std::lock_guard<std::mutex> lk(g_mu);
    p = g_scratch[dev];
  }
  return hc::conv_masked_on(ly, ct_in, mask, c0_ext, c1_out, B, p, (hipStream_t)stream);
}
