// Library-private definitions shared by hc_host.cpp, hc_server.cpp and hc_client.cpp.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <mutex>
#include <string>

#include "../../include/hc.h"
#include "hc_internal.h"

struct hc_ctx {
  uint32_t N = 0, logn = 0, L = 0;
  uint64_t t = 0;
  uint32_t q[hc::kMaxLimbs] = {};
  uint32_t psi[hc::kMaxLimbs] = {};
  uint32_t delta[hc::kMaxLimbs] = {};
  int device = 0;
  hc::LimbConsts consts{};
  uint2 *d_tw = nullptr;  // [2][L][N]: forward then inverse
  hc::Twiddles tw{};
  hc_tuning tune{};        // 0 fields = defaults
  bool check_inputs = false;  // HC_CHECK_INPUTS=1 at creation: conv entry points validate their inputs
  unsigned long long *d_count = nullptr;  // the input check's device counter ...
  std::unique_ptr<std::mutex> count_mu{new std::mutex};  // ... used by one call at a time
  hc::DecodeConsts dec{};     // exact decryption rounding (client side)
  // batch (slot) encoding, present when t is a prime = 1 mod 2N: transforms modulo t
  bool batch_ok = false;
  hc::LimbConsts consts_t{};  // L = 1, q[0] = t
  uint2 *d_tw_t = nullptr;    // [2][N]
  hc::Twiddles tw_t{};
};

struct hc_layer {
  hc_ctx *ctx = nullptr;
  hc_conv_shape shape{};
  hc_layout lay{};
  hc::ConvGeom geom{};
  uint32_t *d_w = nullptr;  // [c_out][w_cts][L][N], NTT domain
  size_t w_elems = 0;
  int32_t *d_wt = nullptr;  // [wt_rows][c_in][f f] int32 filters (coefficient-domain conv)
  uint32_t wt_rows = 0;     // c_out rounded up to a multiple of 16, extra rows zero
  bool direct_one = false;  // the coefficient-domain conv is the faster path for one image
  // per-layer launch shapes chosen by the autotuner, one set per batch size
  // (a few sizes: e.g. the batched graph's and one image's)
  static constexpr int kTuneSlots = 4;
  struct TuneSlot {
    uint32_t B = 0;  // 0: empty
    hc_tuning t{};
  } tunes[kTuneSlots];
  int tune_last = -1;  // slot set most recently
};


namespace hc {

hc_status fail(hc_status s, const std::string &msg);
hc_status hip_fail(hipError_t e, const char *where);

// Launch shapes in effect for B images.
struct Shapes {
  uint32_t fe, ie, ipw;  // ipw: polynomials per workgroup of the masked inverse NTT
  MacShape mac;
};
Shapes shapes_for(const hc_ctx &c, uint32_t B);
// The MAC shape a tuning names (all four tile fields set); depth 0 means 2.
inline MacShape mac_of(const hc_tuning &t) {
  return MacShape{t.mac_rows, t.mac_cols, t.mac_row_groups, t.mac_col_groups, t.mac_depth ? t.mac_depth : 2u,
                  t.mac_lds, t.mac_pre};
}
// The layer's autotuned shapes when tuned for B images, else the context's.
Shapes layer_shapes(const hc_layer *ly, uint32_t B);
// The layer's tuning for B images (nullptr: none); storing one for B replaces
// an earlier one for B, else takes a free slot, else the oldest.
const hc_tuning *layer_tuning_for(const hc_layer *ly, uint32_t B);
void layer_set_tuning(hc_layer *ly, uint32_t B, const hc_tuning &t);

// Constants of the exact decryption rounding for primes q[0..L) and t.
DecodeConsts make_decode_consts(const uint32_t *q, uint32_t L, uint64_t t);

// Sum offsets of the coefficient-domain conv for the context's primes.
DirectConsts direct_consts(const hc_ctx &c);

// Device workspace of one layer's conv for B images (X-hat, plus Y-hat when masked).
size_t ws_bytes_for(const hc_layer *ly, uint32_t B, bool masked);

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// hc_conv_masked after its argument checks, on the device already current:
// the input check (when the context has it on), then forward NTT, MAC and
// masked inverse NTT with X-hat and Y-hat in ws (ws_bytes_for(ly, B, true)).
hc_status conv_masked_on(const hc_layer *ly, const uint32_t *ct_in, const uint32_t *mask, uint32_t *c0_ext,
                         uint32_t *c1_out, uint32_t B, void *ws, hipStream_t st);

// Looks up the device address of hc_conv_masked_noalloc's scratch array on
// `device` (which must be current) once; later calls return at once.
hc_status noalloc_init(int device);

// Forward NTT, MAC and masked inverse NTT of one layer for a group of images
// whose buffers are given per image (at most kMaxTab).
hc_status enqueue_conv_gather(const hc_layer *ly, uint32_t B, const uint32_t *const *ct_in,
                              const uint32_t *const *mask, uint32_t *const *c0, uint32_t *const *c1, void *ws,
                              hipStream_t st);

}  // namespace hc
