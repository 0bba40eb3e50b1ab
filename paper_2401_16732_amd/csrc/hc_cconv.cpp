// Entry points of libhconv (include/hc.h) for the conventional convolution
// with batch encoding (section "Conventional Convolution"; HRot and eq.
// keySwitching in "Background: Homomorphic Encryption"): rotation-order slot
// encoding, switching-key generation (client side), the layer with its
// resident NTT-domain weight plaintexts, and the run: forward NTT of the
// inputs and of c1's digits, automorphism + key switching per rotation
// (k_cc_keyswitch), PMult and sum over inputs and rotations (the
// multiply-accumulate kernel of the DRot path, with plaintexts as weights),
// inverse NTT. Kernels live in hc_cconv.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <new>
#include <vector>

#include "../../include/hc.h"
#include "hc_internal.h"
#include "hc_objects.h"

using hc::fail;
using hc::hip_fail;


struct hc_cconv {
  hc_ctx *ctx = nullptr;
  hc_conv_shape shape{};
  hc::CcGeom cg{};
  uint32_t T = 0, D = 0, LD = 0;
  std::vector<uint32_t> gal;     // Galois element of each rotation
  uint32_t *d_gal = nullptr;     // [R]
  uint32_t *d_rot = nullptr;     // [R][4] (swap, d, ky, kx)
  uint32_t *d_pow3 = nullptr;    // [N/2] 3^c mod 2N
  uint32_t *d_pt = nullptr;      // NTT-domain weight plaintexts, g_out x g_in R, blocked as launch_weight_block
  hc::MacShape mac{};
  hc::ConvGeom mg{};             // the multiply-accumulate's view: c_out = g_out, G = G_w = g_in R, T = 1
};

namespace {

#define CC_HIP(call)                                  \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

hc_status need_slots(const hc_ctx *c) {
  if (!c->batch_ok)
    return fail(HC_EUNSUPPORTED, "batch encoding needs a context whose t is a prime = 1 mod 2N below 2^30");
  return HC_OK;
}

size_t words_ws(const hc_cconv *cc, uint32_t B) {
  const hc_ctx &c = *cc->ctx;
  const size_t LN = (size_t)c.L * c.N, gi = (size_t)B * cc->cg.g_in;
  // X-hat, digits, rotated ciphertexts, Y-hat
  return gi * 2 * LN + gi * cc->LD * LN + gi * cc->cg.R * 2 * LN + (size_t)B * cc->mg.O * 2 * LN;
}

void destroy(hc_cconv *cc) {
  if (!cc) return;
  hc::DeviceGuard dg(cc->ctx->device);
  (void)hipFree(cc->d_gal);
  (void)hipFree(cc->d_rot);
  (void)hipFree(cc->d_pow3);
  (void)hipFree(cc->d_pt);
  delete cc;
}

}  // namespace

extern "C" {

hc_status hc_cconv_create(hc_ctx *c, const hc_conv_shape *s, const int8_t *filters, uint32_t decomp_bits,
                          void *stream, hc_cconv **out) {
  if (!c || !s || !filters || !out) return fail(HC_EINVAL, "null argument");
  *out = nullptr;
  hc_status st_ = need_slots(c);
  if (st_ != HC_OK) return st_;
  if (s->c_in == 0 || s->c_out == 0 || s->h == 0 || s->w == 0 || s->f % 2 == 0)
    return fail(HC_EINVAL, "empty shape or even filter width");
  if (s->stride != 1) return fail(HC_EUNSUPPORTED, "the conventional convolution here is stride 1");
  const uint64_t hw = (uint64_t)s->h * s->w;
  if (hw > c->N / 2) return fail(HC_EUNSUPPORTED, "the conventional layout needs h w <= N/2");
  if ((s->f - 1) / 2 >= s->h || (s->f - 1) / 2 >= s->w) return fail(HC_EUNSUPPORTED, "filter wider than the image");
  if (decomp_bits < 2 || decomp_bits > 16) return fail(HC_EUNSUPPORTED, "decomposition bits must be in [2, 16]");
  hc::DeviceGuard dg(c->device);
  hc_cconv *cc = new (std::nothrow) hc_cconv;
  if (!cc) return fail(HC_ENOMEM, "host allocation");
  cc->ctx = c;
  cc->shape = *s;
  hc::CcGeom &g = cc->cg;
  g.N = c->N;
  g.logn = c->logn;
  g.c_in = s->c_in;
  g.c_out = s->c_out;
  g.h = s->h;
  g.w = s->w;
  g.f = s->f;
  g.p = (s->f - 1) / 2;
  g.c_r = 1;
  while (2ull * g.c_r * hw <= c->N / 2) g.c_r *= 2;
  g.bsz = (c->N / 2) / g.c_r;
  g.c_n = 2 * g.c_r;
  g.g_in = (s->c_in + g.c_n - 1) / g.c_n;
  const uint32_t g_out = (s->c_out + g.c_n - 1) / g.c_n;
  g.R = g.c_n * s->f * s->f;
  cc->T = decomp_bits;
  cc->D = (30 + decomp_bits - 1) / decomp_bits;
  cc->LD = c->L * cc->D;
  // rotations in the order (swap, d, ky, kx), swap slowest
  const uint32_t two_n = 2 * c->N, half = c->N / 2;
  std::vector<uint32_t> rot_tab;
  for (uint32_t swap = 0; swap < 2; ++swap)
    for (uint32_t d = 0; d < g.c_r; ++d)
      for (uint32_t ky = 0; ky < s->f; ++ky)
        for (uint32_t kx = 0; kx < s->f; ++kx) {
          const int64_t off = ((int64_t)ky - g.p) * s->w + ((int64_t)kx - g.p);
          const uint32_t rho = (uint32_t)((((int64_t)d * g.bsz + off) % half + half) % half);
          uint64_t gv = 1;
          for (uint32_t i = 0; i < rho; ++i) gv = gv * 3 % two_n;
          if (swap) gv = (two_n - gv) % two_n;
          cc->gal.push_back((uint32_t)gv);
          rot_tab.insert(rot_tab.end(), {swap, d, ky, kx});
        }
  std::vector<uint32_t> pow3(half);
  for (uint32_t i = 0, v = 1; i < half; ++i, v = (uint32_t)((uint64_t)v * 3 % two_n)) pow3[i] = v;
  // the multiply-accumulate's geometry and tile (32-bit offsets must fit)
  hc::ConvGeom &mg = cc->mg;
  mg = hc::ConvGeom{};
  mg.N = c->N;
  mg.L = c->L;
  mg.c_in = g.g_in * g.R;
  mg.c_out = g_out;
  mg.f = 1;
  mg.s = 1;
  mg.cn = 1;
  mg.T = 1;
  mg.G = mg.G_w = g.g_in * g.R;
  mg.O = g_out;
  mg.w_ld = g_out;
  const hc::MacShape cands[] = {{1, 8, 1, 4, 2, 0, 0}, {1, 4, 1, 4, 2, 0, 0}, {1, 8, 2, 4, 2, 0, 0}};
  bool found = false;
  for (const auto &m : cands)
    if (!found && hc::mac_variant_ok(m) && hc::mac_offsets_fit(mg, m)) cc->mac = m, found = true;
  if (!found) {
    delete cc;
    return fail(HC_EUNSUPPORTED, "layer too large for the multiply-accumulate's 32-bit offsets");
  }
  const size_t R = g.R, n_pt = (size_t)g_out * g.g_in * R, LN = (size_t)c->L * c->N;
  hipStream_t st = (hipStream_t)stream;
  int8_t *d_f = nullptr;
  uint32_t *d_z = nullptr;
  const size_t chunk = std::min<size_t>(n_pt, 2048);
  const size_t fbytes = (size_t)s->c_out * s->c_in * s->f * s->f;
  hipError_t e = hipMalloc((void **)&cc->d_gal, R * 4);
  if (e == hipSuccess) e = hipMalloc((void **)&cc->d_rot, R * 16);
  if (e == hipSuccess) e = hipMalloc((void **)&cc->d_pow3, (size_t)half * 4);
  if (e == hipSuccess) e = hipMalloc((void **)&cc->d_pt, n_pt * LN * 4);
  if (e == hipSuccess) e = hipMalloc((void **)&d_f, fbytes);
  if (e == hipSuccess) e = hipMalloc((void **)&d_z, chunk * c->N * 4);
  if (e != hipSuccess) {
    (void)hipFree(d_f);
    (void)hipFree(d_z);
    destroy(cc);
    return fail(HC_ENOMEM, "conventional layer allocation");
  }
  e = hipMemcpy(cc->d_gal, cc->gal.data(), R * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(cc->d_rot, rot_tab.data(), R * 16, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(cc->d_pow3, pow3.data(), (size_t)half * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_f, filters, fbytes, hipMemcpyHostToDevice);
  // weight plaintexts, chunk by chunk: slots -> polynomial mod t -> centred
  // lift into every limb -> forward NTT (resident)
  const hc::Shapes sh = hc::shapes_for(*c, 1);
  for (size_t p0 = 0; p0 < n_pt && e == hipSuccess; p0 += chunk) {
    const size_t np = std::min(chunk, n_pt - p0);
    uint32_t *dst = cc->d_pt + p0 * LN;
    e = hc::launch_cc_weight_slots(d_f, cc->d_rot, cc->d_pow3, d_z, g, p0, np, (uint32_t)c->t, st);
    if (e == hipSuccess) e = hc::launch_intt_full(c->logn, sh.ie, d_z, d_z, np, c->consts_t, c->tw_t, st);
    if (e == hipSuccess) e = hc::launch_lift_plain(d_z, dst, np, c->N, 1, c->consts, st);
    if (e == hipSuccess) e = hc::launch_ntt_fwd(c->logn, sh.fe, dst, dst, np * c->L, c->consts, c->tw, st);
  }
  // the multiply-accumulate's blocked layout
  uint32_t *d_blk = nullptr;
  if (e == hipSuccess) e = hipMalloc((void **)&d_blk, n_pt * LN * 4);
  if (e == hipSuccess) e = hc::launch_weight_block(cc->d_pt, d_blk, g_out, (uint32_t)(g.g_in * R), c->L, c->N, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(cc->d_pt);
  cc->d_pt = d_blk;
  (void)hipFree(d_f);
  (void)hipFree(d_z);
  if (e != hipSuccess) {
    destroy(cc);
    return hip_fail(e, "conventional weight encoding");
  }
  *out = cc;
  return HC_OK;
}

void hc_cconv_destroy(hc_cconv *cc) { destroy(cc); }

hc_status hc_cconv_info(const hc_cconv *cc, hc_cconv_layout *out, uint32_t *galois) {
  if (!cc || !out) return fail(HC_EINVAL, "null argument");
  out->c_r = cc->cg.c_r;
  out->block = cc->cg.bsz;
  out->c_n = cc->cg.c_n;
  out->g_in = cc->cg.g_in;
  out->g_out = cc->mg.O;
  out->rotations = cc->cg.R;
  out->decomp_bits = cc->T;
  out->digits = cc->LD;
  if (galois) std::copy(cc->gal.begin(), cc->gal.end(), galois);
  return HC_OK;
}

hc_status hc_cconv_keys_size(const hc_cconv *cc, size_t *bytes) {
  if (!cc || !bytes) return fail(HC_EINVAL, "null argument");
  *bytes = (size_t)cc->cg.R * cc->LD * 2 * cc->ctx->L * cc->ctx->N * 4;
  return HC_OK;
}

hc_status hc_cconv_keygen_workspace_size(const hc_cconv *cc, size_t *bytes) {
  if (!cc || !bytes) return fail(HC_EINVAL, "null argument");
  const size_t LN = (size_t)cc->ctx->L * cc->ctx->N;
  *bytes = (2 * (size_t)cc->cg.R * cc->LD * LN + LN) * 4;
  return HC_OK;
}

hc_status hc_cconv_keygen(const hc_cconv *cc, const uint32_t *sk, const uint32_t *a, const int32_t *e_err,
                          uint32_t *keys, void *ws, size_t ws_bytes, void *stream) {
  if (!cc || !sk || !a || !e_err || !keys || !ws) return fail(HC_EINVAL, "null argument");
  size_t need = 0;
  (void)hc_cconv_keygen_workspace_size(cc, &need);
  if (ws_bytes < need) return fail(HC_EINVAL, "workspace too small");
  const hc_ctx &c = *cc->ctx;
  hc::DeviceGuard dg(c.device);
  hipStream_t st = (hipStream_t)stream;
  const size_t nk = (size_t)cc->cg.R * cc->LD, LN = (size_t)c.L * c.N;
  uint32_t *ah = (uint32_t *)ws, *eh = ah + nk * LN, *sh = eh + nk * LN;
  const hc::Shapes shp = hc::shapes_for(c, 1);
  CC_HIP(hc::launch_ntt_fwd(c.logn, shp.fe, a, ah, nk * c.L, c.consts, c.tw, st));
  CC_HIP(hc::launch_cc_lift_signed(e_err, eh, nk, c.N, c.consts, st));
  CC_HIP(hc::launch_ntt_fwd(c.logn, shp.fe, eh, eh, nk * c.L, c.consts, c.tw, st));
  CC_HIP(hc::launch_ntt_fwd(c.logn, shp.fe, sk, sh, c.L, c.consts, c.tw, st));
  CC_HIP(hc::launch_cc_keygen(ah, eh, sh, cc->d_gal, keys, cc->cg.R, cc->LD, cc->D, cc->T, c.logn, c.consts, st));
  return HC_OK;
}

hc_status hc_cconv_workspace_size(const hc_cconv *cc, uint32_t B, size_t *bytes) {
  if (!cc || !bytes) return fail(HC_EINVAL, "null argument");
  *bytes = words_ws(cc, B) * 4;
  return HC_OK;
}

hc_status hc_cconv_run(const hc_cconv *cc, const uint32_t *keys, const uint32_t *ct_in, uint32_t *ct_out, uint32_t B,
                       void *ws, size_t ws_bytes, void *stream) {
  if (!cc || (B && (!keys || !ct_in || !ct_out || !ws))) return fail(HC_EINVAL, "null argument");
  if (B == 0) return HC_OK;
  if (ws_bytes < words_ws(cc, B) * 4) return fail(HC_EINVAL, "workspace too small");
  const hc_ctx &c = *cc->ctx;
  hc::DeviceGuard dg(c.device);
  hipStream_t st = (hipStream_t)stream;
  const size_t LN = (size_t)c.L * c.N, gi = (size_t)B * cc->cg.g_in;
  uint32_t *xh = (uint32_t *)ws, *dh = xh + gi * 2 * LN, *rot = dh + gi * cc->LD * LN;
  uint32_t *yh = rot + gi * cc->cg.R * 2 * LN;
  const hc::Shapes sh = hc::shapes_for(c, B);
  CC_HIP(hc::launch_ntt_fwd(c.logn, sh.fe, ct_in, xh, gi * 2 * c.L, c.consts, c.tw, st));
  CC_HIP(hc::launch_cc_digits(ct_in, dh, gi, c.N, c.L, cc->T, cc->D, st));
  CC_HIP(hc::launch_ntt_fwd(c.logn, sh.fe, dh, dh, gi * cc->LD * c.L, c.consts, c.tw, st));
  CC_HIP(hc::launch_cc_keyswitch(xh, dh, keys, cc->d_gal, rot, gi, cc->cg.R, cc->LD, c.logn, c.consts, st));
  CC_HIP(hc::launch_mac(cc->mg, cc->mac, rot, cc->d_pt, yh, B, c.consts, c.tw, st));
  CC_HIP(hc::launch_intt_full(c.logn, sh.ie, yh, ct_out, (size_t)B * cc->mg.O * 2 * c.L, c.consts, c.tw, st));
  return HC_OK;
}

hc_status hc_rot_encode(const hc_ctx *c, const uint32_t *z, uint32_t *p, uint32_t n, void *stream) {
  if (!c || (n && (!z || !p))) return fail(HC_EINVAL, "null argument");
  hc_status s = need_slots(c);
  if (s != HC_OK || n == 0) return s;
  if (z == p) return fail(HC_EINVAL, "z and p must differ");
  hc::DeviceGuard dg(c->device);
  hipStream_t st = (hipStream_t)stream;
  const uint32_t half = c->N / 2, two_n = 2 * c->N;
  std::vector<uint32_t> pow3(half);
  for (uint32_t i = 0, v = 1; i < half; ++i, v = (uint32_t)((uint64_t)v * 3 % two_n)) pow3[i] = v;
  uint32_t *d_pow3 = nullptr;
  CC_HIP(hipMalloc((void **)&d_pow3, half * 4));
  hipError_t e = hipMemcpy(d_pow3, pow3.data(), half * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hc::launch_cc_slot_perm(z, p, d_pow3, n, c->logn, 0, st);
  if (e == hipSuccess)
    e = hc::launch_intt_full(c->logn, hc::shapes_for(*c, 1).ie, p, p, n, c->consts_t, c->tw_t, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d_pow3);
  if (e != hipSuccess) return hip_fail(e, "hc_rot_encode");
  return HC_OK;
}

hc_status hc_rot_decode(const hc_ctx *c, const uint32_t *p, uint32_t *z, uint32_t n, void *ws, size_t ws_bytes,
                        void *stream) {
  if (!c || (n && (!z || !p || !ws))) return fail(HC_EINVAL, "null argument");
  hc_status s = need_slots(c);
  if (s != HC_OK || n == 0) return s;
  if (ws_bytes < (size_t)n * c->N * 4) return fail(HC_EINVAL, "workspace too small");
  if ((uintptr_t)ws & 15u) return fail(HC_EINVAL, "ws must be 16-byte aligned");
  hc::DeviceGuard dg(c->device);
  hipStream_t st = (hipStream_t)stream;
  const uint32_t half = c->N / 2, two_n = 2 * c->N;
  std::vector<uint32_t> pow3(half);
  for (uint32_t i = 0, v = 1; i < half; ++i, v = (uint32_t)((uint64_t)v * 3 % two_n)) pow3[i] = v;
  uint32_t *d_pow3 = nullptr;
  CC_HIP(hipMalloc((void **)&d_pow3, half * 4));
  hipError_t e = hipMemcpy(d_pow3, pow3.data(), half * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hc::launch_ntt_fwd(c->logn, hc::shapes_for(*c, 1).fe, p, (uint32_t *)ws, n, c->consts_t, c->tw_t, st);
  if (e == hipSuccess) e = hc::launch_cc_slot_perm((const uint32_t *)ws, z, d_pow3, n, c->logn, 1, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d_pow3);
  if (e != hipSuccess) return hip_fail(e, "hc_rot_decode");
  return HC_OK;
}

}  // extern "C"
