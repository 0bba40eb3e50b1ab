// Entry points of libhconv (include/hc.h) for the steps around the
// convolution: on the client side the offline encryptions of zero, direct
// encoding with online encryption of a layer's input (Algorithm 2, section
// "Moving Data-independent Operations to Offline Phase") and BFV decryption
// (eq. bfv_dec); batch encoding and the server steps of the x^2 + x protocol
// (section "Proposed Secure Computation of Polynomial Activation Function").
// Kernels live in hc_client.hip; decryption's ring product c1 * s is the
// fused forward NTT / product / inverse NTT kernel of hc_ntt.hip.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/hc.h"
#include "hc_internal.h"
#include "hc_objects.h"

using hc::fail;
using hc::hip_fail;

namespace {

#define CL_HIP(call)                                  \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

using u128 = unsigned __int128;

uint64_t powmod(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = (uint64_t)((u128)r * a % m);
    a = (uint64_t)((u128)a * a % m);
    e >>= 1;
  }
  return r;
}

uint32_t shoup(uint32_t w, uint32_t q) { return (uint32_t)(((uint64_t)w << 32) / q); }

// True when [a, a + na) and [b, b + nb) (words) share memory.
bool overlap(const uint32_t *a, size_t na, const uint32_t *b, size_t nb) {
  const uintptr_t a0 = (uintptr_t)a, a1 = a0 + na * 4, b0 = (uintptr_t)b, b1 = b0 + nb * 4;
  return a0 < b1 && b0 < a1;
}

hc::EncGeom enc_geom(const hc_layer &ly) {
  hc::EncGeom e{};
  e.h = ly.shape.h;
  e.w = ly.shape.w;
  e.sub = ly.lay.sub;
  e.pad = ly.lay.pad;
  e.h_enc = ly.lay.h_enc;
  e.w_enc = ly.lay.w_enc;
  e.h_pad = ly.lay.h_pad;
  e.rows_per_ct = ly.lay.tiled ? ly.lay.rows_out_per_tile + ly.shape.f - 1 : ly.lay.h_pad;
  return e;
}

// NTT(s) into s_hat [L][N], then c1s [P][N] <- c1 * s for c1 [P][N] (c1 == c1s
// allowed): forward NTT, product and inverse NTT in one kernel per polynomial;
// with keep_bits < log2 N only the coefficients below 2^keep_bits are formed.
hc_status ring_times_secret(const hc_ctx &c, const uint32_t *sk, const uint32_t *c1, uint32_t *c1s, size_t np,
                            uint32_t *s_hat, hipStream_t st, uint32_t keep_bits = 32) {
  const hc::Shapes sh = hc::shapes_for(c, 1);
  CL_HIP(hc::launch_ntt_fwd(c.logn, sh.fe, sk, s_hat, c.L, c.consts, c.tw, st));
  CL_HIP(hc::launch_ring_mul(c.logn, sh.ie, c1, c1s, np, s_hat, 0, c.consts, c.tw, st, keep_bits));
  return HC_OK;
}

}  // namespace

hc::DecodeConsts hc::make_decode_consts(const uint32_t *q, uint32_t L, uint64_t t) {
  DecodeConsts d{};
  for (uint32_t l = 0; l < L; ++l) {
    const uint64_t ql = q[l];
    uint64_t star = 1;  // (q / q_l) mod q_l
    for (uint32_t k = 0; k < L; ++k)
      if (k != l) star = star * q[k] % ql;
    d.qt[l] = (uint32_t)powmod(star, ql - 2, ql);
    d.qt_p[l] = shoup(d.qt[l], (uint32_t)ql);
    d.a[l] = (uint32_t)((t / ql) % t);
    // floor(tau 2^160 / q_l), tau = t mod q_l < q_l: five base-2^32 digits by long division
    uint64_t rem = t % ql;
    for (int w = 4; w >= 0; --w) {
      const uint64_t num = rem << 32;
      d.phi[l][w] = (uint32_t)(num / ql);
      rem = num % ql;
    }
  }
  return d;
}

hc::DirectConsts hc::direct_consts(const hc_ctx &c) {
  DirectConsts d{};
  for (uint32_t l = 0; l < c.L; ++l) d.bias[l] = (uint64_t)c.q[l] * (((1ull << 55) + c.q[l] - 1) / c.q[l]);
  return d;
}

hc_status hc_encrypt_online(const hc_layer *ly, const uint32_t *act, const uint32_t *ct_zero, uint32_t *ct_in,
                            uint32_t B, void *stream) {
  if (!ly || (B && (!act || !ct_zero || !ct_in))) return fail(HC_EINVAL, "null argument");
  if (B == 0) return HC_OK;
  const hc_ctx &c = *ly->ctx;
  const size_t ct_words = (size_t)B * ly->lay.in_cts * 2 * c.L * c.N;
  const size_t act_words = (size_t)B * ly->shape.c_in * ly->shape.h * ly->shape.w;
  const bool in_place = ct_in == ct_zero;
  if (!in_place && overlap(ct_in, ct_words, ct_zero, ct_words))
    return fail(HC_EINVAL, "ct_in overlaps ct_zero without being the same buffer");
  if (overlap(ct_in, ct_words, act, act_words)) return fail(HC_EINVAL, "ct_in overlaps act");
  hc::DeviceGuard dg(c.device);
  CL_HIP(hc::launch_encrypt_online(ly->geom, enc_geom(*ly), act, ct_zero, ct_in, B, !in_place, c.consts,
                                   (hipStream_t)stream));
  return HC_OK;
}

hc_status hc_encrypt_zero(const hc_ctx *c, const uint32_t *a, const uint32_t *sk, const int32_t *e, uint32_t *ct_zero,
                          uint32_t count, void *ws, size_t ws_bytes, void *stream) {
  if (!c || (count && (!a || !sk || !e || !ct_zero || !ws))) return fail(HC_EINVAL, "null argument");
  if (count == 0) return HC_OK;
  const size_t np = (size_t)count * c->L;
  if (ws_bytes < (np + c->L) * c->N * sizeof(uint32_t)) return fail(HC_EINVAL, "workspace too small");
  if ((uintptr_t)ws & 15u) return fail(HC_EINVAL, "ws must be 16-byte aligned");
  const size_t ct_words = 2 * np * c->N;
  if (overlap(ct_zero, ct_words, a, np * c->N) || overlap(ct_zero, ct_words, (const uint32_t *)ws, np * c->N))
    return fail(HC_EINVAL, "ct_zero overlaps a or ws");
  uint32_t *as = (uint32_t *)ws, *s_hat = as + np * c->N;
  hipStream_t st = (hipStream_t)stream;
  hc::DeviceGuard dg(c->device);
  hc_status s = ring_times_secret(*c, sk, a, as, np, s_hat, st);
  if (s != HC_OK) return s;
  CL_HIP(hc::launch_encrypt_zero(a, as, e, ct_zero, count, c->N, c->consts, st));
  return HC_OK;
}

hc_status hc_decrypt_workspace_size(const hc_layer *ly, uint32_t B, size_t *bytes) {
  if (!ly || !bytes) return fail(HC_EINVAL, "null argument");
  const hc_ctx &c = *ly->ctx;
  *bytes = ((size_t)B * ly->lay.out_cts + 1) * c.L * c.N * sizeof(uint32_t);
  return HC_OK;
}

hc_status hc_decrypt_extracted(const hc_layer *ly, const uint32_t *c0_ext, const uint32_t *c1_out,
                               const uint32_t *sk, uint32_t *m, uint32_t B, void *ws, size_t ws_bytes,
                               void *stream) {
  if (!ly || (B && (!c0_ext || !c1_out || !sk || !m || !ws))) return fail(HC_EINVAL, "null argument");
  if (B == 0) return HC_OK;
  const hc_ctx &c = *ly->ctx;
  size_t need = 0;
  (void)hc_decrypt_workspace_size(ly, B, &need);
  if (ws_bytes < need) return fail(HC_EINVAL, "workspace too small");
  if ((uintptr_t)ws & 15u) return fail(HC_EINVAL, "ws must be 16-byte aligned");
  const size_t np = (size_t)B * ly->lay.out_cts * c.L;
  uint32_t *c1s = (uint32_t *)ws, *s_hat = c1s + np * c.N;
  hipStream_t st = (hipStream_t)stream;
  hc::DeviceGuard dg(c.device);
  // every extracted coefficient lies below 2^prune_bits
  hc_status s = ring_times_secret(c, sk, c1_out, c1s, np, s_hat, st, ly->geom.prune_bits);
  if (s != HC_OK) return s;
  CL_HIP(hc::launch_decrypt_extracted(ly->geom, c0_ext, c1s, m, B, c.consts, c.dec, st));
  return HC_OK;
}

hc_status hc_decrypt(const hc_ctx *c, const uint32_t *ct, const uint32_t *sk, uint32_t *m, uint32_t count, void *ws,
                     size_t ws_bytes, void *stream) {
  if (!c || (count && (!ct || !sk || !m || !ws))) return fail(HC_EINVAL, "null argument");
  if (count == 0) return HC_OK;
  const size_t np = (size_t)count * c->L;
  if (ws_bytes < (np + c->L) * c->N * sizeof(uint32_t)) return fail(HC_EINVAL, "workspace too small");
  if ((uintptr_t)ws & 15u) return fail(HC_EINVAL, "ws must be 16-byte aligned");
  uint32_t *c1s = (uint32_t *)ws, *s_hat = c1s + np * c->N;
  hipStream_t st = (hipStream_t)stream;
  hc::DeviceGuard dg(c->device);
  CL_HIP(hc::launch_gather_c1(ct, c1s, count, c->L, c->N, st));
  hc_status s = ring_times_secret(*c, sk, c1s, c1s, np, s_hat, st);
  if (s != HC_OK) return s;
  CL_HIP(hc::launch_decrypt_full(ct, c1s, m, count, c->N, c->consts, c->dec, st));
  return HC_OK;
}

// ------------------------------------------------------------- batch encoding, x^2 + x protocol
namespace {
hc_status need_batch(const hc_ctx *c) {
  if (!c->batch_ok) return fail(HC_EUNSUPPORTED, "batch encoding needs a prime t = 1 mod 2N below 2^30");
  return HC_OK;
}
}  // namespace

hc_status hc_batch_encode(const hc_ctx *c, const uint32_t *z, uint32_t *p, uint32_t n, void *stream) {
  if (!c || (n && (!z || !p))) return fail(HC_EINVAL, "null argument");
  hc_status s = need_batch(c);
  if (s != HC_OK || n == 0) return s;
  hc::DeviceGuard dg(c->device);
  CL_HIP(hc::launch_intt_full(c->logn, hc::shapes_for(*c, 1).ie, z, p, n, c->consts_t, c->tw_t,
                              (hipStream_t)stream));
  return HC_OK;
}

hc_status hc_batch_decode(const hc_ctx *c, const uint32_t *p, uint32_t *z, uint32_t n, void *stream) {
  if (!c || (n && (!z || !p))) return fail(HC_EINVAL, "null argument");
  hc_status s = need_batch(c);
  if (s != HC_OK || n == 0) return s;
  if ((uintptr_t)z & 15u) return fail(HC_EINVAL, "z must be 16-byte aligned");
  hc::DeviceGuard dg(c->device);
  CL_HIP(hc::launch_ntt_fwd(c->logn, hc::shapes_for(*c, 1).fe, p, z, n, c->consts_t, c->tw_t, (hipStream_t)stream));
  return HC_OK;
}

hc_status hc_encrypt_plain(const hc_ctx *c, const uint32_t *p, const uint32_t *ct_zero, uint32_t *ct, uint32_t n,
                           void *stream) {
  if (!c || (n && (!p || !ct_zero || !ct))) return fail(HC_EINVAL, "null argument");
  if (n == 0) return HC_OK;
  const size_t words = (size_t)n * 2 * c->L * c->N;
  if (ct != ct_zero && overlap(ct, words, ct_zero, words))
    return fail(HC_EINVAL, "ct overlaps ct_zero without being the same buffer");
  hipStream_t st = (hipStream_t)stream;
  hc::DeviceGuard dg(c->device);
  if (ct != ct_zero) CL_HIP(hipMemcpyAsync(ct, ct_zero, words * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
  CL_HIP(hc::launch_add_plain(ct, p, n, c->N, c->consts, st));
  return HC_OK;
}

hc_status hc_act_workspace_size(const hc_ctx *c, uint32_t n_ct, size_t *bytes) {
  if (!c || !bytes) return fail(HC_EINVAL, "null argument");
  *bytes = (size_t)n_ct * (c->L + 2) * c->N * sizeof(uint32_t);
  return HC_OK;
}

hc_status hc_act_pmult(const hc_ctx *c, const uint32_t *ct_batch, const uint32_t *r, const uint32_t *v,
                       uint32_t *ct_out, uint32_t n_ct, void *ws, size_t ws_bytes, void *stream) {
  if (!c || (n_ct && (!ct_batch || !r || !v || !ct_out || !ws))) return fail(HC_EINVAL, "null argument");
  hc_status s = need_batch(c);
  if (s != HC_OK || n_ct == 0) return s;
  size_t need = 0;
  (void)hc_act_workspace_size(c, n_ct, &need);
  if (ws_bytes < need) return fail(HC_EINVAL, "workspace too small");
  if ((uintptr_t)ws & 15u) return fail(HC_EINVAL, "ws must be 16-byte aligned");
  const size_t words = (size_t)n_ct * 2 * c->L * c->N;
  if (ct_out != ct_batch && overlap(ct_out, words, ct_batch, words))
    return fail(HC_EINVAL, "ct_out overlaps ct_batch without being the same buffer");
  const size_t pw = (size_t)n_ct * c->N;
  uint32_t *pr = (uint32_t *)ws, *pv = pr + pw, *lifted = pv + pw;
  hipStream_t st = (hipStream_t)stream;
  const hc::Shapes sh = hc::shapes_for(*c, 1);
  hc::DeviceGuard dg(c->device);
  // batch-encode r and v (inverse transforms modulo t; slot k = bit-reversed evaluation order)
  CL_HIP(hc::launch_intt_full(c->logn, sh.ie, r, pr, n_ct, c->consts_t, c->tw_t, st));
  CL_HIP(hc::launch_intt_full(c->logn, sh.ie, v, pv, n_ct, c->consts_t, c->tw_t, st));
  // encode(2r) = 2 encode(r): lift to every limb, NTT, then PMult of both components
  CL_HIP(hc::launch_lift_plain(pr, lifted, n_ct, c->N, 2, c->consts, st));
  CL_HIP(hc::launch_ntt_fwd(c->logn, sh.fe, lifted, lifted, (size_t)n_ct * c->L, c->consts, c->tw, st));
  // PMult of both components, with + Delta * encode(v) on c0 as it is stored
  CL_HIP(hc::launch_ring_mul(c->logn, sh.ie, ct_batch, ct_out, (size_t)n_ct * 2 * c->L, lifted, 2 * c->L, c->consts,
                             c->tw, st, 32, pv));
  return HC_OK;
}

hc_status hc_act_combine(const hc_layer *ly, const uint32_t *ct_x, const uint32_t *ct_y, const uint32_t *r,
                         const uint32_t *v, uint32_t *ct_out, uint32_t B, void *stream) {
  if (!ly || (B && (!ct_x || !ct_y || !r || !v || !ct_out))) return fail(HC_EINVAL, "null argument");
  if (B == 0) return HC_OK;
  const hc_ctx &c = *ly->ctx;
  const size_t words = (size_t)B * ly->lay.in_cts * 2 * c.L * c.N;
  if ((ct_out != ct_x && overlap(ct_out, words, ct_x, words)) || (ct_out != ct_y && overlap(ct_out, words, ct_y, words)))
    return fail(HC_EINVAL, "ct_out partly overlaps ct_x or ct_y");
  hc::DeviceGuard dg(c.device);
  CL_HIP(hc::launch_act_combine(ly->geom, enc_geom(*ly), ct_x, ct_y, r, v, ct_out, B, c.consts,
                                (hipStream_t)stream));
  return HC_OK;
}
