// Client-side entry points of libhconv (include/hc.h): the offline encryptions
// of zero and direct encoding with online encryption of a layer's input
// (Algorithm 2, section "Moving Data-independent Operations to Offline
// Phase"), and BFV decryption (eq. bfv_dec) of the masked convolution's outputs
// or of whole ciphertexts.
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
// allowed): forward NTT, product and inverse NTT in one kernel per polynomial.
hc_status ring_times_secret(const hc_ctx &c, const uint32_t *sk, const uint32_t *c1, uint32_t *c1s, size_t np,
                            uint32_t *s_hat, hipStream_t st) {
  const hc::Shapes sh = hc::shapes_for(c, 1);
  CL_HIP(hc::launch_ntt_fwd(c.logn, sh.fe, sk, s_hat, c.L, c.consts, c.tw, st));
  CL_HIP(hc::launch_ring_mul(c.logn, sh.ie, c1, c1s, np, s_hat, c.consts, c.tw, st));
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
  hc_status s = ring_times_secret(c, sk, c1_out, c1s, np, s_hat, st);
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
