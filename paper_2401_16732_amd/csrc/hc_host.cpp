// Host side of libhconv: the C ABI declared in include/hc.h.
//
// Parameters (RNS primes, roots of unity, twiddle and Shoup tables, Delta),
// the direct-encoding layout planner, resident weight encoding, the per-layer
// launch sequences and the graph-recorded batch. Kernels live in hc_ntt.hip,
// hc_mac.hip and hc_intt_masked_*.hip; the client-side entry points in
// hc_client.cpp, the serving loop in hc_server.cpp.
#include "../../include/hc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hc_internal.h"
#include "hc_objects.h"

using hc::ConvGeom;
using hc::LimbConsts;
using hc::Twiddles;
using u128 = unsigned __int128;

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace hc {
hc_status fail(hc_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}
hc_status hip_fail(hipError_t e, const char *where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  return HC_EDEVICE;
}
}  // namespace hc
using hc::fail;
using hc::hip_fail;
using hc::Shapes;
using hc::DeviceGuard;

namespace {
#define HC_HIP(call)                                  \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

// ------------------------------------------------------------- number theory
uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }
uint64_t powmod64(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = mulmod64(r, a, m);
    a = mulmod64(a, a, m);
    e >>= 1;
  }
  return r;
}
// Deterministic Miller-Rabin for n < 3.3e24 with the first 13 prime bases.
bool is_prime(uint64_t n) {
  if (n < 2) return false;
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41};
  for (uint64_t p : bases) {
    if (n % p == 0) return n == p;
  }
  uint64_t d = n - 1;
  int r = 0;
  while ((d & 1) == 0) {
    d >>= 1;
    ++r;
  }
  for (uint64_t a : bases) {
    uint64_t x = powmod64(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < r; ++i) {
      x = mulmod64(x, x, n);
      if (x == n - 1) {
        comp = false;
        break;
      }
    }
    if (comp) return false;
  }
  return true;
}
uint32_t shoup_of(uint32_t w, uint32_t q) { return (uint32_t)(((uint64_t)w << 32) / q); }
uint32_t bitrev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

// Transform tables of one prime q for ring degree N: fw[i] = {psi^brv(i), Shoup},
// iw[i] = {psi^-brv(i), Shoup}, with psi the first x^((q-1)/2N), x = 2, 3, ...,
// whose N-th power is -1; fills slot l of k with q and the inverse transform's
// constants. Returns psi, or 0 when q has no primitive 2N-th root.
uint32_t limb_tables(uint32_t q, uint32_t N, uint32_t logn, uint2 *fw, uint2 *iw, LimbConsts &k, uint32_t l) {
  const uint64_t two_n = 2ull * N;
  uint64_t psi = 0;
  for (uint64_t x = 2; x < q; ++x) {
    const uint64_t cand = powmod64(x, (q - 1) / two_n, q);
    if (powmod64(cand, N, q) == q - 1) {
      psi = cand;
      break;
    }
  }
  if (!psi) return 0;
  const uint64_t ipsi = powmod64(psi, q - 2, q);
  for (uint32_t i = 0; i < N; ++i) {
    const uint32_t e = bitrev(i, (int)logn);
    const uint32_t a = (uint32_t)powmod64(psi, e, q);
    const uint32_t b = (uint32_t)powmod64(ipsi, e, q);
    fw[i] = make_uint2(a, shoup_of(a, q));
    iw[i] = make_uint2(b, shoup_of(b, q));
  }
  const uint32_t ninv = (uint32_t)powmod64(N, q - 2, q);
  const uint32_t ninvw = (uint32_t)mulmod64(ninv, iw[1].x, q);
  k.q[l] = q;
  k.ninv[l] = ninv;
  k.ninv_p[l] = shoup_of(ninv, q);
  k.ninvw[l] = ninvw;
  k.ninvw_p[l] = shoup_of(ninvw, q);
  k.r2[l] = (uint32_t)((1ull << 32) % q);
  k.r2_p[l] = shoup_of(k.r2[l], q);
  k.one_p[l] = shoup_of(1, q);
  return (uint32_t)psi;
}

}  // namespace

constexpr int kChains = 4;  // concurrent chains of layers in a batch graph

struct hc_batch {
  hc_ctx *ctx = nullptr;
  std::vector<const hc_layer *> layers;
  uint32_t B = 0;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  std::vector<size_t> ws_off;  // per layer: start of its workspace region (shared within a chain)
  hipStream_t side[kChains] = {};
  hipEvent_t fork = nullptr, join[kChains] = {};
  hipGraphExec_t exec = nullptr;
  std::vector<const void *> key;  // pointers the graph was recorded with
  // grid cap of the graph's DMA-staged MAC launches (0: one workgroup per
  // tile): capped, a MAC leaves room on every compute unit for the kernels
  // of the other chains; 4 per compute unit by default
  uint32_t mac_cap = 0;
  // chunked two-stream pipeline (hc_batch_run_pipelined): its own workspace
  // (X-hat of the largest layer + Y-hat chunk buffers), streams and events
  void *pws = nullptr;
  size_t pws_bytes = 0;
  hipStream_t pa = nullptr, pb = nullptr;
  std::vector<hipEvent_t> pev;  // one per chunk and direction, recorded once per run
};

namespace {

bool valid_ring(uint32_t N) { return N >= 1024 && N <= 16384 && (N & (N - 1)) == 0; }

// The L largest primes < 2^30 with q = 1 mod 2N, descending.
bool auto_primes(uint32_t N, uint32_t L, uint32_t *q) {
  const uint64_t two_n = 2ull * N;
  uint64_t cand = (((1ull << 30) - 2) / two_n) * two_n + 1;
  for (uint32_t l = 0; l < L; cand -= two_n) {
    if (cand < two_n) return false;
    if (is_prime(cand)) q[l++] = (uint32_t)cand;
  }
  return true;
}

hc_status plan_impl(uint32_t N, const hc_conv_shape &s, hc_layout &o) {
  if (s.c_in == 0 || s.c_out == 0 || s.h == 0 || s.w == 0 || s.stride == 0)
    return fail(HC_EINVAL, "empty convolution shape");
  if (s.f % 2 == 0) return fail(HC_EUNSUPPORTED, "filter width must be odd");
  std::memset(&o, 0, sizeof(o));
  if (s.f == 1 && s.stride > 1) {
    o.sub = s.stride;
    o.s = 1;
    o.h_enc = (s.h + s.stride - 1) / s.stride;
    o.w_enc = (s.w + s.stride - 1) / s.stride;
  } else {
    o.sub = 1;
    o.s = s.stride;
    o.h_enc = s.h;
    o.w_enc = s.w;
  }
  o.pad = (s.f - 1) / 2;
  o.h_pad = o.h_enc + 2 * o.pad;
  o.w_pad = o.w_enc + 2 * o.pad;
  const uint64_t F = (uint64_t)o.h_pad * o.w_pad;
  const uint32_t grid_rows = o.h_pad - s.f + 1;
  if ((uint64_t)s.f * o.w_pad > N) return fail(HC_EUNSUPPORTED, "f * padded width exceeds the ring degree");
  if (F <= N) {
    o.footprint = (uint32_t)F;
    o.tiled = 0;
    o.cn = N / (uint32_t)F;
    o.tiles = 1;
    o.rows_out_per_tile = grid_rows;
    o.in_cts = (s.c_in + o.cn - 1) / o.cn;
    o.w_cts = o.in_cts;
  } else {
    const uint32_t R = N / o.w_pad;
    const uint32_t ro = ((R - s.f + 1) / o.s) * o.s;
    if (ro == 0) return fail(HC_EUNSUPPORTED, "no output row fits one ciphertext");
    if (F > 0xffffffffu) return fail(HC_EUNSUPPORTED, "input too large");
    o.footprint = (uint32_t)F;
    o.tiled = 1;
    o.cn = 1;
    o.rows_out_per_tile = ro;
    o.tiles = (grid_rows + ro - 1) / ro;
    o.in_cts = s.c_in * o.tiles;
    o.w_cts = s.c_in;
  }
  o.out_cts = s.c_out * o.tiles;
  o.ho = (o.h_pad - s.f) / o.s + 1;
  o.wo = (o.w_pad - s.f) / o.s + 1;
  return HC_OK;
}

ConvGeom geom_of(const hc_ctx &c, const hc_conv_shape &s, const hc_layout &o) {
  ConvGeom g{};
  g.N = c.N;
  g.L = c.L;
  g.c_in = s.c_in;
  g.c_out = s.c_out;
  g.f = s.f;
  g.s = o.s;
  g.cn = o.cn;
  g.tiled = o.tiled;
  g.T = o.tiles;
  g.r_o = o.rows_out_per_tile;
  g.G = o.in_cts;
  g.G_w = o.w_cts;
  g.O = o.out_cts;
  g.w_pad = o.w_pad;
  g.F = o.footprint;
  g.ho = o.ho;
  g.wo = o.wo;
  // largest extracted coefficient: output row s*oy - tau*r_o < r_o (and below the
  // stride-1 grid), column s*(wo-1)
  const uint32_t rows = std::min(o.rows_out_per_tile, o.h_pad - s.f + 1);
  const uint64_t e_max = (uint64_t)(((rows - 1) / o.s) * o.s) * o.w_pad + (uint64_t)o.s * (o.wo - 1);
  uint32_t pb = 0;
  while ((1ull << pb) <= e_max) ++pb;
  g.prune_bits = std::min(pb, c.logn);
  g.w_ld = s.c_out;
  return g;
}

size_t ct_words(const hc_ctx &c) { return (size_t)2 * c.L * c.N; }


// Defaults measured on MI355X (ResNet-50 layer mix, N = 8192).
uint32_t default_fwd_elog(uint32_t logn) { return logn >= 13 ? 5 : 4; }
uint32_t default_inv_elog(uint32_t logn) { return logn >= 10 ? 4 : 3; }
}  // namespace

hc::Shapes hc::shapes_for(const hc_ctx &c, uint32_t B) {
  Shapes s{};
  s.fe = c.tune.fwd_elog ? c.tune.fwd_elog : default_fwd_elog(c.logn);
  s.ie = c.tune.inv_elog ? c.tune.inv_elog : default_inv_elog(c.logn);
  s.ipw = c.tune.inv_polys ? c.tune.inv_polys : 1;
  if (c.tune.mac_rows) {
    s.mac = mac_of(c.tune);
  } else if (B >= 16) {
    s.mac = {4, 8, 4, 2, 2, 0, 0};
  } else if (B >= 4) {
    s.mac = {4, 4, 1, 4, 2, 0, 0};
  } else if (B >= 2) {
    s.mac = {2, 4, 1, 4, 2, 0, 0};
  } else {
    s.mac = {1, 8, 1, 4, 2, 0, 0};
  }
  return s;
}

const hc_tuning *hc::layer_tuning_for(const hc_layer *ly, uint32_t B) {
  if (B == 0) return nullptr;
  for (const auto &sl : ly->tunes)
    if (sl.B == B) return &sl.t;
  return nullptr;
}

void hc::layer_set_tuning(hc_layer *ly, uint32_t B, const hc_tuning &t) {
  int k = -1;
  for (int i = 0; i < hc_layer::kTuneSlots && k < 0; ++i)
    if (ly->tunes[i].B == B) k = i;
  for (int i = 0; i < hc_layer::kTuneSlots && k < 0; ++i)
    if (ly->tunes[i].B == 0) k = i;
  if (k < 0) k = (ly->tune_last + 1) % hc_layer::kTuneSlots;  // slots fill in order: the next is the oldest
  ly->tunes[k].B = B;
  ly->tunes[k].t = t;
  ly->tune_last = k;
}

hc::Shapes hc::layer_shapes(const hc_layer *ly, uint32_t B) {
  hc::Shapes s = shapes_for(*ly->ctx, B);
  if (const hc_tuning *tp = layer_tuning_for(ly, B)) {
    const hc_tuning &t = *tp;
    if (t.fwd_elog) s.fe = t.fwd_elog;
    if (t.inv_elog) s.ie = t.inv_elog;
    if (t.inv_polys) s.ipw = t.inv_polys;
    if (t.mac_rows) s.mac = mac_of(t);
  }
  // c0's transform in the MAC only where the layer allows it (a context-wide
  // tuning applies to every layer)
  if (s.mac.pre == hc::kMacC0 && !hc::mac_c0_ok(ly->geom)) s.mac.pre = 0;
  if (!hc::intt_masked_ok(ly->ctx->logn, s.ie, s.ipw, s.mac.pre)) s.ipw = 1;  // e.g. a tuned e = 5 under a context's 2
  return s;
}

namespace {
using hc::shapes_for;

// Optional per-stage timing: events recorded on the launch stream around each kernel.
struct StageTimer {
  hipEvent_t ev[6] = {};
  bool on = false;
};

// A2 -> A4 (+A5 when masked) for one layer on B images.
hc_status enqueue_conv(const hc_layer *ly, const uint32_t *ct_in, uint32_t *ct_out, const uint32_t *mask,
                       uint32_t *c0_ext, uint32_t *c1_out, uint32_t B, void *ws, bool masked, hipStream_t st,
                       StageTimer *tm = nullptr, uint32_t mac_cap = 0) {
  const hc_ctx &c = *ly->ctx;
  const ConvGeom &g = ly->geom;
  const bool timed = tm && tm->on;
  const Shapes sh = hc::layer_shapes(ly, B);
  if (!hc::mac_offsets_fit(g, sh.mac))
    return fail(HC_EUNSUPPORTED, "layer too large for the selected MAC tile (32-bit offsets); use smaller mac_rows");
  uint32_t *xhat = (uint32_t *)ws;
  const size_t npin = (size_t)B * g.G * 2 * c.L;
  if (timed) HC_HIP(hipEventRecord(tm->ev[0], st));
  HC_HIP(hc::launch_ntt_fwd(c.logn, sh.fe, ct_in, xhat, npin, c.consts, c.tw, st));
  if (timed) HC_HIP(hipEventRecord(tm->ev[1], st));
  if (!masked) {
    hc::MacShape m = sh.mac;
    m.pre = 0;  // the full inverse NTT runs every stage
    HC_HIP(hc::launch_mac(g, m, xhat, ly->d_w, ct_out, B, c.consts, c.tw, st));
    HC_HIP(hc::launch_intt_full(c.logn, sh.ie, ct_out, ct_out, (size_t)B * g.O * 2 * c.L, c.consts, c.tw, st,
                                false));  // the weights carry N^-1
  } else {
    uint32_t *yhat = xhat + npin * c.N;
    if (timed) HC_HIP(hipEventRecord(tm->ev[2], st));
    HC_HIP(hc::launch_mac(g, sh.mac, xhat, ly->d_w, yhat, B, c.consts, c.tw, st, mac_cap));
    if (timed) HC_HIP(hipEventRecord(tm->ev[3], st));
    if (timed) HC_HIP(hipEventRecord(tm->ev[4], st));
    HC_HIP(hc::launch_intt_masked(g, c.logn, sh.ie, sh.ipw, sh.mac.pre, yhat, mask, c0_ext, c1_out, B, c.consts,
                                  c.tw, st));
    if (timed) HC_HIP(hipEventRecord(tm->ev[5], st));
  }
  return HC_OK;
}

}  // namespace

size_t hc::ws_bytes_for(const hc_layer *ly, uint32_t B, bool masked) {
  const hc_ctx &c = *ly->ctx;
  size_t w = (size_t)B * ly->geom.G * ct_words(c);
  if (masked) w += (size_t)B * ly->geom.O * ct_words(c);
  return w * sizeof(uint32_t);
}
using hc::ws_bytes_for;

hc_status hc::enqueue_conv_gather(const hc_layer *ly, uint32_t B, const uint32_t *const *ct_in,
                                  const uint32_t *const *mask, uint32_t *const *c0, uint32_t *const *c1, void *ws,
                                  hipStream_t st) {
  const hc_ctx &c = *ly->ctx;
  const ConvGeom &g = ly->geom;
  if (B == 0 || B > hc::kMaxTab) return fail(HC_EINVAL, "group size out of range");
  const Shapes sh = hc::layer_shapes(ly, B);
  if (!hc::mac_offsets_fit(g, sh.mac)) return fail(HC_EUNSUPPORTED, "layer too large for the MAC tile");
  hc::ImgPtrs in{};
  hc::OutPtrs out{};
  in.n = out.n = B;
  for (uint32_t b = 0; b < B; ++b) {
    in.p[b] = (uint64_t)(uintptr_t)ct_in[b];
    out.mask[b] = (uint64_t)(uintptr_t)mask[b];
    out.c0[b] = (uint64_t)(uintptr_t)c0[b];
    out.c1[b] = (uint64_t)(uintptr_t)c1[b];
  }
  uint32_t *xhat = (uint32_t *)ws;
  const uint32_t ppi = g.G * 2 * c.L;
  const size_t npin = (size_t)B * ppi;
  HC_HIP(hc::launch_ntt_fwd(c.logn, sh.fe, nullptr, xhat, npin, c.consts, c.tw, st, &in, ppi));
  uint32_t *yhat = xhat + npin * c.N;
  HC_HIP(hc::launch_mac(g, sh.mac, xhat, ly->d_w, yhat, B, c.consts, c.tw, st));
  HC_HIP(hc::launch_intt_masked(g, c.logn, sh.ie, sh.ipw, sh.mac.pre, yhat, nullptr, nullptr, nullptr, B, c.consts,
                                c.tw, st, &out));
  return HC_OK;
}

// ------------------------------------------------------------- ABI
extern "C" {

const char *hc_status_string(hc_status s) {
  switch (s) {
    case HC_OK: return "ok";
    case HC_EINVAL: return "invalid argument";
    case HC_EUNSUPPORTED: return "unsupported";
    case HC_ENOMEM: return "out of memory";
    case HC_EDEVICE: return "device error";
    case HC_ESTATE: return "invalid state";
  }
  return "unknown status";
}

const char *hc_last_error(void) { return g_last_error.c_str(); }

hc_status hc_ctx_create(uint32_t N, uint32_t L, const uint32_t *primes, uint64_t t, int hip_device, hc_ctx **out) {
  if (!out) return fail(HC_EINVAL, "out is null");
  *out = nullptr;
  if (!valid_ring(N)) return fail(HC_EUNSUPPORTED, "N must be a power of two in [1024, 16384]");
  if (L < 1 || L > (uint32_t)hc::kMaxLimbs) return fail(HC_EUNSUPPORTED, "L must be in [1, 4]");
  if (t < 2 || t > (1ull << 30)) return fail(HC_EUNSUPPORTED, "t must be in [2, 2^30]");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev)
    return fail(HC_EDEVICE, "no such HIP device");
  hc_ctx *c = new (std::nothrow) hc_ctx;
  if (!c) return fail(HC_ENOMEM, "host allocation");
  c->N = N;
  c->L = L;
  c->t = t;
  c->device = hip_device;
  {
    const char *chk = std::getenv("HC_CHECK_INPUTS");
    c->check_inputs = chk && chk[0] == '1';
  }
  while ((1u << c->logn) < N) ++c->logn;
  const uint64_t two_n = 2ull * N;
  if (primes) {
    for (uint32_t l = 0; l < L; ++l) {
      const uint32_t q = primes[l];
      if (q >= (1u << 30) || q % two_n != 1 || !is_prime(q)) {
        delete c;
        return fail(HC_EINVAL, "prime " + std::to_string(q) + " is not a prime < 2^30 with q = 1 mod 2N");
      }
      for (uint32_t k = 0; k < l; ++k)
        if (primes[k] == q) {
          delete c;
          return fail(HC_EINVAL, "primes must be distinct");
        }
      c->q[l] = q;
    }
  } else if (!auto_primes(N, L, c->q)) {
    delete c;
    return fail(HC_EUNSUPPORTED, "not enough primes");
  }
  // centred plaintext values |m| <= t/2 must be residues of every limb
  for (uint32_t l = 0; l < L; ++l)
    if (t >= 2ull * c->q[l]) {
      delete c;
      return fail(HC_EUNSUPPORTED, "t must be below 2 q_l for every prime");
    }
  c->dec = hc::make_decode_consts(c->q, L, t);
  // Delta = floor(q / t), q = prod q_l < 2^120 (Notation table)
  u128 Q = 1;
  for (uint32_t l = 0; l < L; ++l) Q *= c->q[l];
  const u128 D = Q / t;
  LimbConsts &k = c->consts;
  std::memset(&k, 0, sizeof(k));
  k.t = (uint32_t)t;
  k.L = L;
  std::vector<uint2> tw((size_t)2 * L * N);
  for (uint32_t l = 0; l < L; ++l) {
    const uint32_t q = c->q[l];
    c->delta[l] = (uint32_t)(D % q);
    c->psi[l] = limb_tables(q, N, c->logn, tw.data() + (size_t)l * N, tw.data() + ((size_t)L + l) * N, k, l);
    if (!c->psi[l]) {
      delete c;
      return fail(HC_EINVAL, "no primitive 2N-th root of unity");
    }
    k.delta[l] = c->delta[l];
    k.delta_p[l] = shoup_of(c->delta[l], q);
    // terms that fit between folds: fold leaves acc < 2^32 * r2 + 2^32; each
    // term adds at most (q-1)^2; keep the total below 2^64
    const u128 lim = ((u128)1 << 64) - 1;
    const u128 base = ((u128)1 << 32) * k.r2[l] + ((u128)1 << 32);
    const u128 term = (u128)(q - 1) * (q - 1);
    u128 n_terms = (lim - base) / term;
    // at least 8 (n_terms >= 11 for q < 2^30), so the MAC's register ring
    // (2..4 ciphertexts deep) completes at least two turns between folds
    k.fold[l] = (uint32_t)std::min<u128>(n_terms, 64) & ~3u;
    if (k.fold[l] < 4) {
      delete c;
      return fail(HC_EINVAL, "prime too large for 64-bit accumulation");
    }
  }
  DeviceGuard dg(hip_device);
  const size_t bytes = tw.size() * sizeof(uint2);
  hipError_t e = hipMalloc((void **)&c->d_tw, bytes);
  if (e != hipSuccess) {
    delete c;
    return fail(HC_ENOMEM, "twiddle allocation");
  }
  e = hipMemcpy(c->d_tw, tw.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(c->d_tw);
    delete c;
    return hip_fail(e, "twiddle upload");
  }
  c->tw.fwd = c->d_tw;
  c->tw.inv = c->d_tw + (size_t)L * N;
  // the input check's counter
  e = hipMalloc((void **)&c->d_count, sizeof(unsigned long long));
  if (e != hipSuccess) {
    hc_ctx_destroy(c);
    return fail(HC_ENOMEM, "counter allocation");
  }
  // hc_conv_masked_noalloc's scratch address on this device; a failure here
  // only affects that entry point, which looks again and reports it
  (void)hc::noalloc_init(hip_device);
  // batch (slot) encoding: transforms modulo t itself when t is a prime = 1 mod 2N
  if (t < (1ull << 30) && t % two_n == 1 && is_prime(t)) {
    std::vector<uint2> twt((size_t)2 * N);
    LimbConsts &kt = c->consts_t;
    std::memset(&kt, 0, sizeof(kt));
    kt.L = 1;
    kt.t = (uint32_t)t;
    if (limb_tables((uint32_t)t, N, c->logn, twt.data(), twt.data() + N, kt, 0)) {
      e = hipMalloc((void **)&c->d_tw_t, twt.size() * sizeof(uint2));
      if (e == hipSuccess) e = hipMemcpy(c->d_tw_t, twt.data(), twt.size() * sizeof(uint2), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        hc_ctx_destroy(c);
        return hip_fail(e, "batch-encoding twiddles");
      }
      c->tw_t.fwd = c->d_tw_t;
      c->tw_t.inv = c->d_tw_t + N;
      c->batch_ok = true;
    }
  }
  *out = c;
  return HC_OK;
}

hc_status hc_ctx_info(const hc_ctx *c, uint32_t *primes_out, uint32_t *delta_out) {
  if (!c) return fail(HC_EINVAL, "ctx is null");
  for (uint32_t l = 0; l < c->L; ++l) {
    if (primes_out) primes_out[l] = c->q[l];
    if (delta_out) delta_out[l] = c->delta[l];
  }
  return HC_OK;
}

void hc_ctx_destroy(hc_ctx *c) {
  if (!c) return;
  DeviceGuard dg(c->device);
  if (c->d_tw) (void)hipFree(c->d_tw);
  if (c->d_tw_t) (void)hipFree(c->d_tw_t);
  if (c->d_count) (void)hipFree(c->d_count);
  delete c;
}

hc_status hc_ctx_set_tuning(hc_ctx *c, const hc_tuning *t) {
  if (!c || !t) return fail(HC_EINVAL, "null argument");
  if (t->fwd_elog && !hc::ntt_variant_ok(c->logn, t->fwd_elog))
    return fail(HC_EUNSUPPORTED, "forward NTT shape not available for this N");
  if (t->inv_elog && !hc::ntt_variant_ok(c->logn, t->inv_elog))
    return fail(HC_EUNSUPPORTED, "inverse NTT shape not available for this N");
  if (t->inv_polys &&
      !hc::intt_masked_ok(c->logn, t->inv_elog ? t->inv_elog : default_inv_elog(c->logn), t->inv_polys, 0))
    return fail(HC_EUNSUPPORTED, "inverse NTT polynomials per workgroup not available for this shape");
  if (t->mac_pre == hc::kMacPre && c->logn < 12) return fail(HC_EUNSUPPORTED, "MAC epilogue stages need N >= 4096");
  const bool any = t->mac_rows || t->mac_cols || t->mac_row_groups || t->mac_col_groups || t->mac_depth ||
                   t->mac_lds || t->mac_pre;
  const bool all = t->mac_rows && t->mac_cols && t->mac_row_groups && t->mac_col_groups;
  if (any && !all) return fail(HC_EINVAL, "set all four MAC fields or none");
  if (all && !hc::mac_variant_ok(hc::mac_of(*t)))
    return fail(HC_EUNSUPPORTED, "MAC tile not available");
  c->tune = *t;
  return HC_OK;
}

hc_status hc_ctx_get_tuning(const hc_ctx *c, hc_tuning *out) {
  if (!c || !out) return fail(HC_EINVAL, "null argument");
  *out = c->tune;
  return HC_OK;
}

hc_status hc_plan(const hc_ctx *c, const hc_conv_shape *s, hc_layout *o) {
  if (!c || !s || !o) return fail(HC_EINVAL, "null argument");
  return plan_impl(c->N, *s, *o);
}

hc_status hc_plan_ring(uint32_t N, const hc_conv_shape *s, hc_layout *o) {
  if (!s || !o) return fail(HC_EINVAL, "null argument");
  if (!valid_ring(N)) return fail(HC_EUNSUPPORTED, "N must be a power of two in [1024, 16384]");
  return plan_impl(N, *s, *o);
}

hc_status hc_ring_params(uint32_t N, uint32_t L, uint64_t t, uint32_t *primes_out, uint32_t *delta_out) {
  if (!valid_ring(N)) return fail(HC_EUNSUPPORTED, "N must be a power of two in [1024, 16384]");
  if (L < 1 || L > (uint32_t)hc::kMaxLimbs) return fail(HC_EUNSUPPORTED, "L must be in [1, 4]");
  if (t < 2 || t > (1ull << 30)) return fail(HC_EUNSUPPORTED, "t must be in [2, 2^30]");
  uint32_t q[hc::kMaxLimbs];
  if (!auto_primes(N, L, q)) return fail(HC_EUNSUPPORTED, "not enough primes");
  u128 Q = 1;
  for (uint32_t l = 0; l < L; ++l) Q *= q[l];
  const u128 D = Q / t;
  for (uint32_t l = 0; l < L; ++l) {
    if (primes_out) primes_out[l] = q[l];
    if (delta_out) delta_out[l] = (uint32_t)(D % q[l]);
  }
  return HC_OK;
}

hc_status hc_layer_create(hc_ctx *c, const hc_conv_shape *s, const int8_t *filters, void *stream, hc_layer **out) {
  if (!c || !s || !filters || !out) return fail(HC_EINVAL, "null argument");
  *out = nullptr;
  hc_layout lay;
  hc_status st = plan_impl(c->N, *s, lay);
  if (st != HC_OK) return st;
  DeviceGuard dg(c->device);
  hc_layer *ly = new (std::nothrow) hc_layer;
  if (!ly) return fail(HC_ENOMEM, "host allocation");
  ly->ctx = c;
  ly->shape = *s;
  ly->lay = lay;
  ly->geom = geom_of(*c, *s, lay);
  ly->w_elems = (size_t)s->c_out * lay.w_cts * c->L * c->N;
  hipStream_t hs = (hipStream_t)stream;
  if (hipMalloc((void **)&ly->d_w, ly->w_elems * sizeof(uint32_t)) != hipSuccess) {
    delete ly;
    return fail(HC_ENOMEM, "weight allocation");
  }
  const size_t fbytes = (size_t)s->c_out * s->c_in * s->f * s->f;
  int8_t *d_f = nullptr;
  hipError_t e = hipMalloc((void **)&d_f, fbytes);
  if (e == hipSuccess) e = hipMemcpyAsync(d_f, filters, fbytes, hipMemcpyHostToDevice, hs);
  if (e == hipSuccess) e = hc::launch_fill_zero(ly->d_w, ly->w_elems, hs);
  if (e == hipSuccess) e = hc::launch_weight_scatter(ly->geom, d_f, ly->d_w, c->consts, hs);
  if (e == hipSuccess)
    e = hc::launch_ntt_fwd(c->logn, shapes_for(*c, 1).fe, ly->d_w, ly->d_w, (size_t)s->c_out * lay.w_cts * c->L,
                           c->consts, c->tw, hs);
  // stored times N^-1: every sum then carries the inverse NTT's final factor,
  // and the inverse NTT of the convolution skips it
  if (e == hipSuccess) e = hc::launch_scale_ninv(ly->d_w, ly->w_elems, c->N, c->consts, hs);
  // then in the multiply-accumulate's blocked layout (runs of channels per
  // coefficient block and input ciphertext)
  uint32_t *d_wb = nullptr;
  if (e == hipSuccess) e = hipMalloc((void **)&d_wb, ly->w_elems * sizeof(uint32_t));
  if (e == hipSuccess) e = hc::launch_weight_block(ly->d_w, d_wb, s->c_out, lay.w_cts, c->L, c->N, hs);
  // int32 filter table for the coefficient-domain conv, rows padded to 16.
  // At one image it beats the NTT path where c_n f^2 <= 2 (measured on the
  // ResNet-50 layer mix at N = 8192: exactly those layers win, all others lose).
  ly->wt_rows = (s->c_out + 15u) / 16u * 16u;
  ly->direct_one = !lay.tiled && (uint64_t)lay.cn * s->f * s->f <= 2 && (uint64_t)s->c_in * s->f * s->f <= (1u << 17);
  const size_t taps = (size_t)s->f * s->f;
  std::vector<int32_t> wt((size_t)ly->wt_rows * s->c_in * taps, 0);
  for (size_t k = 0; k < (size_t)s->c_out * s->c_in * taps; ++k) wt[k] = filters[k];
  if (e == hipSuccess) e = hipMalloc((void **)&ly->d_wt, wt.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemcpyAsync(ly->d_wt, wt.data(), wt.size() * sizeof(int32_t), hipMemcpyHostToDevice, hs);
  if (e == hipSuccess) e = hipStreamSynchronize(hs);
  if (d_f) (void)hipFree(d_f);
  (void)hipFree(ly->d_w);  // the natural-layout copy
  ly->d_w = d_wb;
  if (e != hipSuccess) {
    if (ly->d_w) (void)hipFree(ly->d_w);
    if (ly->d_wt) (void)hipFree(ly->d_wt);
    delete ly;
    return hip_fail(e, "weight encoding");
  }
  *out = ly;
  return HC_OK;
}

void hc_layer_destroy(hc_layer *ly) {
  if (!ly) return;
  DeviceGuard dg(ly->ctx->device);
  if (ly->d_w) (void)hipFree(ly->d_w);
  if (ly->d_wt) (void)hipFree(ly->d_wt);
  delete ly;
}

hc_status hc_layer_plan(const hc_layer *ly, hc_layout *out) {
  if (!ly || !out) return fail(HC_EINVAL, "null argument");
  *out = ly->lay;
  return HC_OK;
}

hc_status hc_workspace_size(const hc_layer *ly, uint32_t B, int masked, size_t *bytes) {
  if (!ly || !bytes) return fail(HC_EINVAL, "null argument");
  *bytes = ws_bytes_for(ly, B, masked != 0);
  return HC_OK;
}

namespace {
// Number of non-canonical words in npolys polynomials [..][L][N], counted on
// the device; the call waits for the stream.
// It uses the context's counter (allocated with the context): no allocation
// here, and calls on one context are serialised. Refused (HC_ESTATE) while
// the stream is being captured into a graph, since it waits for the stream.
hc_status count_noncanonical(const hc_ctx &c, const uint32_t *p, size_t npolys, hipStream_t st, uint64_t *n_bad) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HC_HIP(hipStreamIsCapturing(st, &cap));
  if (cap != hipStreamCaptureStatusNone)
    return fail(HC_ESTATE, "the residue check waits for its stream and cannot run under graph capture");
  std::lock_guard<std::mutex> lk(*c.count_mu);
  unsigned long long *d = c.d_count;
  static const unsigned long long zero = 0;
  unsigned long long h = 0;
  hipError_t e = hipMemcpyAsync(d, &zero, sizeof(zero), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hc::launch_count_noncanonical(p, npolys, c.N, c.consts, d, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "residue check");
  *n_bad = h;
  return HC_OK;
}
// With HC_CHECK_INPUTS=1: HC_EINVAL when an input ciphertext word is not canonical.
hc_status check_input(const hc_layer *ly, const uint32_t *ct_in, uint32_t B, hipStream_t st) {
  if (!ly->ctx->check_inputs) return HC_OK;
  uint64_t bad = 0;
  hc_status s = count_noncanonical(*ly->ctx, ct_in, (size_t)B * ly->lay.in_cts * 2 * ly->ctx->L, st, &bad);
  if (s != HC_OK) return s;
  return bad ? fail(HC_EINVAL, "input ciphertext word not below its prime") : HC_OK;
}
}  // namespace

}  // extern "C"

hc_status hc::conv_masked_on(const hc_layer *ly, const uint32_t *ct_in, const uint32_t *mask, uint32_t *c0_ext,
                             uint32_t *c1_out, uint32_t B, void *ws, hipStream_t st) {
  hc_status s = check_input(ly, ct_in, B, st);
  if (s != HC_OK) return s;
  return enqueue_conv(ly, ct_in, nullptr, mask, c0_ext, c1_out, B, ws, true, st);
}

extern "C" {

hc_status hc_check_residues(const hc_ctx *c, const uint32_t *polys, size_t npolys, void *stream, uint64_t *n_bad) {
  if (!c || !n_bad || (npolys && !polys)) return fail(HC_EINVAL, "null argument");
  *n_bad = 0;
  if (npolys == 0) return HC_OK;
  DeviceGuard dg(c->device);
  return count_noncanonical(*c, polys, npolys, (hipStream_t)stream, n_bad);
}

hc_status hc_conv(const hc_layer *ly, const uint32_t *ct_in, uint32_t *ct_out, uint32_t B, void *ws, size_t ws_bytes,
                  void *stream) {
  if (!ly || (B && (!ct_in || !ct_out || !ws))) return fail(HC_EINVAL, "null argument");
  if (B == 0) return HC_OK;
  if (ws_bytes < ws_bytes_for(ly, B, false)) return fail(HC_EINVAL, "workspace too small");
  DeviceGuard dg(ly->ctx->device);
  hc_status s = check_input(ly, ct_in, B, (hipStream_t)stream);
  if (s != HC_OK) return s;
  return enqueue_conv(ly, ct_in, ct_out, nullptr, nullptr, nullptr, B, ws, false, (hipStream_t)stream);
}

hc_status hc_mask_extract(const hc_layer *ly, const uint32_t *ct_out, const uint32_t *mask, uint32_t *c0_ext,
                          uint32_t *c1_out, uint32_t B, void *stream) {
  if (!ly || (B && (!ct_out || !mask || !c0_ext || !c1_out))) return fail(HC_EINVAL, "null argument");
  if (B == 0) return HC_OK;
  if (((uintptr_t)ct_out | (uintptr_t)c1_out) & 15u) return fail(HC_EINVAL, "ct_out and c1_out must be 16-byte aligned");
  DeviceGuard dg(ly->ctx->device);
  HC_HIP(hc::launch_mask_extract(ly->geom, ct_out, mask, c0_ext, c1_out, B, ly->ctx->consts, (hipStream_t)stream));
  return HC_OK;
}

hc_status hc_conv_masked_direct(const hc_layer *ly, const uint32_t *ct_in, const uint32_t *mask, uint32_t *c0_ext,
                                uint32_t *c1_out, uint32_t B, void *stream) {
  if (!ly || (B && (!ct_in || !mask || !c0_ext || !c1_out))) return fail(HC_EINVAL, "null argument");
  if (ly->lay.tiled) return fail(HC_EUNSUPPORTED, "the coefficient-domain conv covers untiled layers only");
  if ((uint64_t)ly->shape.c_in * ly->shape.f * ly->shape.f > (1u << 17))
    return fail(HC_EUNSUPPORTED, "c_in f^2 above 2^17 (64-bit sum bound)");
  if ((uint64_t)B * ly->ctx->L > 65535) return fail(HC_EUNSUPPORTED, "B L above 65535");
  if (B == 0) return HC_OK;
  const hc_ctx &c = *ly->ctx;
  DeviceGuard dg(c.device);
  hc_status s = check_input(ly, ct_in, B, (hipStream_t)stream);
  if (s != HC_OK) return s;
  HC_HIP(hc::launch_conv_direct(ly->geom, ct_in, ly->d_wt, ly->wt_rows, mask, c0_ext, c1_out, B,
                                hc::direct_consts(c), c.consts, (hipStream_t)stream));
  return HC_OK;
}

hc_status hc_conv_masked(const hc_layer *ly, const uint32_t *ct_in, const uint32_t *mask, uint32_t *c0_ext,
                         uint32_t *c1_out, uint32_t B, void *ws, size_t ws_bytes, void *stream) {
  if (!ly || (B && (!ct_in || !mask || !c0_ext || !c1_out || !ws))) return fail(HC_EINVAL, "null argument");
  if (B == 0) return HC_OK;
  if (ws_bytes < ws_bytes_for(ly, B, true)) return fail(HC_EINVAL, "workspace too small");
  DeviceGuard dg(ly->ctx->device);
  return hc::conv_masked_on(ly, ct_in, mask, c0_ext, c1_out, B, ws, (hipStream_t)stream);
}

hc_status hc_poly_mul(const hc_ctx *c, const uint32_t *a, const uint32_t *b, uint32_t *out, uint32_t count, void *ws,
                      size_t ws_bytes, void *stream) {
  if (!c || (count && (!a || !b || !out || !ws))) return fail(HC_EINVAL, "null argument");
  if (count == 0) return HC_OK;
  const size_t np = (size_t)count * c->L;
  if (ws_bytes < 2 * np * c->N * sizeof(uint32_t)) return fail(HC_EINVAL, "workspace too small");
  DeviceGuard dg(c->device);
  hipStream_t st = (hipStream_t)stream;
  uint32_t *wa = (uint32_t *)ws, *wb = wa + np * c->N;
  const Shapes sh = shapes_for(*c, 1);
  HC_HIP(hc::launch_ntt_fwd(c->logn, sh.fe, a, wa, np, c->consts, c->tw, st));
  HC_HIP(hc::launch_ntt_fwd(c->logn, sh.fe, b, wb, np, c->consts, c->tw, st));
  HC_HIP(hc::launch_pointwise_mul(wa, wb, wa, np, c->N, c->consts, st));
  HC_HIP(hc::launch_intt_full(c->logn, sh.ie, wa, out, np, c->consts, c->tw, st));
  return HC_OK;
}

hc_status hc_sync(hc_ctx *c) {
  if (!c) return fail(HC_EINVAL, "ctx is null");
  DeviceGuard dg(c->device);
  HC_HIP(hipDeviceSynchronize());
  return HC_OK;
}

// ------------------------------------------------------------- batch (graph)
hc_status hc_batch_create(hc_ctx *c, const hc_layer *const *layers, uint32_t n, uint32_t B, hc_batch **out) {
  if (!c || !out || (n && !layers)) return fail(HC_EINVAL, "null argument");
  *out = nullptr;
  if (n == 0 || B == 0) return fail(HC_EINVAL, "empty batch");
  for (uint32_t k = 0; k < n; ++k) {
    if (!layers[k]) return fail(HC_EINVAL, "null layer");
    if (layers[k]->ctx != c) return fail(HC_ESTATE, "layer belongs to another context");
  }
  DeviceGuard dg(c->device);
  hc_batch *bt = new (std::nothrow) hc_batch;
  if (!bt) return fail(HC_ENOMEM, "host allocation");
  bt->ctx = c;
  bt->B = B;
  bt->layers.assign(layers, layers + n);
  // Layer k runs in chain k % kChains of the recorded graph; layers of one
  // chain run one after another, so each chain needs one region, sized for
  // its largest layer.
  size_t region[kChains] = {};
  for (uint32_t k = 0; k < n; ++k)
    region[k % kChains] = std::max(region[k % kChains], (ws_bytes_for(layers[k], B, true) + 255) & ~(size_t)255);
  size_t start[kChains], off = 0;
  for (int c = 0; c < kChains; ++c) start[c] = off, off += region[c];
  for (uint32_t k = 0; k < n; ++k) bt->ws_off.push_back(start[k % kChains]);
  bt->ws_bytes = off;
  if (hipMalloc(&bt->ws, off) != hipSuccess) {
    delete bt;
    return fail(HC_ENOMEM, "batch workspace allocation");
  }
  hipError_t e = hipEventCreateWithFlags(&bt->fork, hipEventDisableTiming);
  for (int s = 0; s < kChains && e == hipSuccess; ++s) {
    e = hipStreamCreateWithFlags(&bt->side[s], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&bt->join[s], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    hc_batch_destroy(bt);
    return hip_fail(e, "batch streams");
  }
  bt->mac_cap = 0;  // one workgroup per MAC tile (hc_batch_set_mac_cap)
  *out = bt;
  return HC_OK;
}

hc_status hc_batch_workspace_bytes(const hc_batch *bt, size_t *bytes) {
  if (!bt || !bytes) return fail(HC_EINVAL, "null argument");
  *bytes = bt->ws_bytes;
  return HC_OK;
}

static hc_status batch_check(hc_batch *bt, const uint32_t *const *ct_in, const uint32_t *const *mask,
                             uint32_t *const *c0, uint32_t *const *c1) {
  if (!bt || !ct_in || !mask || !c0 || !c1) return fail(HC_EINVAL, "null argument");
  for (size_t k = 0; k < bt->layers.size(); ++k)
    if (!ct_in[k] || !mask[k] || !c0[k] || !c1[k]) return fail(HC_EINVAL, "null buffer for a layer");
  return HC_OK;
}

hc_status hc_batch_run_eager(hc_batch *bt, const uint32_t *const *ct_in, const uint32_t *const *mask,
                             uint32_t *const *c0, uint32_t *const *c1, void *stream) {
  hc_status s = batch_check(bt, ct_in, mask, c0, c1);
  if (s != HC_OK) return s;
  DeviceGuard dg(bt->ctx->device);
  for (size_t k = 0; k < bt->layers.size(); ++k) {
    s = enqueue_conv(bt->layers[k], ct_in[k], nullptr, mask[k], c0[k], c1[k], bt->B,
                     (char *)bt->ws + bt->ws_off[k], true, (hipStream_t)stream);
    if (s != HC_OK) return s;
  }
  return HC_OK;
}

hc_status hc_batch_run(hc_batch *bt, const uint32_t *const *ct_in, const uint32_t *const *mask, uint32_t *const *c0,
                       uint32_t *const *c1, void *stream) {
  hc_status s = batch_check(bt, ct_in, mask, c0, c1);
  if (s != HC_OK) return s;
  DeviceGuard dg(bt->ctx->device);
  hipStream_t st = (hipStream_t)stream;
  const size_t n = bt->layers.size();
  std::vector<const void *> key;
  key.reserve(4 * n + 4);
  key.push_back((const void *)(uintptr_t)bt->ctx->tune.fwd_elog);
  key.push_back((const void *)(uintptr_t)bt->ctx->tune.inv_elog);
  key.push_back((const void *)(uintptr_t)bt->ctx->tune.mac_rows);
  key.push_back((const void *)(uintptr_t)bt->ctx->tune.mac_cols);
  key.push_back((const void *)(uintptr_t)bt->ctx->tune.mac_row_groups);
  key.push_back((const void *)(uintptr_t)bt->ctx->tune.mac_col_groups);
  key.push_back((const void *)(uintptr_t)bt->ctx->tune.mac_depth);
  key.push_back((const void *)(uintptr_t)bt->ctx->tune.mac_lds);
  key.push_back((const void *)(uintptr_t)bt->ctx->tune.inv_polys);
  key.push_back((const void *)(uintptr_t)bt->ctx->tune.mac_pre);
  key.push_back((const void *)(uintptr_t)bt->mac_cap);
  for (size_t k = 0; k < n; ++k) {
    key.push_back(ct_in[k]);
    key.push_back(mask[k]);
    key.push_back(c0[k]);
    key.push_back(c1[k]);
  }
  if (!bt->exec || key != bt->key) {
    if (bt->exec) {
      (void)hipGraphExecDestroy(bt->exec);
      bt->exec = nullptr;
    }
    // Record: the layers are independent, so they are spread over 4 side
    // streams forked from and joined back into the capturing stream; the
    // graph then holds 4 concurrent chains.
    hipStream_t cap = nullptr;
    HC_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = hipEventRecord(bt->fork, cap);
    for (int sd = 0; sd < kChains && e == hipSuccess; ++sd) e = hipStreamWaitEvent(bt->side[sd], bt->fork, 0);
    hc_status cs = HC_OK;
    for (size_t k = 0; k < n && e == hipSuccess && cs == HC_OK; ++k)
      cs = enqueue_conv(bt->layers[k], ct_in[k], nullptr, mask[k], c0[k], c1[k], bt->B,
                        (char *)bt->ws + bt->ws_off[k], true, bt->side[k % kChains], nullptr, bt->mac_cap);
    for (int sd = 0; sd < kChains && e == hipSuccess; ++sd) {
      e = hipEventRecord(bt->join[sd], bt->side[sd]);
      if (e == hipSuccess) e = hipStreamWaitEvent(cap, bt->join[sd], 0);
    }
    hipError_t e2 = hipStreamEndCapture(cap, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess && cs == HC_OK) e = hipGraphInstantiate(&bt->exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cap);
    if (cs != HC_OK) return cs;
    if (e != hipSuccess) return hip_fail(e, "batch graph capture");
    bt->key = key;
  }
  HC_HIP(hipGraphLaunch(bt->exec, st));
  return HC_OK;
}

hc_status hc_batch_run_timed(hc_batch *bt, const uint32_t *const *ct_in, const uint32_t *const *mask,
                             uint32_t *const *c0, uint32_t *const *c1, void *stream, double *stage_ms) {
  hc_status s = batch_check(bt, ct_in, mask, c0, c1);
  if (s != HC_OK) return s;
  if (!stage_ms) return fail(HC_EINVAL, "stage_ms is null");
  DeviceGuard dg(bt->ctx->device);
  hipStream_t st = (hipStream_t)stream;
  StageTimer tm;
  tm.on = true;
  for (int k = 0; k < 6; ++k) HC_HIP(hipEventCreate(&tm.ev[k]));
  hc_status out = HC_OK;
  for (size_t k = 0; k < bt->layers.size() && out == HC_OK; ++k) {
    out = enqueue_conv(bt->layers[k], ct_in[k], nullptr, mask[k], c0[k], c1[k], bt->B,
                       (char *)bt->ws + bt->ws_off[k], true, st, &tm);
    if (out != HC_OK) break;
    hipError_t e = hipEventSynchronize(tm.ev[5]);
    float a = 0, b = 0, c = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&a, tm.ev[0], tm.ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&b, tm.ev[2], tm.ev[3]);
    if (e == hipSuccess) e = hipEventElapsedTime(&c, tm.ev[4], tm.ev[5]);
    if (e != hipSuccess) out = hip_fail(e, "stage timing");
    stage_ms[0] += a;
    stage_ms[1] += b;
    stage_ms[2] += c;
  }
  for (int k = 0; k < 6; ++k) (void)hipEventDestroy(tm.ev[k]);
  return out;
}

}  // extern "C"

namespace {

// Output channels per chunk of layer ly for the pipelined run: about
// chunk_bytes of Y-hat, a multiple of the MAC's channel tile, at least one tile.
uint32_t chunk_channels(const hc_layer *ly, uint32_t B, uint64_t chunk_bytes) {
  const hc_ctx &c = *ly->ctx;
  const hc::ConvGeom &g = ly->geom;
  const uint64_t per_ch = (uint64_t)B * g.T * 2 * c.L * c.N * 4;
  const hc::Shapes sh = hc::layer_shapes(ly, B);
  const uint32_t tile = sh.mac.cg * sh.mac.ct;
  uint64_t n = chunk_bytes / per_ch;
  n = n / tile * tile;
  if (n < tile) n = tile;
  return (uint32_t)std::min<uint64_t>(n, g.c_out);
}

}  // namespace

extern "C" {

hc_status hc_batch_run_pipelined(hc_batch *bt, const uint32_t *const *ct_in, const uint32_t *const *mask,
                                 uint32_t *const *c0, uint32_t *const *c1, uint64_t chunk_bytes, uint32_t nbuf,
                                 void *stream) {
  hc_status s = batch_check(bt, ct_in, mask, c0, c1);
  if (s != HC_OK) return s;
  if (chunk_bytes == 0 || nbuf < 2 || nbuf > 8) return fail(HC_EINVAL, "chunk_bytes > 0 and 2 <= nbuf <= 8");
  const hc_ctx &c = *bt->ctx;
  DeviceGuard dg(c.device);
  hipStream_t st = (hipStream_t)stream;
  const uint32_t B = bt->B;
  const size_t n = bt->layers.size();
  // workspace: X-hat of the largest layer, then nbuf chunk buffers of the largest chunk
  size_t xbytes = 0, ybytes = 0, nchunks = 0;
  std::vector<uint32_t> nch(n);
  for (size_t k = 0; k < n; ++k) {
    const hc_layer *ly = bt->layers[k];
    const hc::ConvGeom &g = ly->geom;
    nch[k] = chunk_channels(ly, B, chunk_bytes);
    xbytes = std::max(xbytes, (size_t)B * g.G * 2 * c.L * c.N * 4);
    ybytes = std::max(ybytes, (size_t)B * nch[k] * g.T * 2 * c.L * c.N * 4);
    nchunks += (g.c_out + nch[k] - 1) / nch[k];
  }
  xbytes = (xbytes + 255) & ~(size_t)255;
  ybytes = (ybytes + 255) & ~(size_t)255;
  const size_t need = xbytes + nbuf * ybytes;
  if (bt->pws_bytes < need) {
    HC_HIP(hipDeviceSynchronize());
    if (bt->pws) (void)hipFree(bt->pws);
    bt->pws = nullptr;
    bt->pws_bytes = 0;
    if (hipMalloc(&bt->pws, need) != hipSuccess) return fail(HC_ENOMEM, "pipeline workspace allocation");
    bt->pws_bytes = need;
  }
  if (!bt->pa) HC_HIP(hipStreamCreateWithFlags(&bt->pa, hipStreamNonBlocking));
  if (!bt->pb) HC_HIP(hipStreamCreateWithFlags(&bt->pb, hipStreamNonBlocking));
  // events: 2 per chunk (MAC done, inverse done) + start + 2 ends
  const size_t nev = 2 * nchunks + 3;
  while (bt->pev.size() < nev) {
    hipEvent_t ev = nullptr;
    HC_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    bt->pev.push_back(ev);
  }
  hipEvent_t ev_start = bt->pev[2 * nchunks], ev_ea = bt->pev[2 * nchunks + 1], ev_eb = bt->pev[2 * nchunks + 2];
  hipStream_t sa = bt->pa, sb = bt->pb;
  HC_HIP(hipEventRecord(ev_start, st));
  HC_HIP(hipStreamWaitEvent(sa, ev_start, 0));
  HC_HIP(hipStreamWaitEvent(sb, ev_start, 0));
  uint32_t *xhat = (uint32_t *)bt->pws;
  size_t ci = 0;  // running chunk index over all layers
  for (size_t k = 0; k < n; ++k) {
    const hc_layer *ly = bt->layers[k];
    const hc::ConvGeom &g = ly->geom;
    const Shapes sh = hc::layer_shapes(ly, B);
    const size_t npin = (size_t)B * g.G * 2 * c.L;
    // stream A: the layer's forward NTT (after the previous layer's last MAC, in stream order)
    HC_HIP(hc::launch_ntt_fwd(c.logn, sh.fe, ct_in[k], xhat, npin, c.consts, c.tw, sa));
    const size_t hw = (size_t)g.ho * g.wo;
    for (uint32_t i0 = 0; i0 < g.c_out; i0 += nch[k], ++ci) {
      const uint32_t nc = std::min(nch[k], g.c_out - i0);
      hc::ConvGeom gc = g;
      gc.c_out = nc;
      gc.O = nc * g.T;
      uint32_t *ybuf = (uint32_t *)((char *)bt->pws + xbytes + (ci % nbuf) * ybytes);
      hipEvent_t mac_done = bt->pev[2 * ci], inv_done = bt->pev[2 * ci + 1];
      if (ci >= nbuf) HC_HIP(hipStreamWaitEvent(sa, bt->pev[2 * (ci - nbuf) + 1], 0));  // buffer free again
      if (!hc::mac_offsets_fit(gc, sh.mac)) return fail(HC_EUNSUPPORTED, "layer too large for the MAC tile");
      HC_HIP(hc::launch_mac(gc, sh.mac, xhat, ly->d_w + (size_t)i0 * 64, ybuf, B, c.consts, c.tw, sa));
      HC_HIP(hipEventRecord(mac_done, sa));
      HC_HIP(hipStreamWaitEvent(sb, mac_done, 0));
      // inverse NTT + mask + extraction of the chunk, at most kMaxTab images per launch
      for (uint32_t b0 = 0; b0 < B; b0 += hc::kMaxTab) {
        const uint32_t nb = std::min<uint32_t>(hc::kMaxTab, B - b0);
        hc::OutPtrs out{};
        out.n = nb;
        for (uint32_t b = 0; b < nb; ++b) {
          const size_t bi = b0 + b;
          out.mask[b] = (uint64_t)(uintptr_t)(mask[k] + (bi * g.c_out + i0) * hw);
          out.c0[b] = (uint64_t)(uintptr_t)(c0[k] + (bi * g.c_out + i0) * c.L * hw);
          out.c1[b] = (uint64_t)(uintptr_t)(c1[k] + (bi * g.O + (size_t)i0 * g.T) * c.L * c.N);
        }
        const uint32_t *ysrc = ybuf + (size_t)b0 * gc.O * 2 * c.L * c.N;
        HC_HIP(hc::launch_intt_masked(gc, c.logn, sh.ie, sh.ipw, sh.mac.pre, ysrc, nullptr, nullptr, nullptr, nb,
                                      c.consts, c.tw, sb, &out));
      }
      HC_HIP(hipEventRecord(inv_done, sb));
    }
  }
  HC_HIP(hipEventRecord(ev_ea, sa));
  HC_HIP(hipEventRecord(ev_eb, sb));
  HC_HIP(hipStreamWaitEvent(st, ev_ea, 0));
  HC_HIP(hipStreamWaitEvent(st, ev_eb, 0));
  return HC_OK;
}

}  // extern "C"

// ------------------------------------------------------------- autotuner
namespace {

std::string tune_key(const hc_layer *ly, uint32_t B, const char *arch) {
  const hc_conv_shape &s = ly->shape;
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s N=%u L=%u B=%u %u-%u %ux%u f%u s%u", arch, ly->ctx->N, ly->ctx->L, B, s.c_in,
                s.c_out, s.h, s.w, s.f, s.stride);
  return buf;
}

// Mean milliseconds of `reps` launches of fn on stream st (after one warm-up).
template <class F>
hc_status time_it(F fn, hipStream_t st, int reps, float *ms) {
  hipEvent_t a, b;
  HC_HIP(hipEventCreate(&a));
  HC_HIP(hipEventCreate(&b));
  hipError_t e = fn();
  if (e == hipSuccess) e = hipEventRecord(a, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = fn();
  if (e == hipSuccess) e = hipEventRecord(b, st);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return hip_fail(e, "autotune timing");
  *ms /= reps;
  return HC_OK;
}

// (images, channels per thread; image, channel wave groups; loads in flight; LDS-staged;
//  inverse NTT stages in the MAC's epilogue)
const uint32_t kMacCand[][7] = {
    {1, 8, 1, 4, 2, 0, 0}, {1, 4, 1, 4, 2, 0, 0}, {2, 4, 1, 4, 2, 0, 0}, {4, 4, 1, 4, 2, 0, 0},
    {4, 2, 1, 4, 2, 0, 0}, {8, 2, 1, 4, 2, 0, 0}, {4, 4, 4, 2, 2, 0, 0}, {4, 8, 4, 2, 2, 0, 0},
    {2, 8, 4, 2, 2, 0, 0}, {4, 4, 2, 4, 2, 0, 0}, {2, 4, 4, 4, 2, 0, 0}, {1, 8, 2, 4, 2, 0, 0},
    {4, 8, 4, 2, 3, 0, 0}, {2, 8, 4, 2, 4, 0, 0}, {4, 4, 4, 2, 4, 0, 0}, {4, 4, 2, 4, 4, 0, 0},
    {1, 8, 2, 4, 4, 0, 0}, {2, 4, 4, 4, 4, 0, 0}, {1, 8, 1, 4, 4, 0, 0}, {4, 8, 4, 2, 2, 1, 0},
    {4, 8, 4, 2, 3, 1, 0}, {4, 8, 2, 2, 2, 1, 0}, {4, 8, 2, 2, 3, 1, 0}, {2, 8, 4, 2, 3, 1, 0},
    {4, 4, 4, 2, 3, 1, 0}, {2, 8, 2, 2, 3, 1, 0}, {4, 8, 4, 2, 2, 1, 5}, {4, 8, 2, 2, 2, 1, 5},
    {4, 8, 2, 2, 3, 1, 5}, {4, 8, 2, 2, 3, 2, 0}, {4, 8, 2, 2, 4, 2, 0}, {4, 8, 2, 2, 6, 2, 0},
    {4, 8, 4, 2, 3, 2, 0}, {4, 8, 4, 2, 4, 2, 0}, {2, 8, 4, 2, 4, 2, 0}, {4, 4, 4, 2, 4, 2, 0},
    {2, 8, 2, 2, 4, 2, 0}, {4, 4, 2, 2, 4, 2, 0}, {4, 8, 2, 2, 3, 2, 5}, {4, 8, 2, 2, 4, 2, 5},
    {4, 8, 4, 2, 4, 2, 5}, {4, 8, 2, 2, 3, 2, 6}, {4, 8, 2, 2, 4, 2, 6}, {4, 8, 4, 2, 3, 2, 6},
    {4, 8, 4, 2, 4, 2, 6}};

}  // namespace

extern "C" {

hc_status hc_batch_autotune(hc_batch *bt, const uint32_t *const *ct_in, const uint32_t *const *mask,
                            uint32_t *const *c0, uint32_t *const *c1, void *stream, const char *cache_path) {
  hc_status s = batch_check(bt, ct_in, mask, c0, c1);
  if (s != HC_OK) return s;
  DeviceGuard dg(bt->ctx->device);
  hipDeviceProp_t prop;
  HC_HIP(hipGetDeviceProperties(&prop, bt->ctx->device));
  std::string arch = prop.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  std::map<std::string, hc_tuning> cache;
  if (cache_path) {
    FILE *f = std::fopen(cache_path, "r");
    if (f) {
      char line[512];
      while (std::fgets(line, sizeof(line), f)) {
        char *bar = std::strchr(line, '|');
        if (!bar) continue;
        *bar = 0;
        hc_tuning t{};
        if (std::sscanf(bar + 1, "%u %u %u %u %u %u %u %u %u %u", &t.fwd_elog, &t.inv_elog, &t.mac_rows,
                        &t.mac_cols, &t.mac_row_groups, &t.mac_col_groups, &t.mac_depth, &t.mac_lds,
                        &t.inv_polys, &t.mac_pre) >= 6)
          cache[line] = t;
      }
      std::fclose(f);
    }
  }
  hipStream_t st = (hipStream_t)stream;
  const hc_ctx &c = *bt->ctx;
  const uint32_t B = bt->B;
  const int reps = 3;
  std::string appended;
  for (size_t k = 0; k < bt->layers.size(); ++k) {
    hc_layer *ly = const_cast<hc_layer *>(bt->layers[k]);
    const std::string key = tune_key(ly, B, arch.c_str());
    auto hit = cache.find(key);
    if (hit != cache.end()) {
      const hc_tuning &t = hit->second;
      if (hc::ntt_variant_ok(c.logn, t.fwd_elog) &&
          hc::intt_masked_ok(c.logn, t.inv_elog, t.inv_polys ? t.inv_polys : 1, t.mac_pre) &&
          hc::mac_variant_ok(hc::mac_of(t)) && hc::mac_offsets_fit(ly->geom, hc::mac_of(t))) {
        hc::layer_set_tuning(ly, B, t);
        continue;
      }
    }
    const hc::ConvGeom &g = ly->geom;
    uint32_t *xhat = (uint32_t *)((char *)bt->ws + bt->ws_off[k]);
    const size_t npin = (size_t)B * g.G * 2 * c.L;
    uint32_t *yhat = xhat + npin * c.N;
    hc_tuning best{};
    float best_ms = 1e30f;
    for (uint32_t e = 3; e <= 6; ++e) {
      if (!hc::ntt_variant_ok(c.logn, e)) continue;
      float ms;
      s = time_it([&] { return hc::launch_ntt_fwd(c.logn, e, ct_in[k], xhat, npin, c.consts, c.tw, st); }, st, reps,
                  &ms);
      if (s != HC_OK) return s;
      if (ms < best_ms) best_ms = ms, best.fwd_elog = e;
    }
    // MAC and inverse NTT are chosen together: with epilogue stages (pre) the
    // MAC does part of the inverse transform, so compare MAC + inverse NTT
    // totals of the best of each with and without them.
    float best_total = 1e30f;
    for (uint32_t pre : {0u, hc::kMacPre, hc::kMacC0}) {
      if (pre == hc::kMacPre && c.logn < 12) continue;
      if (pre == hc::kMacC0 && !hc::mac_c0_ok(g)) continue;
      float mac_ms = 1e30f, inv_ms = 1e30f;
      hc_tuning t = best;
      for (const auto &m : kMacCand) {
        const hc::MacShape shape{m[0], m[1], m[2], m[3], m[4], m[5], m[6]};
        if (shape.pre != pre || !hc::mac_variant_ok(shape) || !hc::mac_offsets_fit(g, shape)) continue;
        float ms;
        s = time_it([&] { return hc::launch_mac(g, shape, xhat, ly->d_w, yhat, B, c.consts, c.tw, st); }, st,
                    reps, &ms);
        if (s != HC_OK) return s;
        if (ms < mac_ms) {
          mac_ms = ms;
          t.mac_rows = m[0], t.mac_cols = m[1], t.mac_row_groups = m[2], t.mac_col_groups = m[3];
          t.mac_depth = m[4], t.mac_lds = m[5], t.mac_pre = m[6];
        }
      }
      if (mac_ms >= 1e30f) continue;
      for (uint32_t e = 3; e <= 6; ++e) {
        for (uint32_t npw = 1; npw <= 2; ++npw) {
          if (!hc::intt_masked_ok(c.logn, e, npw, pre)) continue;
          float ms;
          s = time_it([&] {
            return hc::launch_intt_masked(g, c.logn, e, npw, pre, yhat, mask[k], c0[k], c1[k], B, c.consts, c.tw,
                                          st);
          }, st, reps, &ms);
          if (s != HC_OK) return s;
          if (ms < inv_ms) inv_ms = ms, t.inv_elog = e, t.inv_polys = npw;
        }
      }
      if (mac_ms + inv_ms < best_total) best_total = mac_ms + inv_ms, best = t;
    }
    hc::layer_set_tuning(ly, B, best);
    char buf[128];
    std::snprintf(buf, sizeof(buf), "|%u %u %u %u %u %u %u %u %u %u\n", best.fwd_elog, best.inv_elog,
                  best.mac_rows, best.mac_cols, best.mac_row_groups, best.mac_col_groups, best.mac_depth,
                  best.mac_lds, best.inv_polys, best.mac_pre);
    appended += key + buf;
  }
  if (cache_path && !appended.empty()) {
    FILE *f = std::fopen(cache_path, "a");
    if (f) {
      std::fputs(appended.c_str(), f);
      std::fclose(f);
    }
  }
  if (bt->exec) {
    (void)hipGraphExecDestroy(bt->exec);
    bt->exec = nullptr;
  }
  return HC_OK;
}

hc_status hc_batch_get_mac_cap(const hc_batch *bt, uint32_t *cap) {
  if (!bt || !cap) return fail(HC_EINVAL, "null argument");
  *cap = bt->mac_cap;
  return HC_OK;
}

hc_status hc_batch_set_mac_cap(hc_batch *bt, uint32_t cap) {
  if (!bt) return fail(HC_EINVAL, "null argument");
  if (cap != 0 && cap < 8) return fail(HC_EINVAL, "a MAC grid cap is 0 or at least 8");
  bt->mac_cap = cap;
  return HC_OK;
}

hc_status hc_layer_get_tuning(const hc_layer *ly, uint32_t *B, hc_tuning *out) {
  if (!ly || !B || !out) return fail(HC_EINVAL, "null argument");
  if (ly->tune_last < 0) {
    *B = 0;
    *out = hc_tuning{};
  } else {
    *B = ly->tunes[ly->tune_last].B;
    *out = ly->tunes[ly->tune_last].t;
  }
  return HC_OK;
}

hc_status hc_layer_get_tuning_for(const hc_layer *ly, uint32_t B, hc_tuning *out) {
  if (!ly || !out) return fail(HC_EINVAL, "null argument");
  const hc_tuning *t = hc::layer_tuning_for(ly, B);
  *out = t ? *t : hc_tuning{};
  return t ? HC_OK : HC_ESTATE;
}

hc_status hc_layer_clear_tuning(hc_layer *ly) {
  if (!ly) return fail(HC_EINVAL, "null argument");
  for (auto &sl : ly->tunes) sl = hc_layer::TuneSlot{};
  ly->tune_last = -1;
  return HC_OK;
}

void hc_batch_destroy(hc_batch *bt) {
  if (!bt) return;
  DeviceGuard dg(bt->ctx->device);
  if (bt->pa) (void)hipStreamSynchronize(bt->pa);
  if (bt->pb) (void)hipStreamSynchronize(bt->pb);
  for (hipEvent_t ev : bt->pev) (void)hipEventDestroy(ev);
  if (bt->pa) (void)hipStreamDestroy(bt->pa);
  if (bt->pb) (void)hipStreamDestroy(bt->pb);
  if (bt->pws) (void)hipFree(bt->pws);
  if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
  for (int s = 0; s < kChains; ++s) {
    if (bt->side[s]) (void)hipStreamDestroy(bt->side[s]);
    if (bt->join[s]) (void)hipEventDestroy(bt->join[s]);
  }
  if (bt->fork) (void)hipEventDestroy(bt->fork);
  if (bt->ws) (void)hipFree(bt->ws);
  delete bt;
}

}  // extern "C"
