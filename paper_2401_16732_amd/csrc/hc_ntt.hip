// gfx950 kernels of the homomorphic convolution: forward NTT, full inverse NTT,
// weight encoding and the small helper kernels, with their launchers. The
// masked inverse NTT lives in hc_intt_masked.h, the multiply-accumulate in
// hc_mac.hip.
#include "hc_device.h"
#include "hc_intt_masked.h"

namespace hc {

// ---------------------------------------------------------------- forward NTT kernel
// One workgroup per polynomial of in/out [P][N] (limb = poly mod L). Input
// canonical; output canonical, in bit-reversed evaluation order.
// With a pointer table (tab.n > 0) polynomial `poly` is read from image
// poly / ppi at polynomial poly % ppi of that image's buffer instead.
template <int LOGN, int ELOG>
__global__ __launch_bounds__(1 << (LOGN - ELOG)) void k_ntt_fwd(const uint32_t *in, uint32_t *out, LimbConsts c,
                                                                 Twiddles tws, ImgPtrs tab, uint32_t ppi) {
  constexpr int N = 1 << LOGN, E = 1 << ELOG, NT = 1 << (LOGN - ELOG), NP = n_pass(LOGN, ELOG);
  __shared__ uint32_t lds[N + N / 32];
  const uint32_t tid = threadIdx.x;
  const size_t poly = blockIdx.x;
  const uint32_t l = (uint32_t)(poly % c.L);
  const uint32_t q = c.q[l];
  const uint2 *tw = tws.fwd + (size_t)l * N;
  // table entries are integers: cast to the global address space so the
  // loads are global rather than flat ones (which also count as LDS accesses)
  using gu32 = __attribute__((address_space(1))) const uint32_t;
  gu32 *src = tab.n ? (gu32 *)tab.p[poly / ppi] + (poly % ppi) * N : (gu32 *)in + poly * N;
  uint32_t v[E];
  {
    constexpr int LO = pass_lo_fwd(LOGN, ELOG, 0), EP = pass_bits(LOGN, ELOG, 0);
    gu32 *sb = src + gidx<LOGN, ELOG, LO, EP>(tid, 0);
#pragma unroll
    for (int u = 0; u < E; ++u) v[u] = __builtin_nontemporal_load(sb + gidx<LOGN, ELOG, LO, EP>(0, u));
  }
  FwdPasses<LOGN, ELOG, NP - 1>::run(v, lds, tid, tw, q);
  // the last pass (bits [0, EP)) leaves runs of 2^EP consecutive coefficients
  // in each thread: canonicalise and store them 16 bytes at a time
  constexpr int EPL = pass_bits(LOGN, ELOG, NP - 1);
  static_assert(pass_lo_fwd(LOGN, ELOG, NP - 1) == 0 && EPL >= 2, "last forward pass covers the low bits");
  uint32_t *dst = out + poly * N;
  const uint32_t q2 = 2 * q;
#pragma unroll
  for (int u = 0; u < E; u += 4) {
    uint4 t4;
    t4.x = csub(csub(v[u], q2), q);
    t4.y = csub(csub(v[u + 1], q2), q);
    t4.z = csub(csub(v[u + 2], q2), q);
    t4.w = csub(csub(v[u + 3], q2), q);
    *reinterpret_cast<uint4 *>(dst + gidx<LOGN, ELOG, 0, EPL>(tid, 0) + gidx<LOGN, ELOG, 0, EPL>(0, u)) = t4;
  }
  (void)NT;
}

// Full mode: [P][N] -> [P][N] canonical (in place allowed). SC: the last
// stage multiplies by N^-1 (false for inputs that carry it already).
template <int LOGN, int ELOG, bool SC>
__global__ __launch_bounds__(1 << (LOGN - ELOG)) __attribute__((amdgpu_waves_per_eu(ntt_min_waves(ELOG, 1)))) void k_intt_full(const uint32_t *in, uint32_t *out, LimbConsts c,
                                                                   Twiddles tws) {
  constexpr int N = 1 << LOGN, E = 1 << ELOG, NP = n_pass(LOGN, ELOG);
  __shared__ uint32_t lds[N + N / 32];
  const uint32_t tid = threadIdx.x;
  const size_t poly = blockIdx.x;
  const uint32_t l = (uint32_t)(poly % c.L);
  uint32_t v[1][E];
  const uint32_t *const src[1] = {in + poly * N};
  intt_core<LOGN, ELOG, 0, 1, 0, SC>(src, v, lds, tid, c, tws.inv + (size_t)l * N, l);
  constexpr int LO = pass_lo_inv(LOGN, ELOG, NP - 1), EP = pass_bits(LOGN, ELOG, NP - 1);
  uint32_t *dst = out + poly * N;
  const uint32_t q = c.q[l];
  uint32_t *db = dst + gidx<LOGN, ELOG, LO, EP>(tid, 0);
#pragma unroll
  for (int u = 0; u < E; ++u) db[gidx<LOGN, ELOG, LO, EP>(0, u)] = csub(v[0][u], q);
}

// Negacyclic product of each polynomial of in [P][N] (limb = poly mod L) with
// the polynomial whose NTT is row poly / mul_div of mul [..][L][N] at the same
// limb (row 0 for every polynomial when mul_div is 0; bit-reversed evaluation
// order, canonical, 16-byte aligned), in one pass over HBM: the forward transform,
// the pointwise product as the forward's last pass leaves its registers, one
// LDS exchange into the inverse transform's first-pass layout, the inverse
// transform, and a canonical store (in place allowed). PS > 0: only outputs
// below 2^(LOGN - PS) are wanted; the inverse prunes its top PS stages (as the
// masked inverse NTT does for c0) and the other outputs are not stored.
// ADD: the polynomials are ciphertexts [..][2][L][N], and c0 of ciphertext r
// gains Delta_l (centred addp[r][k] mod q_l) as it is stored (a plaintext
// addition, addp [..][N] in [0, t)).
template <int LOGN, int ELOG, int PS, bool ADD>
__global__ __launch_bounds__(1 << (LOGN - ELOG)) void k_ring_mul(const uint32_t *in, uint32_t *out,
                                                                  const uint32_t *mul, uint32_t mul_div,
                                                                  const uint32_t *addp, LimbConsts c,
                                                                  Twiddles tws) {
  constexpr int N = 1 << LOGN, E = 1 << ELOG, NP = n_pass(LOGN, ELOG);
  __shared__ uint32_t lds[N + N / 32];
  const uint32_t tid = threadIdx.x;
  const size_t poly = blockIdx.x;
  const uint32_t l = (uint32_t)(poly % c.L);
  const uint32_t q = c.q[l];
  using gu32 = __attribute__((address_space(1))) const uint32_t;
  uint32_t v[1][E];
  {
    constexpr int LO = pass_lo_fwd(LOGN, ELOG, 0), EP = pass_bits(LOGN, ELOG, 0);
    gu32 *sb = (gu32 *)in + poly * N + gidx<LOGN, ELOG, LO, EP>(tid, 0);
#pragma unroll
    for (int u = 0; u < E; ++u) v[0][u] = __builtin_nontemporal_load(sb + gidx<LOGN, ELOG, LO, EP>(0, u));
  }
  FwdPasses<LOGN, ELOG, NP - 1>::run(v[0], lds, tid, tws.fwd + (size_t)l * N, q);
  // the forward's last pass covers bits [0, EPL): 2^EPL consecutive words per group
  constexpr int EPL = pass_bits(LOGN, ELOG, NP - 1);
  static_assert(pass_lo_fwd(LOGN, ELOG, NP - 1) == 0 && EPL >= 2, "last forward pass covers the low bits");
  const uint32_t q2 = 2 * q;
  const size_t mrow = mul_div ? poly / mul_div : 0;
  const uint32_t *ml = mul + (mrow * c.L + l) * N + gidx<LOGN, ELOG, 0, EPL>(tid, 0);
#pragma unroll
  for (int u = 0; u < E; u += 4) {
    const uint4 s4 = *reinterpret_cast<const uint4 *>(ml + gidx<LOGN, ELOG, 0, EPL>(0, u));
    const uint32_t sv[4] = {s4.x, s4.y, s4.z, s4.w};
#pragma unroll
    for (int j = 0; j < 4; ++j)
      v[0][u + j] = reduce64((uint64_t)csub(csub(v[0][u + j], q2), q) * sv[j], q, c.r2[l], c.r2_p[l], c.one_p[l]);
  }
  // each thread writes back the LDS words its last forward pass read, so the
  // exchange needs only the barrier before the reads
  regs_to_lds<LOGN, ELOG, 0, EPL>(v[0], lds, tid);
  __syncthreads();
  lds_to_regs<LOGN, ELOG, 0, pass_bits(LOGN, ELOG, 0)>(v[0], lds, tid);
  const uint2 *itw = tws.inv + (size_t)l * N;
  if constexpr (ELOG <= 4) {
    const EarlyTws<LOGN, ELOG, 0> t(itw, tid);
    intt_passes<LOGN, ELOG, PS, 1, 0>(v, lds, tid, c, t, l);
  } else {
    intt_passes<LOGN, ELOG, PS, 1, 0>(v, lds, tid, c, MemTws<LOGN, ELOG, 0>{itw, tid}, l);
  }
  constexpr int LO = pass_lo_inv(LOGN, ELOG, NP - 1), EP = pass_bits(LOGN, ELOG, NP - 1);
  const uint32_t base = gidx<LOGN, ELOG, LO, EP>(tid, 0);
  uint32_t *db = out + poly * N + base;
  if constexpr (ADD) {
    if (((poly / c.L) & 1) == 0) {  // c0 of its ciphertext
      const uint32_t *ap = addp + (poly / (2 * c.L)) * N + base;
      const uint32_t half = c.t / 2;
#pragma unroll
      for (int u = 0; u < E; ++u) {
        const uint32_t j = gidx<LOGN, ELOG, LO, EP>(0, u);
        const uint32_t m = ap[j];
        // Delta_l (centred m mod q_l): m <= t/2 is m itself, else m - t + q (t < 2 q_l)
        const uint32_t mc = m > half ? m - c.t + q : m;
        db[j] = csub(csub(v[0][u], q) + csub(shoup_lazy(mc, c.delta[l], c.delta_p[l], q), q), q);
      }
      return;
    }
  }
#pragma unroll
  for (int u = 0; u < E; ++u) {
    const uint32_t j = gidx<LOGN, ELOG, LO, EP>(0, u);
    if (PS == 0 || base + j < (uint32_t)(N >> PS)) db[j] = csub(v[0][u], q);
  }
}

// ---------------------------------------------------------------- weight encoding
// What[i][gw][l][idx] = sign * f[i][j][ky][kx] mod q_l with x^(-e) = sign x^idx,
// e = o_j + ky w' + kx (x^0 = 1; x^(-e) = -x^(N-e) for e > 0). The e values of
// one (i, gw) are pairwise distinct, so every slot is written at most once.
__global__ void k_weight_scatter(const int8_t *__restrict__ f, uint32_t *__restrict__ Wt, ConvGeom g,
                                 LimbConsts c) {
  const size_t ff = (size_t)g.f * g.f;
  const size_t total = (size_t)g.c_out * g.c_in * ff;
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  const uint32_t tap = (uint32_t)(id % ff);
  const uint32_t j = (uint32_t)((id / ff) % g.c_in);
  const uint32_t i = (uint32_t)(id / (ff * g.c_in));
  const uint32_t ky = tap / g.f, kx = tap % g.f;
  const uint32_t gw = g.tiled ? j : j / g.cn;
  const uint32_t oj = g.tiled ? 0u : (j % g.cn) * g.F;
  const uint32_t e = oj + ky * g.w_pad + kx;
  const uint32_t idx = e == 0 ? 0u : g.N - e;
  const bool neg = e != 0;
  const int32_t val = f[id];
  for (uint32_t l = 0; l < g.L; ++l) {
    const uint32_t q = c.q[l];
    int32_t sv = neg ? -val : val;
    const uint32_t res = sv >= 0 ? (uint32_t)sv : q - (uint32_t)(-sv);
    Wt[(((size_t)i * g.G_w + gw) * g.L + l) * g.N + idx] = res;
  }
}

// [c][gw][l][N] -> [l][kb][gw][c][64], 16 bytes per thread: both sides move
// whole 256-byte runs.
__global__ __launch_bounds__(256) void k_weight_block(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                      uint32_t c_out, uint32_t G_w, uint32_t L, uint32_t N,
                                                      size_t n4) {
  const uint32_t nkb = N / 64;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x) {
    const uint32_t j4 = (uint32_t)(i & 15u);
    size_t r = i >> 4;
    const uint32_t ch = (uint32_t)(r % c_out);
    r /= c_out;
    const uint32_t gw = (uint32_t)(r % G_w);
    r /= G_w;
    const uint32_t kb = (uint32_t)(r % nkb);
    const uint32_t l = (uint32_t)(r / nkb);
    dst[i] = src[((((size_t)ch * G_w + gw) * L + l) * N + (size_t)kb * 64) / 4 + j4];
  }
}

__global__ void k_fill_zero(uint32_t *p, size_t n) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = id; k < n; k += stride) p[k] = 0u;
}

// ---------------------------------------------------------------- unfused mask + extract
// c0_ext[b][i][l][oy][ox] = ct_out[b][(i,tau)][0][l][e] + Delta_l (r_c mod q_l) mod q_l
__global__ void k_mask_extract(const uint32_t *__restrict__ ct, const uint32_t *__restrict__ mask,
                               uint32_t *__restrict__ c0_ext, ConvGeom g, uint32_t B, LimbConsts c) {
  const size_t total = (size_t)B * g.c_out * g.ho * g.wo;
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  const uint32_t ox = (uint32_t)(id % g.wo);
  const uint32_t oy = (uint32_t)((id / g.wo) % g.ho);
  const uint32_t i = (uint32_t)((id / ((size_t)g.wo * g.ho)) % g.c_out);
  const size_t b = id / ((size_t)g.wo * g.ho * g.c_out);
  const uint32_t Y = g.s * oy;
  const uint32_t tau = Y / g.r_o;
  const uint32_t e = (Y - tau * g.r_o) * g.w_pad + g.s * ox;
  const uint32_t o = i * g.T + tau;
  const uint32_t r = mask[id];
  const uint32_t t = c.t, half = c.t / 2;
  for (uint32_t l = 0; l < g.L; ++l) {
    const uint32_t q = c.q[l];
    const uint32_t rc = r > half ? r - t + q : r;
    const uint32_t add = csub(shoup_lazy(rc, c.delta[l], c.delta_p[l], q), q);
    const uint32_t y = ct[(((b * g.O + o) * 2 + 0) * g.L + l) * (size_t)g.N + e];
    c0_ext[((b * g.c_out + i) * g.L + l) * (size_t)g.ho * g.wo + (size_t)oy * g.wo + ox] = csub(y + add, q);
  }
}

// c1_out[b][o][l][:] = ct[b][o][1][l][:], 16-byte copies.
__global__ void k_copy_c1(const uint4 *__restrict__ ct, uint4 *__restrict__ c1, size_t n_ct, size_t ln4) {
  const size_t total = n_ct * ln4;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < total; id += stride) {
    const size_t ctn = id / ln4, k = id % ln4;
    c1[id] = ct[(2 * ctn + 1) * ln4 + k];
  }
}

// c[j] = a[j] * b[j] mod q over [P][N] (both operands variable).
__global__ void k_pointwise_mul(const uint32_t *__restrict__ a, const uint32_t *__restrict__ b,
                                uint32_t *__restrict__ cc, size_t total, uint32_t N, LimbConsts c) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < total; id += stride) {
    const uint32_t l = (uint32_t)((id / N) % c.L);
    cc[id] = reduce64((uint64_t)a[id] * b[id], c.q[l], c.r2[l], c.r2_p[l], c.one_p[l]);
  }
}

// Count of words that are not canonical residues (word >= q_l of its limb) in
// polynomials laid out [..][L][N]: one atomic add per wave.
__global__ void k_count_noncanonical(const uint32_t *__restrict__ p, size_t total, uint32_t N, LimbConsts c,
                                     unsigned long long *count) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  uint32_t bad = 0;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < total; id += stride) {
    const uint32_t l = (uint32_t)((id / N) % c.L);
    bad += p[id] >= c.q[l] ? 1u : 0u;
  }
  // wave sum, then one vector atomic from lane 0
  for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off);
  if ((threadIdx.x & 63u) == 0 && bad) atomicAdd(count, (unsigned long long)bad);
}

// ---------------------------------------------------------------- launchers
template <int LOGN, int ELOG>
static hipError_t fwd_t(const uint32_t *in, uint32_t *out, size_t np, const LimbConsts &c, const Twiddles &tw,
                        const ImgPtrs &tab, uint32_t ppi, hipStream_t st) {
  if (np == 0) return hipSuccess;
  hipLaunchKernelGGL((k_ntt_fwd<LOGN, ELOG>), dim3((uint32_t)np), dim3(1 << (LOGN - ELOG)), 0, st, in, out, c, tw,
                     tab, ppi);
  return hipGetLastError();
}
template <int LOGN, int ELOG, int PS, bool ADD>
static hipError_t ring_mul_ps(const uint32_t *in, uint32_t *out, size_t np, const uint32_t *mul, uint32_t mul_div,
                              const uint32_t *addp, const LimbConsts &c, const Twiddles &tw, hipStream_t st) {
  hipLaunchKernelGGL((k_ring_mul<LOGN, ELOG, PS, ADD>), dim3((uint32_t)np), dim3(1 << (LOGN - ELOG)), 0, st, in, out,
                     mul, mul_div, addp, c, tw);
  return hipGetLastError();
}
// Pruning fewer stages than allowed is exact: the largest instantiated count
// not above ps (pruned forms exist for ELOG 4, the default shape). The
// plaintext-adding form is unpruned.
template <int LOGN, int ELOG>
static hipError_t ring_mul_t(const uint32_t *in, uint32_t *out, size_t np, const uint32_t *mul, uint32_t mul_div,
                             uint32_t ps, const uint32_t *addp, const LimbConsts &c, const Twiddles &tw,
                             hipStream_t st) {
  if (np == 0) return hipSuccess;
  if (addp) return ring_mul_ps<LOGN, ELOG, 0, true>(in, out, np, mul, mul_div, addp, c, tw, st);
  if constexpr (ELOG == 4) {
    if (ps >= 7) return ring_mul_ps<LOGN, ELOG, 7, false>(in, out, np, mul, mul_div, addp, c, tw, st);
    if (ps >= 5) return ring_mul_ps<LOGN, ELOG, 5, false>(in, out, np, mul, mul_div, addp, c, tw, st);
    if (ps >= 3) return ring_mul_ps<LOGN, ELOG, 3, false>(in, out, np, mul, mul_div, addp, c, tw, st);
  }
  return ring_mul_ps<LOGN, ELOG, 0, false>(in, out, np, mul, mul_div, addp, c, tw, st);
}
template <int LOGN, int ELOG>
static hipError_t inv_t(const uint32_t *in, uint32_t *out, size_t np, const LimbConsts &c, const Twiddles &tw,
                        hipStream_t st, bool scale) {
  if (np == 0) return hipSuccess;
  if (scale)
    hipLaunchKernelGGL((k_intt_full<LOGN, ELOG, true>), dim3((uint32_t)np), dim3(1 << (LOGN - ELOG)), 0, st, in,
                       out, c, tw);
  else
    hipLaunchKernelGGL((k_intt_full<LOGN, ELOG, false>), dim3((uint32_t)np), dim3(1 << (LOGN - ELOG)), 0, st, in,
                       out, c, tw);
  return hipGetLastError();
}
// (LOGN, ELOG) instances: 2^(LOGN - ELOG) threads per polynomial.
#define HC_NTT_CASE(L, E, FN, ...) \
  if (logn == L && elog == E) return FN<L, E>(__VA_ARGS__);
#define HC_NTT_DISPATCH(FN, ...)                                                             \
  HC_NTT_CASE(10, 3, FN, __VA_ARGS__) HC_NTT_CASE(10, 4, FN, __VA_ARGS__)                    \
  HC_NTT_CASE(11, 3, FN, __VA_ARGS__) HC_NTT_CASE(11, 4, FN, __VA_ARGS__)                    \
  HC_NTT_CASE(12, 3, FN, __VA_ARGS__) HC_NTT_CASE(12, 4, FN, __VA_ARGS__)                    \
  HC_NTT_CASE(12, 5, FN, __VA_ARGS__) HC_NTT_CASE(13, 3, FN, __VA_ARGS__)                    \
  HC_NTT_CASE(13, 4, FN, __VA_ARGS__) HC_NTT_CASE(13, 5, FN, __VA_ARGS__)                    \
  HC_NTT_CASE(14, 4, FN, __VA_ARGS__) HC_NTT_CASE(14, 5, FN, __VA_ARGS__)                    \
  return hipErrorInvalidValue;

bool ntt_variant_ok(uint32_t logn, uint32_t elog) {
  switch (logn) {
    case 10: case 11: return elog == 3 || elog == 4;
    case 12: case 13: return elog >= 3 && elog <= 5;
    case 14: return elog == 4 || elog == 5;
  }
  return false;
}

hipError_t launch_ntt_fwd(uint32_t logn, uint32_t elog, const uint32_t *in, uint32_t *out, size_t np,
                          const LimbConsts &c, const Twiddles &tw, hipStream_t st, const ImgPtrs *tab,
                          uint32_t ppi) {
  ImgPtrs none{};
  if (tab && (tab->n == 0 || tab->n > kMaxTab || ppi == 0 || np != (size_t)tab->n * ppi)) return hipErrorInvalidValue;
  const ImgPtrs &t = tab ? *tab : none;
  HC_NTT_DISPATCH(fwd_t, in, out, np, c, tw, t, ppi, st)
}
hipError_t launch_ring_mul(uint32_t logn, uint32_t elog, const uint32_t *in, uint32_t *out, size_t np,
                           const uint32_t *mul, uint32_t mul_div, const LimbConsts &c, const Twiddles &tw,
                           hipStream_t st, uint32_t keep_bits, const uint32_t *addp) {
  if (mul_div && mul_div % c.L) return hipErrorInvalidValue;
  if (addp && np % (2 * c.L)) return hipErrorInvalidValue;  // whole ciphertexts
  const uint32_t ps = keep_bits >= logn ? 0 : logn - keep_bits;
  HC_NTT_DISPATCH(ring_mul_t, in, out, np, mul, mul_div, ps, addp, c, tw, st)
}
hipError_t launch_intt_full(uint32_t logn, uint32_t elog, const uint32_t *in, uint32_t *out, size_t np,
                            const LimbConsts &c, const Twiddles &tw, hipStream_t st, bool scale) {
  HC_NTT_DISPATCH(inv_t, in, out, np, c, tw, st, scale)
}

// p [..][L][N] *= N^-1 mod q_l, canonical out (the convolution's resident
// weights, so that the inverse NTT of its sums needs no final scaling).
__global__ __launch_bounds__(256) void k_scale_ninv(uint32_t *p, size_t n, uint32_t N, LimbConsts c) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const uint32_t l = (uint32_t)((i / N) % c.L);
    const uint32_t q = c.q[l];
    p[i] = csub(shoup_lazy(p[i], c.ninv[l], c.ninv_p[l], q), q);
  }
}
hipError_t launch_scale_ninv(uint32_t *p, size_t n, uint32_t N, const LimbConsts &c, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_scale_ninv, dim3((uint32_t)blocks), dim3(256), 0, st, p, n, N, c);
  return hipGetLastError();
}

bool intt_masked_ok(uint32_t logn, uint32_t elog, uint32_t npw, uint32_t pre) {
  return ntt_variant_ok(logn, elog) && (npw == 1 || (npw == 2 && elog <= 4)) &&
         (pre == 0 || pre == kMacC0 || (pre == kMacPre && logn >= 12));
}

// c0 after a MAC with pre = kMacC0: output (b, i, l, oy, ox) (ox fastest) is
// the sum of the splits' partial sums at its coefficient e = s w_pad oy + s ox,
// Yhat[b][i][0][l][64 sp + 32 (e mod 2) + e / 2], plus Delta_l (r mod q_l), r
// the mask's centred value - the masked inverse NTT's extraction, on the same
// values.
__global__ __launch_bounds__(256) void k_c0_finish(const uint32_t *__restrict__ y, const uint32_t *__restrict__ mask,
                                                   uint32_t *__restrict__ c0_ext, ConvGeom g, uint32_t B,
                                                   LimbConsts c, uint32_t ns, OutPtrs out) {
  const size_t hw = (size_t)g.ho * g.wo;
  const size_t total = (size_t)B * g.c_out * g.L * hw;
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  const uint32_t ox = (uint32_t)(id % g.wo);
  size_t r = id / g.wo;
  const uint32_t oy = (uint32_t)(r % g.ho);
  r /= g.ho;
  const uint32_t l = (uint32_t)(r % g.L);
  r /= g.L;
  const uint32_t i = (uint32_t)(r % g.c_out);
  const size_t b = r / g.c_out;
  const uint32_t q = c.q[l], q2 = 2 * q;
  const uint32_t e = g.s * g.w_pad * oy + g.s * ox;
  const uint32_t *src = y + ((b * g.O + i) * 2 * g.L + l) * (size_t)g.N + (e & 1u) * 32u + (e >> 1);
  uint32_t sum = 0;
  for (uint32_t s = 0; s < ns; ++s) sum = csub(sum + src[s * 64], q2);
  const size_t pix = (size_t)oy * g.wo + ox;
  const uint32_t rv = out.n ? ((const uint32_t *)out.mask[b])[i * hw + pix] : mask[(b * g.c_out + i) * hw + pix];
  const uint32_t t = c.t, half = c.t / 2;
  const uint32_t rc = rv > half ? rv - t + q : rv;  // centred lift of r, taken mod q
  const uint32_t add = csub(shoup_lazy(rc, c.delta[l], c.delta_p[l], q), q);
  const uint32_t v = csub(csub(sum, q) + add, q);
  if (out.n)
    ((uint32_t *)out.c0[b])[((size_t)i * g.L + l) * hw + pix] = v;
  else
    c0_ext[((b * g.c_out + i) * g.L + l) * hw + pix] = v;
}

hipError_t launch_intt_masked(const ConvGeom &g, uint32_t logn, uint32_t elog, uint32_t npw, uint32_t pre,
                              const uint32_t *y, const uint32_t *m, uint32_t *c0, uint32_t *c1, uint32_t B,
                              const LimbConsts &c, const Twiddles &tw, hipStream_t st, const OutPtrs *tab) {
  OutPtrs none{};
  if (tab && (tab->n != B || B > kMaxTab)) return hipErrorInvalidValue;
  if (!intt_masked_ok(logn, elog, npw, pre)) return hipErrorInvalidValue;
  const OutPtrs &t = tab ? *tab : none;
  // after a MAC that finished c0's transform: c1 only, then c0's finish
  const bool c1_only = pre == kMacC0;
  if (c1_only && !mac_c0_ok(g)) return hipErrorInvalidValue;
  const uint32_t ipre = c1_only ? 0u : pre;
  hipError_t e = hipErrorInvalidValue;
  switch (logn) {
    case 10: e = intt_masked_logn<10>(g, elog, npw, ipre, y, m, c0, c1, B, c, tw, t, st, c1_only); break;
    case 11: e = intt_masked_logn<11>(g, elog, npw, ipre, y, m, c0, c1, B, c, tw, t, st, c1_only); break;
    case 12: e = intt_masked_logn<12>(g, elog, npw, ipre, y, m, c0, c1, B, c, tw, t, st, c1_only); break;
    case 13: e = intt_masked_logn<13>(g, elog, npw, ipre, y, m, c0, c1, B, c, tw, t, st, c1_only); break;
    case 14: e = intt_masked_logn<14>(g, elog, npw, ipre, y, m, c0, c1, B, c, tw, t, st, c1_only); break;
  }
  if (e != hipSuccess || !c1_only) return e;
  const size_t total = (size_t)B * g.c_out * g.L * g.ho * g.wo;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_c0_finish, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, st, y, m, c0, g, B, c,
                     c0_splits(g), t);
  return hipGetLastError();
}

hipError_t launch_weight_scatter(const ConvGeom &g, const int8_t *f, uint32_t *w, const LimbConsts &c,
                                 hipStream_t st) {
  const size_t total = (size_t)g.c_out * g.c_in * g.f * g.f;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_weight_scatter, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, st, f, w, g, c);
  return hipGetLastError();
}
hipError_t launch_weight_block(const uint32_t *src, uint32_t *dst, uint32_t c_out, uint32_t G_w, uint32_t L,
                               uint32_t N, hipStream_t st) {
  const size_t n4 = (size_t)c_out * G_w * L * N / 4;
  if (n4 == 0) return hipSuccess;
  if (N % 64 != 0) return hipErrorInvalidValue;
  const size_t blocks = std::min<size_t>((n4 + 255) / 256, 65536);
  hipLaunchKernelGGL(k_weight_block, dim3((uint32_t)blocks), dim3(256), 0, st, (const uint4 *)src, (uint4 *)dst,
                     c_out, G_w, L, N, n4);
  return hipGetLastError();
}
hipError_t launch_fill_zero(uint32_t *p, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_zero, dim3((uint32_t)blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}
hipError_t launch_mask_extract(const ConvGeom &g, const uint32_t *ct, const uint32_t *mask, uint32_t *c0,
                               uint32_t *c1, uint32_t B, const LimbConsts &c, hipStream_t st) {
  const size_t total = (size_t)B * g.c_out * g.ho * g.wo;
  if (total) {
    hipLaunchKernelGGL(k_mask_extract, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, st, ct, mask, c0, g, B,
                       c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const size_t n_ct = (size_t)B * g.O, ln4 = (size_t)g.L * g.N / 4;
  if (n_ct == 0) return hipSuccess;
  size_t blocks = (n_ct * ln4 + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_copy_c1, dim3((uint32_t)blocks), dim3(256), 0, st, (const uint4 *)ct, (uint4 *)c1, n_ct, ln4);
  return hipGetLastError();
}
hipError_t launch_count_noncanonical(const uint32_t *p, size_t np, uint32_t N, const LimbConsts &k,
                                     unsigned long long *count, hipStream_t st) {
  const size_t total = np * N;
  if (total == 0) return hipSuccess;
  size_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_count_noncanonical, dim3((uint32_t)blocks), dim3(256), 0, st, p, total, N, k, count);
  return hipGetLastError();
}
hipError_t launch_pointwise_mul(const uint32_t *a, const uint32_t *b, uint32_t *cc, size_t np, uint32_t N,
                                const LimbConsts &k, hipStream_t st) {
  const size_t total = np * N;
  if (total == 0) return hipSuccess;
  size_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_pointwise_mul, dim3((uint32_t)blocks), dim3(256), 0, st, a, b, cc, total, N, k);
  return hipGetLastError();
}

}  // namespace hc
