// gfx950 kernels of the homomorphic convolution (Flash, arXiv 2401.16732,
// Algorithm 1 evaluated as y_i = sum_g c_g * W_{i,g} in R_q through the NTT).
//
// All arithmetic is exact 32-bit modular arithmetic on the vector ALUs:
//  * Shoup multiplication by precomputed constants (twiddles, N^-1, Delta),
//  * Harvey's lazy butterflies (forward values kept in [0, 4q), inverse in
//    [0, 2q); q < 2^30 so 4q < 2^32),
//  * the multiply-accumulate over input ciphertexts in 64-bit accumulators
//    (v_mad_u64_u32), folded every few terms and reduced once per output: the
//    GPU form of the paper's lazy reduction (Employing Lazy Reduction in
//    Convolution).
// No MFMA: nothing here is a floating-point contraction.
#include <hip/hip_runtime.h>
#include <cstdint>
#include "hc_internal.h"

namespace hc {

// Third word of a gfx9-family raw buffer descriptor (32-bit data, no swizzle,
// no stride), as used for gfx908/90a/94x/950.
constexpr uint32_t kBufferWord3 = 0x00020000u;

// ---------------------------------------------------------------- arithmetic
__device__ __forceinline__ uint32_t shoup_lazy(uint32_t a, uint32_t w, uint32_t wp, uint32_t q) {
  uint32_t Q = __umulhi(a, wp);
  return a * w - Q * q;  // in [0, 2q) for any a < 2^32
}
__device__ __forceinline__ uint32_t csub(uint32_t a, uint32_t m) { return a >= m ? a - m : a; }

// acc < 2^64 -> acc mod q, q < 2^30.
__device__ __forceinline__ uint32_t reduce64(uint64_t acc, uint32_t q, uint32_t r2, uint32_t r2p, uint32_t onep) {
  uint32_t hi = (uint32_t)(acc >> 32), lo = (uint32_t)acc;
  uint32_t r = shoup_lazy(hi, r2, r2p, q) + shoup_lazy(lo, 1u, onep, q);  // [0, 4q)
  r = csub(r, 2 * q);
  return csub(r, q);
}

// ---------------------------------------------------------------- NTT shape
// A polynomial of N = 2^LOGN coefficients is transformed by one workgroup of
// 2^(LOGN - ELOG) threads; each thread holds E = 2^ELOG coefficients in
// registers. The LOGN butterfly stages are split into passes of at most ELOG
// consecutive index bits; within a pass every butterfly's pair lies in one
// thread, and passes exchange data through LDS.
__host__ __device__ constexpr int n_pass(int logn, int elog) { return (logn + elog - 1) / elog; }
__host__ __device__ constexpr int pass_bits(int logn, int elog, int k) {
  return logn / n_pass(logn, elog) + (k < logn % n_pass(logn, elog) ? 1 : 0);
}
// Forward passes walk the index bits from the top down (stage s touches bit
// LOGN-1-s); inverse passes walk them from the bottom up.
__host__ __device__ constexpr int pass_lo_fwd(int logn, int elog, int k) {
  int lo = logn;
  for (int i = 0; i <= k; ++i) lo -= pass_bits(logn, elog, i);
  return lo;
}
__host__ __device__ constexpr int pass_lo_inv(int logn, int elog, int k) {
  int lo = 0;
  for (int i = 0; i < k; ++i) lo += pass_bits(logn, elog, i);
  return lo;
}

// Coefficient index held in register u during a pass over bits [LO, LO+EP).
// u = (grp << EP) | w: w walks the pass bits; the thread id and grp fill the
// remaining bit positions, thread id lowest (so a pass with LO >= thread bits
// reads consecutive words across the wave).
template <int LOGN, int ELOG, int LO, int EP>
__device__ __forceinline__ uint32_t gidx(uint32_t tid, int u) {
  constexpr int TB = LOGN - ELOG;
  const uint32_t w = (uint32_t)u & ((1u << EP) - 1u);
  const uint32_t grp = (uint32_t)u >> EP;
  const uint32_t v = tid | (grp << TB);
  return (v & ((1u << LO) - 1u)) | (w << LO) | ((v >> LO) << (LO + EP));
}
// LDS word address: one pad word per 32 keeps strided passes off a single bank.
// gidx(tid, u) is the OR of a thread part gidx(tid, 0) and a register part
// gidx(0, u) over disjoint bits, so lpad(gidx(tid, u)) = lpad(gidx(tid, 0)) +
// lpad(gidx(0, u)): one base per thread and compile-time offsets per register.
__host__ __device__ constexpr uint32_t lpad(uint32_t j) { return j + (j >> 5); }

// Twiddles of stage bit b (s = LOGN - 1 - b) read at index 2^s + (j >> (b+1)).
// In a pass over bits [LO, LO + EP) with LO >= 6 the thread's share of j above
// bit b comes from tid >> LO, which is the same for all 64 lanes of a wave:
// the base is then wave-uniform and read through the constant address space,
// so the compiler can fetch those twiddles with scalar loads instead of one
// vector load per lane.
using const_u64 = __attribute__((address_space(4))) const uint64_t;
template <int LOGN, int ELOG, int LO, int EP>
struct StageTw {
  static constexpr bool kUniform = LO >= 6;
  const uint2 *vec;
  const_u64 *uni;  // the same {w, w'} pairs as 64-bit words
  __device__ __forceinline__ StageTw(const uint2 *tw, uint32_t tid, int b) {
    const int s = LOGN - 1 - b;
    if constexpr (kUniform) {
      const uint32_t hi = __builtin_amdgcn_readfirstlane(tid >> LO);
      uni = (const_u64 *)(tw + (1u << s) + (((size_t)hi << (LO + EP)) >> (b + 1)));
      vec = nullptr;
    } else {
      vec = tw + (1u << s) + (gidx<LOGN, ELOG, LO, EP>(tid, 0) >> (b + 1));
      uni = nullptr;
    }
  }
  // twiddle of register slot u (the register part of j is gidx(0, u))
  __device__ __forceinline__ uint2 operator()(int u, int b) const {
    const uint32_t k = gidx<LOGN, ELOG, LO, EP>(0, u) >> (b + 1);
    if constexpr (kUniform) {
      const uint64_t t = uni[k];
      return make_uint2((uint32_t)t, (uint32_t)(t >> 32));
    } else {
      return vec[k];
    }
  }
};

// Forward (Cooley-Tukey, natural -> bit-reversed) stages of one pass.
// Stage s works on pairs (j, j + 2^(LOGN-1-s)) with twiddle psi^brv(2^s + j >> (LOGN - s)).
template <int LOGN, int ELOG, int LO, int EP>
__device__ __forceinline__ void fwd_pass(uint32_t (&v)[1 << ELOG], uint32_t tid, const uint2 *__restrict__ tw,
                                         uint32_t q) {
  constexpr int E = 1 << ELOG;
  const uint32_t q2 = 2 * q;
#pragma unroll
  for (int bb = EP - 1; bb >= 0; --bb) {
    const int b = LO + bb;
    const int s = LOGN - 1 - b;
    // twiddle index 2^s + (j >> (b + 1)), split into thread and register parts
    const StageTw<LOGN, ELOG, LO, EP> tws(tw, tid, b);
    (void)s;
#pragma unroll
    for (int u = 0; u < E; ++u) {
      if (u & (1 << bb)) continue;
      const int u2 = u | (1 << bb);
      const uint2 w = tws(u, b);
      uint32_t X = v[u], Y = v[u2];
      X = csub(X, q2);
      const uint32_t T = shoup_lazy(Y, w.x, w.y, q);
      v[u] = X + T;
      v[u2] = X - T + q2;
    }
  }
}

// Inverse (Gentleman-Sande, bit-reversed -> natural) stages of one pass; the
// last stage (s = 0) also multiplies by N^-1.
// Pruning: when only outputs below 2^(LOGN - PS) are wanted, every stage on a
// bit b >= LOGN - PS feeds wanted outputs from its lower (sum) half only - all
// wanted indices have those bits clear - so the difference half, with its
// twiddle multiply, is skipped there. PS = 0 computes the full transform. PS
// is a compile-time constant, so no stage carries a run-time branch.
// M polynomials of one limb go through the stages together (v[m]): each
// twiddle is loaded once for all of them.
template <int LOGN, int ELOG, int LO, int EP, int PS, int M>
__device__ __forceinline__ void inv_pass(uint32_t (&v)[M][1 << ELOG], uint32_t tid, const uint2 *__restrict__ tw,
                                         uint32_t q, uint32_t ninv, uint32_t ninvp, uint32_t ninvw,
                                         uint32_t ninvwp) {
  constexpr int E = 1 << ELOG;
  const uint32_t q2 = 2 * q;
#pragma unroll
  for (int bb = 0; bb < EP; ++bb) {
    const int b = LO + bb;
    const int s = LOGN - 1 - b;
    const bool sum_only = b >= LOGN - PS;
    const StageTw<LOGN, ELOG, LO, EP> tws(tw, tid, b);
#pragma unroll
    for (int u = 0; u < E; ++u) {
      if (u & (1 << bb)) continue;
      const int u2 = u | (1 << bb);
      if (sum_only) {
#pragma unroll
        for (int m = 0; m < M; ++m)
          v[m][u] = s == 0 ? shoup_lazy(v[m][u] + v[m][u2], ninv, ninvp, q) : csub(v[m][u] + v[m][u2], q2);
      } else if (s == 0) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
          const uint32_t X = v[m][u], Y = v[m][u2];
          v[m][u] = shoup_lazy(X + Y, ninv, ninvp, q);
          v[m][u2] = shoup_lazy(X - Y + q2, ninvw, ninvwp, q);
        }
      } else {
        const uint2 w = tws(u, b);
#pragma unroll
        for (int m = 0; m < M; ++m) {
          const uint32_t X = v[m][u], Y = v[m][u2];
          v[m][u] = csub(X + Y, q2);
          v[m][u2] = shoup_lazy(X - Y + q2, w.x, w.y, q);
        }
      }
    }
  }
}

template <int LOGN, int ELOG, int LO, int EP>
__device__ __forceinline__ void regs_to_lds(const uint32_t (&v)[1 << ELOG], uint32_t *lds, uint32_t tid) {
  uint32_t *p = lds + lpad(gidx<LOGN, ELOG, LO, EP>(tid, 0));
#pragma unroll
  for (int u = 0; u < (1 << ELOG); ++u) p[lpad(gidx<LOGN, ELOG, LO, EP>(0, u))] = v[u];
}
template <int LOGN, int ELOG, int LO, int EP>
__device__ __forceinline__ void lds_to_regs(uint32_t (&v)[1 << ELOG], const uint32_t *lds, uint32_t tid) {
  const uint32_t *p = lds + lpad(gidx<LOGN, ELOG, LO, EP>(tid, 0));
#pragma unroll
  for (int u = 0; u < (1 << ELOG); ++u) v[u] = p[lpad(gidx<LOGN, ELOG, LO, EP>(0, u))];
}

template <int LOGN, int ELOG, int K>
struct FwdPasses {
  // pass K reads from LDS (K > 0) and leaves its result in registers
  static __device__ __forceinline__ void run(uint32_t (&v)[1 << ELOG], uint32_t *lds, uint32_t tid,
                                             const uint2 *tw, uint32_t q) {
    constexpr int LO = pass_lo_fwd(LOGN, ELOG, K), EP = pass_bits(LOGN, ELOG, K);
    constexpr int PLO = pass_lo_fwd(LOGN, ELOG, K - 1), PEP = pass_bits(LOGN, ELOG, K - 1);
    FwdPasses<LOGN, ELOG, K - 1>::run(v, lds, tid, tw, q);
    regs_to_lds<LOGN, ELOG, PLO, PEP>(v, lds, tid);
    __syncthreads();
    lds_to_regs<LOGN, ELOG, LO, EP>(v, lds, tid);
    fwd_pass<LOGN, ELOG, LO, EP>(v, tid, tw, q);
  }
};
template <int LOGN, int ELOG>
struct FwdPasses<LOGN, ELOG, 0> {
  // pass 0 expects its inputs already in registers (loaded from global)
  static __device__ __forceinline__ void run(uint32_t (&v)[1 << ELOG], uint32_t *, uint32_t tid, const uint2 *tw,
                                             uint32_t q) {
    constexpr int LO = pass_lo_fwd(LOGN, ELOG, 0), EP = pass_bits(LOGN, ELOG, 0);
    fwd_pass<LOGN, ELOG, LO, EP>(v, tid, tw, q);
  }
};

// Polynomial m exchanges through lds + m * lds_words(LOGN).
__host__ __device__ constexpr uint32_t lds_words(int logn) { return (1u << logn) + (1u << logn) / 32; }

// Inverse passes cover index bits [PRE, LOGN): the stages on bits below PRE
// were done by the multiply-accumulate's epilogue (PRE = 0: all stages here).
__host__ __device__ constexpr int inv_np(int logn, int elog, int pre) { return n_pass(logn - pre, elog); }
__host__ __device__ constexpr int inv_lo(int logn, int elog, int pre, int k) {
  return pre + pass_lo_inv(logn - pre, elog, k);
}
__host__ __device__ constexpr int inv_ep(int logn, int elog, int pre, int k) { return pass_bits(logn - pre, elog, k); }

template <int LOGN, int ELOG, int K, int PS, int M, int PRE>
struct InvPasses {
  static __device__ __forceinline__ void run(uint32_t (&v)[M][1 << ELOG], uint32_t *lds, uint32_t tid,
                                             const uint2 *tw, uint32_t q, uint32_t a, uint32_t ap, uint32_t b,
                                             uint32_t bp) {
    constexpr int LO = inv_lo(LOGN, ELOG, PRE, K), EP = inv_ep(LOGN, ELOG, PRE, K);
    constexpr int PLO = inv_lo(LOGN, ELOG, PRE, K - 1), PEP = inv_ep(LOGN, ELOG, PRE, K - 1);
    InvPasses<LOGN, ELOG, K - 1, PS, M, PRE>::run(v, lds, tid, tw, q, a, ap, b, bp);
#pragma unroll
    for (int m = 0; m < M; ++m) regs_to_lds<LOGN, ELOG, PLO, PEP>(v[m], lds + m * lds_words(LOGN), tid);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < M; ++m) lds_to_regs<LOGN, ELOG, LO, EP>(v[m], lds + m * lds_words(LOGN), tid);
    inv_pass<LOGN, ELOG, LO, EP, PS, M>(v, tid, tw, q, a, ap, b, bp);
  }
};
template <int LOGN, int ELOG, int PS, int M, int PRE>
struct InvPasses<LOGN, ELOG, 0, PS, M, PRE> {
  // pass 0 (bits [PRE, PRE + EP)) expects its inputs already in registers
  static __device__ __forceinline__ void run(uint32_t (&v)[M][1 << ELOG], uint32_t *, uint32_t tid,
                                             const uint2 *tw, uint32_t q, uint32_t a, uint32_t ap, uint32_t b,
                                             uint32_t bp) {
    constexpr int LO = inv_lo(LOGN, ELOG, PRE, 0), EP = inv_ep(LOGN, ELOG, PRE, 0);
    inv_pass<LOGN, ELOG, LO, EP, PS, M>(v, tid, tw, q, a, ap, b, bp);
  }
};

// A pass over bits [0, EP) holds 2^EP consecutive coefficients per group in
// registers: move them with 16-byte accesses.
template <int LOGN, int ELOG, int EP>
__device__ __forceinline__ void load_low_pass(uint32_t (&v)[1 << ELOG], const uint32_t *src, uint32_t tid) {
  static_assert(EP >= 2, "vector access needs 4 consecutive words");
  const uint32_t *sb = src + gidx<LOGN, ELOG, 0, EP>(tid, 0);
#pragma unroll
  for (int u = 0; u < (1 << ELOG); u += 4) {
    const uint4 t4 = *reinterpret_cast<const uint4 *>(sb + gidx<LOGN, ELOG, 0, EP>(0, u));
    v[u] = t4.x;
    v[u + 1] = t4.y;
    v[u + 2] = t4.z;
    v[u + 3] = t4.w;
  }
}

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
  const uint32_t *src = tab.n ? (const uint32_t *)tab.p[poly / ppi] + (poly % ppi) * N : in + poly * N;
  uint32_t v[E];
  {
    constexpr int LO = pass_lo_fwd(LOGN, ELOG, 0), EP = pass_bits(LOGN, ELOG, 0);
    const uint32_t *sb = src + gidx<LOGN, ELOG, LO, EP>(tid, 0);
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

// ---------------------------------------------------------------- inverse NTT kernels
// PS: top stages pruned (see inv_pass); 0 for the whole transform. M
// polynomials src[m] of one limb, LDS of M * lds_words(LOGN) words. PRE:
// stages on bits below PRE already done (the first pass then reads its
// coefficients with coalesced 4-byte loads: lanes map to the low bits).
template <int LOGN, int ELOG, int PS, int M, int PRE>
__device__ __forceinline__ void intt_core(const uint32_t *const (&src)[M], uint32_t (&v)[M][1 << ELOG],
                                          uint32_t *lds, uint32_t tid, const LimbConsts &c, const uint2 *tw,
                                          uint32_t l) {
  constexpr int NP = inv_np(LOGN, ELOG, PRE);
  if constexpr (PRE == 0) {
#pragma unroll
    for (int m = 0; m < M; ++m) load_low_pass<LOGN, ELOG, pass_bits(LOGN, ELOG, 0)>(v[m], src[m], tid);
  } else {
    constexpr int LO = inv_lo(LOGN, ELOG, PRE, 0), EP = inv_ep(LOGN, ELOG, PRE, 0);
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const uint32_t *sb = src[m] + gidx<LOGN, ELOG, LO, EP>(tid, 0);
#pragma unroll
      for (int u = 0; u < (1 << ELOG); ++u) v[m][u] = sb[gidx<LOGN, ELOG, LO, EP>(0, u)];
    }
  }
  InvPasses<LOGN, ELOG, NP - 1, PS, M, PRE>::run(v, lds, tid, tw, c.q[l], c.ninv[l], c.ninv_p[l], c.ninvw[l],
                                                 c.ninvw_p[l]);
}

// Full mode: [P][N] -> [P][N] canonical (in place allowed).
template <int LOGN, int ELOG>
__global__ __launch_bounds__(1 << (LOGN - ELOG)) void k_intt_full(const uint32_t *in, uint32_t *out, LimbConsts c,
                                                                   Twiddles tws) {
  constexpr int N = 1 << LOGN, E = 1 << ELOG, NP = n_pass(LOGN, ELOG);
  __shared__ uint32_t lds[N + N / 32];
  const uint32_t tid = threadIdx.x;
  const size_t poly = blockIdx.x;
  const uint32_t l = (uint32_t)(poly % c.L);
  uint32_t v[1][E];
  const uint32_t *const src[1] = {in + poly * N};
  intt_core<LOGN, ELOG, 0, 1, 0>(src, v, lds, tid, c, tws.inv + (size_t)l * N, l);
  constexpr int LO = pass_lo_inv(LOGN, ELOG, NP - 1), EP = pass_bits(LOGN, ELOG, NP - 1);
  uint32_t *dst = out + poly * N;
  const uint32_t q = c.q[l];
  uint32_t *db = dst + gidx<LOGN, ELOG, LO, EP>(tid, 0);
#pragma unroll
  for (int u = 0; u < E; ++u) db[gidx<LOGN, ELOG, LO, EP>(0, u)] = csub(v[0][u], q);
}

// Masked mode over Yhat [B][O][2][L][N]: c1 polynomials are written whole to
// c1_out [B][O][L][N]; c0 polynomials get the server mask added at the valid
// output coefficients, which are gathered into c0_ext [B][c_out][L][ho][wo].
// With pointer tables (out.n > 0) image b's mask, c0_ext and c1_out are
// separate buffers (out.mask[b], out.c0[b], out.c1[b]) laid out as for B = 1.
// PS: top stages of the c0 transform that are pruned (2^(LOGN - PS) must
// exceed every extracted coefficient index); c1 is always transformed whole.
// M: polynomials per workgroup, those of M consecutive (image, output
// ciphertext) indices bo with the same half p and limb l; workgroup w is
// ((pair 2 + p) L + l), bo = pair M + m. Slots past B O compute a copy of
// slot 0 and store nothing. PRE: the stages on index bits below PRE were done
// by the multiply-accumulate (Yhat holds their output).
template <int LOGN, int ELOG, int PS, int M, int PRE>
__global__ __launch_bounds__(1 << (LOGN - ELOG)) void k_intt_masked(const uint32_t *yhat, const uint32_t *mask,
                                                                     uint32_t *c0_ext, uint32_t *c1_out, ConvGeom g,
                                                                     uint32_t B, LimbConsts c, Twiddles tws,
                                                                     OutPtrs out) {
  constexpr int N = 1 << LOGN, E = 1 << ELOG, NT = 1 << (LOGN - ELOG), NP = inv_np(LOGN, ELOG, PRE);
  __shared__ uint32_t lds[M * lds_words(LOGN)];
  const uint32_t tid = threadIdx.x;
  const uint32_t wg = blockIdx.x;
  const uint32_t l = wg % g.L;
  const uint32_t p = (wg / g.L) % 2;
  const size_t pair = wg / (2 * g.L);
  const size_t nbo = (size_t)B * g.O;
  size_t bo[M];
  bool valid[M];
  const uint32_t *src[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    bo[m] = pair * M + m;
    valid[m] = bo[m] < nbo;  // uniform
    src[m] = yhat + (((valid[m] ? bo[m] : bo[0]) * 2 + p) * g.L + l) * (size_t)N;
  }
  const uint32_t q = c.q[l];
  uint32_t v[M][E];
  constexpr int LO = inv_lo(LOGN, ELOG, PRE, NP - 1), EP = inv_ep(LOGN, ELOG, PRE, NP - 1);
  const uint2 *tw = tws.inv + (size_t)l * N;
  if (p == 1) {
    intt_core<LOGN, ELOG, 0, M, PRE>(src, v, lds, tid, c, tw, l);
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (!valid[m]) continue;
      const uint32_t o = (uint32_t)(bo[m] % g.O);
      const size_t b = bo[m] / g.O;
      uint32_t *dst = out.n ? (uint32_t *)out.c1[b] + ((size_t)o * g.L + l) * N : c1_out + (bo[m] * g.L + l) * (size_t)N;
      uint32_t *db = dst + gidx<LOGN, ELOG, LO, EP>(tid, 0);
#pragma unroll
      for (int u = 0; u < E; ++u) db[gidx<LOGN, ELOG, LO, EP>(0, u)] = csub(v[m][u], q);
    }
    return;
  }
  // c0 needs only its extracted coefficients
  intt_core<LOGN, ELOG, PS, M, PRE>(src, v, lds, tid, c, tw, l);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m) regs_to_lds<LOGN, ELOG, LO, EP>(v[m], lds + m * lds_words(LOGN), tid);
  __syncthreads();
  const uint32_t t = c.t, half = c.t / 2;
  const uint32_t dl = c.delta[l], dlp = c.delta_p[l];
  const size_t hw = (size_t)g.ho * g.wo;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    if (!valid[m]) continue;
    const uint32_t o = (uint32_t)(bo[m] % g.O);
    const size_t b = bo[m] / g.O;
    const uint32_t *lm = lds + m * lds_words(LOGN);
    const uint32_t i = o / g.T, tau = o % g.T;
    // output rows of this tile: s*oy in [tau r_o, (tau+1) r_o)  (r_o is a multiple of s)
    const uint32_t oy0 = tau * g.r_o / g.s;
    const uint32_t oy1 = min(g.ho, (tau + 1) * g.r_o / g.s);
    const uint32_t count = (oy1 > oy0 ? oy1 - oy0 : 0) * g.wo;
    const uint32_t *mrow = out.n ? (const uint32_t *)out.mask[b] + i * hw : mask + (b * g.c_out + i) * hw;
    uint32_t *orow = out.n ? (uint32_t *)out.c0[b] + ((size_t)i * g.L + l) * hw
                           : c0_ext + ((b * g.c_out + i) * g.L + l) * hw;
    for (uint32_t idx = tid; idx < count; idx += NT) {
      const uint32_t oy = oy0 + idx / g.wo, ox = idx % g.wo;
      const uint32_t e = (g.s * oy - tau * g.r_o) * g.w_pad + g.s * ox;
      const uint32_t r = mrow[oy * g.wo + ox];
      const uint32_t rc = r > half ? r - t + q : r;  // centred lift of r, taken mod q
      const uint32_t add = csub(shoup_lazy(rc, dl, dlp, q), q);
      orow[oy * g.wo + ox] = csub(csub(lm[lpad(e)], q) + add, q);
    }
  }
}

// ---------------------------------------------------------------- multiply-accumulate
// Yhat[b][o][p][l][k] = sum_{gw < G_w} What[i][gw][l][k] * Xhat[b][gw T + tau][p][l][k]  mod q_l,
// o = i T + tau.
// Register-tiled form: one thread owns coefficient k and CT output channels
// (same row tile tau) for BT images x 2 polynomials, so each input value it
// loads is used CT times and each weight 2 BT times. A workgroup is RG x CG
// waves over the same 64 coefficients: RG groups of images times CG groups of
// output channels. Waves of one channel group read the same weights and
// waves of one image group the same inputs, which L1 then serves once.
// NS register sets form a ring: the loads of input ciphertext gw + NS are
// issued right after gw's multiply-accumulates, so NS - 1 ciphertexts are in
// flight while one is being multiplied.
template <int BT, int CT, int RG, int CG, int NS>
__global__ __launch_bounds__(64 * RG * CG) void k_mac_tiled(const uint32_t *__restrict__ X,
                                                            const uint32_t *__restrict__ Wt,
                                                            uint32_t *__restrict__ Y, ConvGeom g, uint32_t B,
                                                            uint32_t nib, uint32_t nkb, LimbConsts c) {
  static_assert(NS >= 2 && NS * (CT + 2 * BT) <= 63, "loads in flight beyond the vector memory counter");
  const uint32_t nwg = gridDim.x;
  uint32_t wg = blockIdx.x;
  if ((nwg & 7u) == 0) wg = (wg & 7u) * (nwg >> 3) + (wg >> 3);
  // image tiles vary fastest: the workgroups that share one weight tile run
  // next to each other (on one XCD, by the remap above), then channel tiles,
  // which share input tiles
  const uint32_t nbt = (B + RG * BT - 1) / (RG * BT);
  const uint32_t bt = wg % nbt;
  uint32_t r = wg / nbt;
  const uint32_t ib = r % nib;
  r /= nib;
  const uint32_t tau = r % g.T;
  r /= g.T;
  const uint32_t kb = r % nkb;
  const uint32_t l = r / nkb;
  // wave-uniform indices (readfirstlane keeps the bases in scalar registers)
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t rg = wave % RG, cg = wave / RG;
  const uint32_t i0 = (ib * CG + cg) * CT;
  const uint32_t b0 = (bt * RG + rg) * BT;
  if (i0 >= g.c_out || b0 >= B) return;
  const uint32_t nc = min((uint32_t)CT, g.c_out - i0);
  const uint32_t nb = min((uint32_t)BT, B - b0);
  const uint32_t LN = g.L * g.N;
  // Scalar bases advance by one input ciphertext per step; each (image,
  // polynomial) and each channel adds a wave-uniform byte offset (32-bit;
  // the host guarantees BT*G*2*L*N*4 and CT*G_w*L*N*4 < 2^32), and every
  // lane the same 4 * lane.
  const char *xbase = (const char *)(X + ((size_t)b0 * g.G + tau) * 2 * LN + (size_t)l * g.N + (size_t)kb * 64);
  const char *wbase = (const char *)(Wt + (size_t)i0 * g.G_w * LN + (size_t)l * g.N + (size_t)kb * 64);
  const size_t xstep = (size_t)8 * LN * g.T, wstep = (size_t)4 * LN;  // bytes
  const uint32_t lane4 = lane * 4u;
  uint32_t xo[BT][2], wo[CT];
#pragma unroll
  for (int bb = 0; bb < BT; ++bb) {
    const uint32_t b = (uint32_t)bb < nb ? (uint32_t)bb : 0u;  // clamp: loads of absent images are discarded
    xo[bb][0] = __builtin_amdgcn_readfirstlane(b * g.G * 2 * LN * 4u);
    xo[bb][1] = __builtin_amdgcn_readfirstlane(xo[bb][0] + LN * 4u);
  }
#pragma unroll
  for (int cc = 0; cc < CT; ++cc)
    wo[cc] = __builtin_amdgcn_readfirstlane(((uint32_t)cc < nc ? (uint32_t)cc : 0u) * g.G_w * LN * 4u);
  const uint32_t q = c.q[l], r2 = c.r2[l], fold = c.fold[l];
  uint64_t acc[CT][BT][2];
#pragma unroll
  for (int cc = 0; cc < CT; ++cc)
#pragma unroll
    for (int bb = 0; bb < BT; ++bb) acc[cc][bb][0] = acc[cc][bb][1] = 0;
  const uint32_t G_w = g.G_w;
  // Raw buffer loads: the step's base in the descriptor, the uniform offset
  // in soffset, the lane's in voffset - no vector address arithmetic. Every
  // access is in bounds by construction; num_records is the maximum.
  auto load = [&](uint32_t gw, uint32_t (&w)[CT], uint32_t (&x)[BT][2]) {
    const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(xbase + gw * xstep), (short)0, (int)0xffffffffu, (int)kBufferWord3);
    const __amdgpu_buffer_rsrc_t wr = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(wbase + gw * wstep), (short)0, (int)0xffffffffu, (int)kBufferWord3);
#pragma unroll
    for (int cc = 0; cc < CT; ++cc) w[cc] = __builtin_amdgcn_raw_buffer_load_b32(wr, lane4, wo[cc], 0);
#pragma unroll
    for (int bb = 0; bb < BT; ++bb) {
      x[bb][0] = __builtin_amdgcn_raw_buffer_load_b32(xr, lane4, xo[bb][0], 0);
      x[bb][1] = __builtin_amdgcn_raw_buffer_load_b32(xr, lane4, xo[bb][1], 0);
    }
  };
  auto mac = [&](const uint32_t (&w)[CT], const uint32_t (&x)[BT][2]) {
#pragma unroll
    for (int cc = 0; cc < CT; ++cc)
#pragma unroll
      for (int bb = 0; bb < BT; ++bb) {
        acc[cc][bb][0] += (uint64_t)w[cc] * x[bb][0];
        acc[cc][bb][1] += (uint64_t)w[cc] * x[bb][1];
      }
  };
  // One loop over ring turns. Its body has no data-dependent branches, so the
  // compiler keeps the ring's order: loads past the end re-read the last
  // ciphertext, and sets past the end get zero weights. Every fold / NS turns
  // (at most fold terms) the accumulators are folded, exactly mod q; that
  // branch is uniform and does no loads, so both of its paths leave the same
  // loads in flight. The last partial chunk needs no fold: reduce64 takes any
  // 64-bit value. NS * (CT + 2 BT) loads in flight must stay within the
  // 63 that the vector memory counter can track.
  uint32_t ws[NS][CT], xs[NS][BT][2];
  const uint32_t last = G_w - 1;
  const uint32_t turns_per_fold = fold / NS;
  // the prologue issues the sets in ring order too: the loop's first wait
  // is computed from the order on entry as well as around the loop
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    asm volatile("" ::: "memory");
    load(min((uint32_t)j, last), ws[j], xs[j]);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
  }
  uint32_t turn = 0;
  for (uint32_t gw = 0; gw < G_w; gw += NS) {
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      // sched_barrier keeps each group in place: a set's loads are all
      // issued before the next set's, so waiting for one never waits for
      // a later one
      if (j > 0) {
        const bool tail = gw + j >= G_w;
#pragma unroll
        for (int cc = 0; cc < CT; ++cc) ws[j][cc] = tail ? 0u : ws[j][cc];
      }
      mac(ws[j], xs[j]);
      __builtin_amdgcn_sched_barrier(0);
      asm volatile("" ::: "memory");  // compiler-only barrier: loads stay in this slot
      load(min(gw + NS + j, last), ws[j], xs[j]);
      asm volatile("" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
    }
    if (++turn == turns_per_fold) {
      turn = 0;
#pragma unroll
      for (int cc = 0; cc < CT; ++cc)
#pragma unroll
        for (int bb = 0; bb < BT; ++bb)
#pragma unroll
          for (int pp = 0; pp < 2; ++pp)
            acc[cc][bb][pp] = (uint64_t)(uint32_t)(acc[cc][bb][pp] >> 32) * r2 + (uint32_t)acc[cc][bb][pp];
    }
  }
  const uint32_t r2p = c.r2_p[l], onep = c.one_p[l];
  const uint32_t k = kb * 64 + lane;
#pragma unroll
  for (int cc = 0; cc < CT; ++cc) {
    if ((uint32_t)cc >= nc) continue;
    const uint32_t o = (i0 + cc) * g.T + tau;
#pragma unroll
    for (int bb = 0; bb < BT; ++bb) {
      if ((uint32_t)bb >= nb) continue;
      uint32_t *y = Y + (((size_t)(b0 + bb) * g.O + o) * 2) * LN + (size_t)l * g.N + k;
      y[0] = reduce64(acc[cc][bb][0], q, r2, r2p, onep);
      y[LN] = reduce64(acc[cc][bb][1], q, r2, r2p, onep);
    }
  }
}

// LDS-staged form of the same register tile. Per input ciphertext ("step")
// the workgroup needs NX = RG BT 2 input segments and NW = CG CT weight
// segments of 64 coefficients (256 bytes). They are loaded once per
// workgroup - every thread the same number of bytes of each, 16 at a time
// where the share allows - into a ring of R register sets (R steps in
// flight), written to one of two LDS buffers, and each wave reads its
// operands from there. One barrier per step orders the LDS buffers: step g
// is read from buffer g & 1 while step g + 1 is written to the other.
template <int BYTES>
struct Chunk;  // one thread's share of one operand per step
template <>
struct Chunk<4> {
  uint32_t v;
  __device__ void load(__amdgpu_buffer_rsrc_t r, uint32_t off) { v = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0); }
  __device__ void store(char *lds) const { *(uint32_t *)lds = v; }
};
template <>
struct Chunk<8> {
  uint2 v;
  __device__ void load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    v = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  }
  __device__ void store(char *lds) const { *(uint2 *)lds = v; }
};
template <>
struct Chunk<16> {
  uint4 v;
  __device__ void load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    v = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  }
  __device__ void store(char *lds) const { *(uint4 *)lds = v; }
};

// PRE > 0 (tiles with one output polynomial per lane, 2 BT CT = 64): before
// storing, the epilogue applies the inverse NTT's first PRE Gentleman-Sande
// stages (index bits 0 .. PRE-1), which act within the workgroup's block of 64
// coefficients. In two rounds, one per half of the block, each wave moves its
// 64 polynomials x 32 coefficients through LDS so that a lane holds 32
// consecutive coefficients of one polynomial, runs the stages in registers
// with twiddles that are the same for every lane (scalar loads, shared by the
// whole workgroup), and goes back through LDS so that the stores are
// coalesced. The masked inverse NTT then starts at bit PRE.
template <int BT, int CT, int RG, int CG, int R, int PRE>
__global__ __launch_bounds__(64 * RG * CG) void k_mac_lds(const uint32_t *__restrict__ X,
                                                          const uint32_t *__restrict__ Wt,
                                                          uint32_t *__restrict__ Y, ConvGeom g, uint32_t B,
                                                          uint32_t nib, uint32_t nkb, LimbConsts c,
                                                          const uint2 *__restrict__ twinv) {
  constexpr int NT = 64 * RG * CG;
  constexpr int NX = RG * BT * 2, NW = CG * CT;               // segments per step
  constexpr int XB = NX * 256 / NT, WB = NW * 256 / NT;       // bytes per thread per step
  static_assert(NX * 256 % NT == 0 && NW * 256 % NT == 0, "shares must be whole");
  constexpr int XW = XB < 16 ? XB : 16, WWD = WB < 16 ? WB : 16;  // access widths
  constexpr int KX = XB / XW, KW = WB / WWD;                      // accesses per thread per step
  static_assert((XW == 4 || XW == 8 || XW == 16) && (WWD == 4 || WWD == 8 || WWD == 16), "access width");
  static_assert(R >= 2 && R * (KX + KW) <= 63, "loads in flight beyond the vector memory counter");
  constexpr uint32_t BUFB = (NX + NW) * 256;  // bytes per LDS buffer
  static_assert(PRE == 0 || (PRE == 5 && 2 * BT * CT == 64), "epilogue stages need one polynomial per lane");
  constexpr uint32_t RWW = 64 * 36;             // epilogue: words per wave (64 x (32 + 4 pad))
  constexpr uint32_t LDSB = PRE ? (2 * BUFB > RG * CG * RWW * 4 ? 2 * BUFB : RG * CG * RWW * 4) : 2 * BUFB;
  __shared__ uint4 stage4[LDSB / 16];
  char *stage = (char *)stage4;
  const uint32_t nwg = gridDim.x;
  uint32_t wg = blockIdx.x;
  if ((nwg & 7u) == 0) wg = (wg & 7u) * (nwg >> 3) + (wg >> 3);
  // image tiles vary fastest: the workgroups that share one weight tile run
  // next to each other (on one XCD, by the remap above), then channel tiles,
  // which share input tiles
  const uint32_t nbt = (B + RG * BT - 1) / (RG * BT);
  const uint32_t bt = wg % nbt;
  uint32_t r = wg / nbt;
  const uint32_t ib = r % nib;
  r /= nib;
  const uint32_t tau = r % g.T;
  r /= g.T;
  const uint32_t kb = r % nkb;
  const uint32_t l = r / nkb;
  const uint32_t tid = threadIdx.x;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t lane = tid & 63u;
  const uint32_t rg = wave % RG, cg = wave / RG;
  // workgroup tile: images [bw, bw + nbw), channels [iw, iw + ncw)
  const uint32_t bw = bt * RG * BT, iw = ib * CG * CT;
  if (bw >= B || iw >= g.c_out) return;  // uniform over the workgroup
  const uint32_t nbw = min((uint32_t)(RG * BT), B - bw), ncw = min((uint32_t)(CG * CT), g.c_out - iw);
  const uint32_t LN = g.L * g.N;
  // Per-thread global byte offsets and LDS byte positions of its accesses
  // (fixed for the whole loop). Byte e of the step's input share sits in
  // segment e / 256 = 2 i + p; absent images and channels read image /
  // channel 0 of the tile, whose results are never stored.
  uint32_t xoff[KX], woff[KW];
#pragma unroll
  for (int k = 0; k < KX; ++k) {
    const uint32_t e = (tid + k * NT) * XW, seg = e >> 8, i = seg >> 1;
    xoff[k] = (((i < nbw ? i : 0u) * g.G * 2 + (seg & 1u)) * LN) * 4u + (e & 255u);
  }
#pragma unroll
  for (int k = 0; k < KW; ++k) {
    const uint32_t e = (tid + k * NT) * WWD, cc = e >> 8;
    woff[k] = ((cc < ncw ? cc : 0u) * g.G_w * LN) * 4u + (e & 255u);
  }
  const char *xbase = (const char *)(X + ((size_t)bw * g.G + tau) * 2 * LN + (size_t)l * g.N + (size_t)kb * 64);
  const char *wbase = (const char *)(Wt + (size_t)iw * g.G_w * LN + (size_t)l * g.N + (size_t)kb * 64);
  const size_t xstep = (size_t)8 * LN * g.T, wstep = (size_t)4 * LN;  // bytes
  const uint32_t G_w = g.G_w, last = G_w - 1;
  using CX = Chunk<XW>;
  using CW = Chunk<WWD>;
  auto gload = [&](uint32_t gw, CX (&rx)[KX], CW (&rw)[KW]) {
    const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(xbase + gw * xstep), (short)0, (int)0xffffffffu, (int)kBufferWord3);
    const __amdgpu_buffer_rsrc_t wr = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(wbase + gw * wstep), (short)0, (int)0xffffffffu, (int)kBufferWord3);
#pragma unroll
    for (int k = 0; k < KX; ++k) rx[k].load(xr, xoff[k]);
#pragma unroll
    for (int k = 0; k < KW; ++k) rw[k].load(wr, woff[k]);
  };
  auto lstore = [&](uint32_t buf, const CX (&rx)[KX], const CW (&rw)[KW]) {
    char *sb = stage + buf * BUFB;
#pragma unroll
    for (int k = 0; k < KX; ++k) rx[k].store(sb + (tid + k * NT) * XW);
#pragma unroll
    for (int k = 0; k < KW; ++k) rw[k].store(sb + NX * 256 + (tid + k * NT) * WWD);
  };
  const uint32_t q = c.q[l], r2 = c.r2[l], fold = c.fold[l];
  uint64_t acc[CT][BT][2];
#pragma unroll
  for (int cc = 0; cc < CT; ++cc)
#pragma unroll
    for (int bb = 0; bb < BT; ++bb) acc[cc][bb][0] = acc[cc][bb][1] = 0;
  // this wave's operands inside a stage buffer (words)
  const uint32_t *xs0 = (const uint32_t *)stage + (rg * BT * 2) * 64 + lane;
  const uint32_t *ws0 = (const uint32_t *)stage + (NX + cg * CT) * 64 + lane;
  constexpr uint32_t BUFW = BUFB / 4;  // words per buffer
  CX rx[R][KX];
  CW rw[R][KW];
  // prologue: steps 0 .. R-1 in flight, step 0 into buffer 0, step R into set 0
#pragma unroll
  for (int j = 0; j < R; ++j) {
    asm volatile("" ::: "memory");
    gload(min((uint32_t)j, last), rx[j], rw[j]);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
  }
  lstore(0, rx[0], rw[0]);
  asm volatile("" ::: "memory");
  gload(min((uint32_t)R, last), rx[0], rw[0]);
  asm volatile("" ::: "memory");
  __syncthreads();
  uint32_t since_fold = 0;
  // step g: operands from buffer g & 1; set (g + 1) % R holds step g + 1 and
  // goes to the other buffer, then reloads with step g + 1 + R
  for (uint32_t g0 = 0; g0 < G_w; g0 += R) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const uint32_t gw = g0 + j;
      if (gw >= G_w) break;  // uniform
      const uint32_t *xs = xs0 + (gw & 1u) * BUFW, *wsp = ws0 + (gw & 1u) * BUFW;
      uint32_t w[CT], x[BT][2];
#pragma unroll
      for (int cc = 0; cc < CT; ++cc) w[cc] = wsp[cc * 64];
#pragma unroll
      for (int bb = 0; bb < BT; ++bb) {
        x[bb][0] = xs[(bb * 2) * 64];
        x[bb][1] = xs[(bb * 2 + 1) * 64];
      }
      const int jn = (j + 1) % R;
      asm volatile("" ::: "memory");
      lstore((gw + 1) & 1u, rx[jn], rw[jn]);
      asm volatile("" ::: "memory");
      gload(min(gw + 1 + R, last), rx[jn], rw[jn]);
      asm volatile("" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int cc = 0; cc < CT; ++cc)
#pragma unroll
        for (int bb = 0; bb < BT; ++bb) {
          acc[cc][bb][0] += (uint64_t)w[cc] * x[bb][0];
          acc[cc][bb][1] += (uint64_t)w[cc] * x[bb][1];
        }
      if (++since_fold == fold) {
        since_fold = 0;
#pragma unroll
        for (int cc = 0; cc < CT; ++cc)
#pragma unroll
          for (int bb = 0; bb < BT; ++bb)
#pragma unroll
            for (int pp = 0; pp < 2; ++pp)
              acc[cc][bb][pp] = (uint64_t)(uint32_t)(acc[cc][bb][pp] >> 32) * r2 + (uint32_t)acc[cc][bb][pp];
      }
      __syncthreads();
    }
  }
  // wave tile and its stores
  const uint32_t i0 = iw + cg * CT, b0 = bw + rg * BT;
  const uint32_t r2p = c.r2_p[l], onep = c.one_p[l];
  if constexpr (PRE == 0) {
    if (i0 >= g.c_out || b0 >= B) return;
    const uint32_t nc = min((uint32_t)CT, g.c_out - i0), nb = min((uint32_t)BT, B - b0);
    const uint32_t k = kb * 64 + lane;
#pragma unroll
    for (int cc = 0; cc < CT; ++cc) {
      if ((uint32_t)cc >= nc) continue;
      const uint32_t o = (i0 + cc) * g.T + tau;
#pragma unroll
      for (int bb = 0; bb < BT; ++bb) {
        if ((uint32_t)bb >= nb) continue;
        uint32_t *y = Y + (((size_t)(b0 + bb) * g.O + o) * 2) * LN + (size_t)l * g.N + k;
        y[0] = reduce64(acc[cc][bb][0], q, r2, r2p, onep);
        y[LN] = reduce64(acc[cc][bb][1], q, r2, r2p, onep);
      }
    }
  } else {
    // every wave takes part in the epilogue's barriers, also one whose tile
    // is absent (it stores nothing)
    uint32_t val[CT][BT][2];
#pragma unroll
    for (int cc = 0; cc < CT; ++cc)
#pragma unroll
      for (int bb = 0; bb < BT; ++bb)
#pragma unroll
        for (int pp = 0; pp < 2; ++pp) val[cc][bb][pp] = reduce64(acc[cc][bb][pp], q, r2, r2p, onep);
    // polynomial P = (cc BT + bb) 2 + pp of the wave's tile is row P of the
    // wave's LDS region
    uint32_t *region = (uint32_t *)stage + wave * RWW;
    const uint32_t q2 = 2 * q;
    const uint32_t LOGN = 31 - __builtin_clz(g.N);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      __syncthreads();  // the staging buffers, or the previous round's region, are free
      if ((lane >> 5) == (uint32_t)h) {
#pragma unroll
        for (int cc = 0; cc < CT; ++cc)
#pragma unroll
          for (int bb = 0; bb < BT; ++bb)
#pragma unroll
            for (int pp = 0; pp < 2; ++pp) region[((cc * BT + bb) * 2 + pp) * 36 + (lane & 31u)] = val[cc][bb][pp];
      }
      __syncthreads();
      uint32_t v[32];
      const uint4 *r4 = (const uint4 *)(region + lane * 36);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint4 t4 = r4[k];
        v[4 * k] = t4.x, v[4 * k + 1] = t4.y, v[4 * k + 2] = t4.z, v[4 * k + 3] = t4.w;
      }
      // stages on bits 0 .. PRE-1 of j = kb 64 + h 32 + u; twiddle index
      // 2^(LOGN-1-b) + (j >> (b+1)), the same for every lane of the wave
      const uint32_t j0 = kb * 64 + h * 32;
#pragma unroll
      for (int b = 0; b < PRE; ++b) {
        const_u64 *tw = (const_u64 *)(twinv + (size_t)l * g.N + (1u << (LOGN - 1 - b)) + (j0 >> (b + 1)));
#pragma unroll
        for (int u = 0; u < 32; ++u) {
          if (u & (1 << b)) continue;
          const int u2 = u | (1 << b);
          const uint64_t wt = tw[u >> (b + 1)];
          const uint32_t X = v[u], Yv = v[u2];
          v[u] = csub(X + Yv, q2);
          v[u2] = shoup_lazy(X - Yv + q2, (uint32_t)wt, (uint32_t)(wt >> 32), q);
        }
      }
      // back through the wave's region so that every store instruction
      // writes two whole 128-byte runs: lanes 0-31 coefficient (lane) of
      // polynomial 2 jp, lanes 32-63 the same of polynomial 2 jp + 1
      uint4 *w4 = (uint4 *)(region + lane * 36);
#pragma unroll
      for (int k = 0; k < 8; ++k) w4[k] = make_uint4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const uint32_t half = lane >> 5, kk = lane & 31u;
#pragma unroll
      for (int jp = 0; jp < 32; ++jp) {
        const uint32_t P = 2 * jp + half;  // this lane's polynomial for the jp-th store
        const uint32_t scc = P / (2 * BT), sbb = (P >> 1) % BT, spp = P & 1u;
        const uint32_t x = region[P * 36 + kk];
        if (i0 + scc < g.c_out && b0 + sbb < B)
          Y[(((size_t)(b0 + sbb) * g.O + (i0 + scc) * g.T + tau) * 2 + spp) * LN + (size_t)l * g.N + kb * 64 +
            h * 32 + kk] = x;
      }
    }
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

// ---------------------------------------------------------------- launchers
template <int LOGN, int ELOG>
static hipError_t fwd_t(const uint32_t *in, uint32_t *out, size_t np, const LimbConsts &c, const Twiddles &tw,
                        const ImgPtrs &tab, uint32_t ppi, hipStream_t st) {
  if (np == 0) return hipSuccess;
  hipLaunchKernelGGL((k_ntt_fwd<LOGN, ELOG>), dim3((uint32_t)np), dim3(1 << (LOGN - ELOG)), 0, st, in, out, c, tw,
                     tab, ppi);
  return hipGetLastError();
}
template <int LOGN, int ELOG>
static hipError_t inv_t(const uint32_t *in, uint32_t *out, size_t np, const LimbConsts &c, const Twiddles &tw,
                        hipStream_t st) {
  if (np == 0) return hipSuccess;
  hipLaunchKernelGGL((k_intt_full<LOGN, ELOG>), dim3((uint32_t)np), dim3(1 << (LOGN - ELOG)), 0, st, in, out, c,
                     tw);
  return hipGetLastError();
}
template <int LOGN, int ELOG, int PS, int M, int PRE>
static hipError_t invm_ps(const ConvGeom &g, const uint32_t *y, const uint32_t *m, uint32_t *c0, uint32_t *c1,
                          uint32_t B, const LimbConsts &c, const Twiddles &tw, const OutPtrs &out, hipStream_t st) {
  const size_t nbo = (size_t)B * g.O;
  const size_t nwg = (nbo + M - 1) / M * 2 * g.L;
  if (nwg == 0) return hipSuccess;
  hipLaunchKernelGGL((k_intt_masked<LOGN, ELOG, PS, M, PRE>), dim3((uint32_t)nwg), dim3(1 << (LOGN - ELOG)), 0, st,
                     y, m, c0, c1, g, B, c, tw, out);
  return hipGetLastError();
}
template <int LOGN, int ELOG, int M, int PRE>
static hipError_t invm_pm(const ConvGeom &g, const uint32_t *y, const uint32_t *m, uint32_t *c0, uint32_t *c1,
                          uint32_t B, const LimbConsts &c, const Twiddles &tw, const OutPtrs &out, hipStream_t st) {
  const int ps = LOGN - (int)g.prune_bits;
  if (ps >= 7) return invm_ps<LOGN, ELOG, 7, M, PRE>(g, y, m, c0, c1, B, c, tw, out, st);
  if (ps >= 5) return invm_ps<LOGN, ELOG, 5, M, PRE>(g, y, m, c0, c1, B, c, tw, out, st);
  if (ps >= 3) return invm_ps<LOGN, ELOG, 3, M, PRE>(g, y, m, c0, c1, B, c, tw, out, st);
  if (ps >= 2) return invm_ps<LOGN, ELOG, 2, M, PRE>(g, y, m, c0, c1, B, c, tw, out, st);
  if (ps >= 1) return invm_ps<LOGN, ELOG, 1, M, PRE>(g, y, m, c0, c1, B, c, tw, out, st);
  return invm_ps<LOGN, ELOG, 0, M, PRE>(g, y, m, c0, c1, B, c, tw, out, st);
}
// Pruning fewer stages than allowed is always exact: take the largest
// instantiated count not above LOGN - prune_bits. Two polynomials per
// workgroup exist for ELOG <= 4 (the register and LDS budgets of ELOG 5);
// the forms that start at bit kMacPre exist for LOGN >= 12.
template <int LOGN, int ELOG>
static hipError_t invm_t(const ConvGeom &g, uint32_t npw, uint32_t pre, const uint32_t *y, const uint32_t *m,
                         uint32_t *c0, uint32_t *c1, uint32_t B, const LimbConsts &c, const Twiddles &tw,
                         const OutPtrs &out, hipStream_t st) {
  if (pre == 0) {
    if (npw == 1) return invm_pm<LOGN, ELOG, 1, 0>(g, y, m, c0, c1, B, c, tw, out, st);
    if constexpr (ELOG <= 4) {
      if (npw == 2) return invm_pm<LOGN, ELOG, 2, 0>(g, y, m, c0, c1, B, c, tw, out, st);
    }
  }
  if constexpr (LOGN >= 12) {
    if (pre == kMacPre) {
      if (npw == 1) return invm_pm<LOGN, ELOG, 1, kMacPre>(g, y, m, c0, c1, B, c, tw, out, st);
      if constexpr (ELOG <= 4) {
        if (npw == 2) return invm_pm<LOGN, ELOG, 2, kMacPre>(g, y, m, c0, c1, B, c, tw, out, st);
      }
    }
  }
  return hipErrorInvalidValue;
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
hipError_t launch_intt_full(uint32_t logn, uint32_t elog, const uint32_t *in, uint32_t *out, size_t np,
                            const LimbConsts &c, const Twiddles &tw, hipStream_t st) {
  HC_NTT_DISPATCH(inv_t, in, out, np, c, tw, st)
}
bool intt_masked_ok(uint32_t logn, uint32_t elog, uint32_t npw, uint32_t pre) {
  return ntt_variant_ok(logn, elog) && (npw == 1 || (npw == 2 && elog <= 4)) &&
         (pre == 0 || (pre == kMacPre && logn >= 12));
}

hipError_t launch_intt_masked(const ConvGeom &g, uint32_t logn, uint32_t elog, uint32_t npw, uint32_t pre,
                              const uint32_t *y, const uint32_t *m, uint32_t *c0, uint32_t *c1, uint32_t B,
                              const LimbConsts &c, const Twiddles &tw, hipStream_t st, const OutPtrs *tab) {
  OutPtrs none{};
  if (tab && (tab->n != B || B > kMaxTab)) return hipErrorInvalidValue;
  const OutPtrs &t = tab ? *tab : none;
  HC_NTT_DISPATCH(invm_t, g, npw, pre, y, m, c0, c1, B, c, tw, t, st)
}

template <int BT, int CT, int RG, int CG, int NS, int LDS, int PRE>
static hipError_t mac_t(const ConvGeom &g, const uint32_t *x, const uint32_t *w, uint32_t *y, uint32_t B,
                        const LimbConsts &c, const Twiddles &tw, hipStream_t st) {
  if (!mac_offsets_fit(g, MacShape{BT, CT, RG, CG, NS, LDS, PRE})) return hipErrorInvalidValue;
  const uint32_t nkb = g.N / 64;
  const uint32_t nib = (g.c_out + CG * CT - 1) / (CG * CT);
  const uint32_t nbt = (B + RG * BT - 1) / (RG * BT);
  const size_t nwg = (size_t)nib * g.T * nkb * g.L * nbt;
  if (nwg == 0) return hipSuccess;
  if constexpr (LDS != 0)
    hipLaunchKernelGGL((k_mac_lds<BT, CT, RG, CG, NS, PRE>), dim3((uint32_t)nwg), dim3(64 * RG * CG), 0, st, x, w,
                       y, g, B, nib, nkb, c, tw.inv);
  else
    hipLaunchKernelGGL((k_mac_tiled<BT, CT, RG, CG, NS>), dim3((uint32_t)nwg), dim3(64 * RG * CG), 0, st, x, w, y,
                       g, B, nib, nkb, c);
  return hipGetLastError();
}

// The register tile's 32-bit offsets span BT images and CT channels; the
// LDS-staged form's span the workgroup's RG BT images and CG CT channels.
bool mac_offsets_fit(const ConvGeom &g, const MacShape &m) {
  const uint64_t ln = (uint64_t)g.L * g.N * 4;
  const uint64_t bi = m.lds ? (uint64_t)m.rg * m.bt : m.bt, ch = m.lds ? (uint64_t)m.cg * m.ct : m.ct;
  return bi * g.G * 2 * ln < (1ull << 32) && ch * g.G_w * ln < (1ull << 32);
}

// (images per thread, channels per thread, image groups, channel groups,
//  loads in flight (register sets), LDS-staged, inverse stages in the epilogue)
#define HC_MAC_VARIANTS(X)                                                                                      \
  X(1, 8, 1, 4, 2, 0, 0) X(1, 4, 1, 4, 2, 0, 0) X(2, 4, 1, 4, 2, 0, 0) X(4, 4, 1, 4, 2, 0, 0)                   \
  X(4, 2, 1, 4, 2, 0, 0) X(8, 2, 1, 4, 2, 0, 0) X(4, 4, 4, 2, 2, 0, 0) X(4, 8, 4, 2, 2, 0, 0)                   \
  X(2, 8, 4, 2, 2, 0, 0) X(4, 4, 2, 4, 2, 0, 0) X(2, 4, 4, 4, 2, 0, 0) X(1, 8, 2, 4, 2, 0, 0)                   \
  X(4, 8, 4, 2, 3, 0, 0) X(2, 8, 4, 2, 4, 0, 0) X(4, 4, 4, 2, 4, 0, 0) X(4, 4, 2, 4, 4, 0, 0)                   \
  X(1, 8, 2, 4, 4, 0, 0) X(2, 4, 4, 4, 4, 0, 0) X(1, 8, 1, 4, 4, 0, 0) X(4, 8, 4, 2, 2, 1, 0)                   \
  X(4, 8, 4, 2, 3, 1, 0) X(4, 8, 2, 2, 2, 1, 0) X(4, 8, 2, 2, 3, 1, 0) X(2, 8, 4, 2, 3, 1, 0)                   \
  X(4, 4, 4, 2, 3, 1, 0) X(2, 8, 2, 2, 3, 1, 0) X(4, 8, 4, 2, 2, 1, 5) X(4, 8, 2, 2, 2, 1, 5)                   \
  X(4, 8, 2, 2, 3, 1, 5)

bool mac_variant_ok(const MacShape &m) {
#define HC_MAC_OK(B_, C_, R_, G_, S_, D_, P_)                                                                 \
  if (m.bt == B_ && m.ct == C_ && m.rg == R_ && m.cg == G_ && m.depth == S_ && m.lds == D_ && m.pre == P_) \
    return true;
  HC_MAC_VARIANTS(HC_MAC_OK)
#undef HC_MAC_OK
  return false;
}

hipError_t launch_mac(const ConvGeom &g, const MacShape &m, const uint32_t *x, const uint32_t *w, uint32_t *y,
                      uint32_t B, const LimbConsts &c, const Twiddles &tw, hipStream_t st) {
  if (m.pre && g.N < 4096) return hipErrorInvalidValue;  // the epilogue's twiddle layout needs N >= 4096
#define HC_MAC_CASE(B_, C_, R_, G_, S_, D_, P_)                                                               \
  if (m.bt == B_ && m.ct == C_ && m.rg == R_ && m.cg == G_ && m.depth == S_ && m.lds == D_ && m.pre == P_) \
    return mac_t<B_, C_, R_, G_, S_, D_, P_>(g, x, w, y, B, c, tw, st);
  HC_MAC_VARIANTS(HC_MAC_CASE)
#undef HC_MAC_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_weight_scatter(const ConvGeom &g, const int8_t *f, uint32_t *w, const LimbConsts &c,
                                 hipStream_t st) {
  const size_t total = (size_t)g.c_out * g.c_in * g.f * g.f;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_weight_scatter, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, st, f, w, g, c);
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
