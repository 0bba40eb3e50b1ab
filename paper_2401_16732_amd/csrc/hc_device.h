// Device code shared by the gfx950 kernels of the homomorphic convolution (Flash, arXiv 2401.16732,
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
#pragma once
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
// a >= m ? a - m : a, for any a, m < 2^32: when a < m the wrapped a - m is
// above a, so the unsigned minimum picks a (one subtraction and one minimum,
// no compare writing the condition mask)
__device__ __forceinline__ uint32_t csub(uint32_t a, uint32_t m) { return min(a, a - m); }

// v_mad_u64_u32 (a * b + c over 64 bits) issues at the rate of a 32-bit
// multiply. Shoup's product a w - floor(a w' / 2^32) q only needs its low 32
// bits, which equal those of (a w) + floor(a w' / 2^32) (2^32 - q): written
// with two of these the subtraction disappears (3 multiplier operations, no
// simple one). Inline assembly, because the compiler narrows a 64-bit product
// whose high half is unused back to v_mul_lo_u32 + v_add_u32. The carry-out
// mask goes to a scalar pair that nothing reads. SB: b is wave-uniform (a
// scalar register); otherwise b is a per-lane value.
template <bool SB>
__device__ __forceinline__ uint64_t mul64(uint32_t a, uint32_t b) {
  uint64_t r, carry;
  if constexpr (SB)
    asm("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(r), "=s"(carry) : "v"(a), "s"(b));
  else
    asm("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(r), "=s"(carry) : "v"(a), "v"(b));
  return r;
}
// low 32 bits of hi * nq + c, nq wave-uniform
__device__ __forceinline__ uint32_t mad_lo_s(uint32_t hi, uint32_t nq, uint64_t c) {
  uint64_t r, carry;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(r), "=s"(carry) : "v"(hi), "s"(nq), "v"(c));
  return (uint32_t)r;
}
// a * b + c over 64 bits, b wave-uniform
__device__ __forceinline__ uint64_t mad64_s(uint32_t a, uint32_t b, uint64_t c) {
  uint64_t r, carry;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(r), "=s"(carry) : "v"(a), "s"(b), "v"(c));
  return r;
}
// shoup_lazy(a, w, wp, q) with nq = 2^32 - q (wave-uniform): the same value
template <bool SW>
__device__ __forceinline__ uint32_t shoup_mad(uint32_t a, uint32_t w, uint32_t wp, uint32_t nq) {
  const uint32_t hi = __umulhi(a, wp);
  return mad_lo_s(hi, nq, mul64<SW>(a, w));
}

// acc < 2^64 -> acc mod q, q < 2^30.
__device__ __forceinline__ uint32_t reduce64(uint64_t acc, uint32_t q, uint32_t r2, uint32_t r2p, uint32_t onep) {
  uint32_t hi = (uint32_t)(acc >> 32), lo = (uint32_t)acc;
  uint32_t r = shoup_lazy(hi, r2, r2p, q) + shoup_lazy(lo, 1u, onep, q);  // [0, 4q)
  r = csub(r, 2 * q);
  return csub(r, q);
}

// acc < 2^64 -> a value in [0, 2q) congruent to acc mod q (q < 2^30), for
// wave-uniform q and r2 = 2^32 mod q. With acc = hi 2^32 + lo, the value
// hi r2 + lo - (floor(hi r2p / 2^32) + floor(lo onep / 2^32)) q is the sum of
// two Shoup remainders, so it lies in [0, 4q) and is exact mod 2^32: the
// first v_mad_u64_u32 takes acc itself as its addend (its low word is lo),
// the second subtracts the quotients' multiple of q. Seven operations where
// the canonical reduce64 takes about twelve; every inverse-NTT input accepts
// [0, 2q).
__device__ __forceinline__ uint32_t reduce64_lazy(uint64_t acc, uint32_t q, uint32_t r2, uint32_t r2p,
                                                  uint32_t onep) {
  const uint32_t hi = (uint32_t)(acc >> 32), lo = (uint32_t)acc;
  const uint32_t Q = __umulhi(hi, r2p) + __umulhi(lo, onep);
  const uint32_t r = mad_lo_s(Q, 0u - q, mad64_s(hi, r2, acc));
  return csub(r, 2 * q);
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
// Waves per SIMD an NTT kernel is compiled for (the compiler then keeps its
// registers within 512 / waves): one polynomial per workgroup at 16
// coefficients per thread fits 64 registers (8 waves), at 32 fits 128 (4);
// other shapes keep the compiler's choice.
__host__ __device__ constexpr int ntt_min_waves(int elog, int m) {
  return m == 1 && elog == 4 ? 8 : m == 1 && elog == 5 ? 4 : 1;
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

// Twiddle sources of a pass over bits [LO, LO + EP): MemTw reads
// each twiddle from the table where it is used; RegTw holds the whole pass's
// twiddles in registers, loaded ahead of time (EarlyTws below).
template <int LOGN, int ELOG, int LO, int EP>
struct MemTw {
  const uint2 *tw;
  uint32_t tid;
  __device__ __forceinline__ uint2 operator()(int bb, int u) const {
    const StageTw<LOGN, ELOG, LO, EP> st(tw, tid, LO + bb);
    return st(u, LO + bb);
  }
};
template <int LOGN, int ELOG, int LO, int EP>
struct RegTw {
  // slot [bb][u] for u with bit bb clear; entries a pass never reads are
  // dropped. The two words are kept apart so that no register pair is tied up.
  uint32_t w[EP][1 << ELOG], wp[EP][1 << ELOG];
  __device__ __forceinline__ void load(const uint2 *tw, uint32_t tid) {
    const MemTw<LOGN, ELOG, LO, EP> m{tw, tid};
#pragma unroll
    for (int bb = 0; bb < EP; ++bb)
#pragma unroll
      for (int u = 0; u < (1 << ELOG); ++u)
        if (!(u & (1 << bb))) {
          const uint2 t = m(bb, u);
          w[bb][u] = t.x;
          wp[bb][u] = t.y;
        }
  }
  __device__ __forceinline__ uint2 operator()(int bb, int u) const { return make_uint2(w[bb][u], wp[bb][u]); }
};

// Forward (Cooley-Tukey, natural -> bit-reversed) stages of one pass.
// Stage s works on pairs (j, j + 2^(LOGN-1-s)) with twiddle psi^brv(2^s + j >> (LOGN - s)).
// tws(bb, u): twiddle {w, w'} of stage bit LO + bb for register slot u
// (index 2^s + (j >> (b + 1)), s = LOGN - 1 - b).
template <int LOGN, int ELOG, int LO, int EP, class TW>
__device__ __forceinline__ void fwd_pass(uint32_t (&v)[1 << ELOG], const TW &tws, uint32_t q) {
  constexpr int E = 1 << ELOG;
  constexpr bool kUniTw = LO >= 6;  // wave-uniform twiddles (scalar registers)
  const uint32_t q2 = 2 * q, nq = 0u - q;
#pragma unroll
  for (int bb = EP - 1; bb >= 0; --bb) {
    // butterflies side by side, one operation at a time (as in inv_pass);
    // pair k is (u, u + 2^bb), u = k with a zero inserted at bit bb
    uint32_t hi[E / 2];
#pragma unroll
    for (int k = 0; k < E / 2; ++k) {
      const int u = ((k >> bb) << (bb + 1)) | (k & ((1 << bb) - 1)), u2 = u | (1 << bb);
      hi[k] = __umulhi(v[u2], tws(bb, u).y);
    }
#pragma unroll
    for (int k = 0; k < E / 2; ++k) {
      const int u = ((k >> bb) << (bb + 1)) | (k & ((1 << bb) - 1)), u2 = u | (1 << bb);
      const uint32_t X = csub(v[u], q2);
      const uint32_t T = mad_lo_s(hi[k], nq, mul64<kUniTw>(v[u2], tws(bb, u).x));  // Shoup: in [0, 2q)
      v[u] = X + T;
      v[u2] = X - T + q2;
    }
  }
}

// Pruned stages keep only the outputs that wanted outputs depend on. With
// A = LOGN - PS (wanted outputs: index < 2^A), the sum a stage on bit b >= A
// leaves at index j is needed only if bits A..b of j are zero: going back
// from the last stage, each pruned stage frees one more index bit. The
// register part of j (gidx(0, u)) is known at compile time, so sums whose
// register part has such a bit set are not computed at all. (Testing the
// thread part too, to let whole waves skip a pass, costs the kernels a third
// more registers, and occupancy, for the branch.)
template <int LOGN, int ELOG, int LO, int EP, int PS>
__device__ __forceinline__ bool pruned_sum_needed(int u, int b) {
  const uint32_t mask = ((2u << b) - 1u) & ~((1u << (LOGN - PS)) - 1u);  // bits A..b
  return (gidx<LOGN, ELOG, LO, EP>(0, u) & mask) == 0;
}

// Inverse (Gentleman-Sande, bit-reversed -> natural) stages of one pass; the
// last stage (s = 0) also multiplies by N^-1, unless SC is false (inputs that
// already carry the factor N^-1: the convolution's weights are stored scaled
// by it, so its sums do), when it is an ordinary stage.
// Pruning: when only outputs below 2^(LOGN - PS) are wanted, every stage on a
// bit b >= LOGN - PS feeds wanted outputs from its lower (sum) half only - all
// wanted indices have those bits clear - so the difference half, with its
// twiddle multiply, is skipped there, and of the sums only those that wanted
// outputs depend on are computed (pruned_sum_needed). PS = 0 computes the
// full transform. PS is a compile-time constant, so no stage carries a
// run-time branch.
// M polynomials of one limb go through the stages together (v[m]): each
// twiddle is loaded once for all of them.
// tws(bb, u): twiddle {w, w'} of stage bit LO + bb for register slot u
// (MemTw, RegTw).
template <int LOGN, int ELOG, int LO, int EP, int PS, int M, bool SC = true, class TW>
__device__ __forceinline__ void inv_pass(uint32_t (&v)[M][1 << ELOG], const TW &tws, uint32_t q, uint32_t ninv,
                                         uint32_t ninvp, uint32_t ninvw, uint32_t ninvwp) {
  constexpr int E = 1 << ELOG;
  // twiddles of a pass starting at bit 6 or above are the same for a whole
  // wave (scalar registers)
  constexpr bool kUniTw = LO >= 6;
  const uint32_t q2 = 2 * q, nq = 0u - q;
#pragma unroll
  for (int bb = 0; bb < EP; ++bb) {
    const int b = LO + bb;
    const int s = LOGN - 1 - b;
    const bool sum_only = b >= LOGN - PS;
    // The stage's butterflies go side by side, one operation at a time, so
    // that independent instructions follow each other rather than each
    // butterfly's dependent chain (Shoup: a w - umulhi(a, w') q). Pair k
    // is (u, u + 2^bb) with u = k with a zero inserted at bit bb.
    if (s == 0 && SC) {
      // N^-1 on the sum; N^-1 psi^-brv(1) on the difference (or nothing: pruned)
      uint32_t a[M][E / 2], d[M][E / 2], ha[M][E / 2], hd[M][E / 2];
#pragma unroll
      for (int m = 0; m < M; ++m)
#pragma unroll
        for (int k = 0; k < E / 2; ++k) {
          const int u = ((k >> bb) << (bb + 1)) | (k & ((1 << bb) - 1)), u2 = u | (1 << bb);
          if (sum_only && !pruned_sum_needed<LOGN, ELOG, LO, EP, PS>(u, b)) continue;
          a[m][k] = v[m][u] + v[m][u2];
          if (!sum_only) d[m][k] = v[m][u] - v[m][u2] + q2;
        }
#pragma unroll
      for (int m = 0; m < M; ++m)
#pragma unroll
        for (int k = 0; k < E / 2; ++k) {
          const int u = ((k >> bb) << (bb + 1)) | (k & ((1 << bb) - 1));
          if (sum_only && !pruned_sum_needed<LOGN, ELOG, LO, EP, PS>(u, b)) continue;
          ha[m][k] = __umulhi(a[m][k], ninvp);
          if (!sum_only) hd[m][k] = __umulhi(d[m][k], ninvwp);
        }
#pragma unroll
      for (int m = 0; m < M; ++m)
#pragma unroll
        for (int k = 0; k < E / 2; ++k) {
          const int u = ((k >> bb) << (bb + 1)) | (k & ((1 << bb) - 1)), u2 = u | (1 << bb);
          if (sum_only && !pruned_sum_needed<LOGN, ELOG, LO, EP, PS>(u, b)) continue;
          v[m][u] = mad_lo_s(ha[m][k], nq, mul64<true>(a[m][k], ninv));
          if (!sum_only) v[m][u2] = mad_lo_s(hd[m][k], nq, mul64<true>(d[m][k], ninvw));
        }
    } else if (sum_only) {
#pragma unroll
      for (int m = 0; m < M; ++m)
#pragma unroll
        for (int k = 0; k < E / 2; ++k) {
          const int u = ((k >> bb) << (bb + 1)) | (k & ((1 << bb) - 1)), u2 = u | (1 << bb);
          if (!pruned_sum_needed<LOGN, ELOG, LO, EP, PS>(u, b)) continue;
          v[m][u] = csub(v[m][u] + v[m][u2], q2);
        }
    } else {
      uint32_t d[M][E / 2], hi[M][E / 2];
#pragma unroll
      for (int m = 0; m < M; ++m)
#pragma unroll
        for (int k = 0; k < E / 2; ++k) {
          const int u = ((k >> bb) << (bb + 1)) | (k & ((1 << bb) - 1)), u2 = u | (1 << bb);
          const uint32_t X = v[m][u], Y = v[m][u2];
          d[m][k] = X - Y + q2;
          v[m][u] = csub(X + Y, q2);
        }
#pragma unroll
      for (int m = 0; m < M; ++m)
#pragma unroll
        for (int k = 0; k < E / 2; ++k) {
          const int u = ((k >> bb) << (bb + 1)) | (k & ((1 << bb) - 1));
          hi[m][k] = __umulhi(d[m][k], tws(bb, u).y);
        }
#pragma unroll
      for (int m = 0; m < M; ++m)
#pragma unroll
        for (int k = 0; k < E / 2; ++k) {
          const int u = ((k >> bb) << (bb + 1)) | (k & ((1 << bb) - 1)), u2 = u | (1 << bb);
          v[m][u2] = mad_lo_s(hi[m][k], nq, mul64<kUniTw>(d[m][k], tws(bb, u).x));  // in [0, 2q)
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
    if constexpr (LO >= 6) {
      // wave-uniform twiddles: scalar loads ahead of the LDS reads (as in InvPasses)
      RegTw<LOGN, ELOG, LO, EP> t;
      t.load(tw, tid);
      __builtin_amdgcn_sched_barrier(0);
      lds_to_regs<LOGN, ELOG, LO, EP>(v, lds, tid);
      fwd_pass<LOGN, ELOG, LO, EP>(v, t, q);
    } else {
      lds_to_regs<LOGN, ELOG, LO, EP>(v, lds, tid);
      fwd_pass<LOGN, ELOG, LO, EP>(v, MemTw<LOGN, ELOG, LO, EP>{tw, tid}, q);
    }
  }
};
template <int LOGN, int ELOG>
struct FwdPasses<LOGN, ELOG, 0> {
  // pass 0 expects its inputs already in registers (loaded from global)
  static __device__ __forceinline__ void run(uint32_t (&v)[1 << ELOG], uint32_t *, uint32_t tid, const uint2 *tw,
                                             uint32_t q) {
    constexpr int LO = pass_lo_fwd(LOGN, ELOG, 0), EP = pass_bits(LOGN, ELOG, 0);
    fwd_pass<LOGN, ELOG, LO, EP>(v, MemTw<LOGN, ELOG, LO, EP>{tw, tid}, q);
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

// Twiddle sets for InvPasses: pass<K>() is the source for inverse pass K.
template <int LOGN, int ELOG, int PRE>
struct MemTws {
  const uint2 *tw;
  uint32_t tid;
  __device__ __forceinline__ const uint2 *table() const { return tw; }
  template <int K>
  __device__ __forceinline__ MemTw<LOGN, ELOG, inv_lo(LOGN, ELOG, PRE, K), inv_ep(LOGN, ELOG, PRE, K)> pass() const {
    return {tw, tid};
  }
};


// Twiddle set whose passes that start below bit 6 (twiddles vary across a
// wave: the first pass, and the second when it starts below bit 6) hold
// their twiddles in registers, loaded when the set is built: before the
// first LDS exchange, so that the second pass's loads are not issued behind
// a barrier and waited for right after it. Later passes read theirs where
// they are used (wave-uniform, scalar loads).
template <int LOGN, int ELOG, int PRE>
struct EarlyTws {
  static constexpr int NP = inv_np(LOGN, ELOG, PRE);
  static constexpr int LO0 = inv_lo(LOGN, ELOG, PRE, 0), EP0 = inv_ep(LOGN, ELOG, PRE, 0);
  static constexpr int LO1 = NP > 1 ? inv_lo(LOGN, ELOG, PRE, 1) : 0;
  static constexpr int EP1 = NP > 1 ? inv_ep(LOGN, ELOG, PRE, 1) : 1;
  static constexpr bool kReg0 = LO0 < 6, kReg1 = NP > 1 && LO1 < 6;
  const uint2 *tw;
  uint32_t tid;
  RegTw<LOGN, ELOG, LO0, EP0> t0;
  RegTw<LOGN, ELOG, LO1, EP1> t1;
  __device__ __forceinline__ EarlyTws(const uint2 *tw_, uint32_t tid_) : tw(tw_), tid(tid_) {
    if constexpr (kReg0) t0.load(tw, tid);
    if constexpr (kReg1) t1.load(tw, tid);
  }
  __device__ __forceinline__ const uint2 *table() const { return tw; }
  template <int K>
  __device__ __forceinline__ auto pass() const {
    if constexpr (K == 0 && kReg0) {
      return t0;
    } else if constexpr (K == 1 && kReg1) {
      return t1;
    } else {
      return MemTw<LOGN, ELOG, inv_lo(LOGN, ELOG, PRE, K), inv_ep(LOGN, ELOG, PRE, K)>{tw, tid};
    }
  }
};

template <int LOGN, int ELOG, int K, int PS, int M, int PRE, bool SC = true>
struct InvPasses {
  template <class TWS>
  static __device__ __forceinline__ void run(uint32_t (&v)[M][1 << ELOG], uint32_t *lds, uint32_t tid,
                                             const TWS &tws, uint32_t q, uint32_t a, uint32_t ap, uint32_t b,
                                             uint32_t bp) {
    constexpr int LO = inv_lo(LOGN, ELOG, PRE, K), EP = inv_ep(LOGN, ELOG, PRE, K);
    constexpr int PLO = inv_lo(LOGN, ELOG, PRE, K - 1), PEP = inv_ep(LOGN, ELOG, PRE, K - 1);
    InvPasses<LOGN, ELOG, K - 1, PS, M, PRE, SC>::run(v, lds, tid, tws, q, a, ap, b, bp);
#pragma unroll
    for (int m = 0; m < M; ++m) regs_to_lds<LOGN, ELOG, PLO, PEP>(v[m], lds + m * lds_words(LOGN), tid);
    __syncthreads();
    if constexpr (LO >= 6) {
      // wave-uniform twiddles: their scalar loads go out ahead of the pass's
      // LDS reads, so that the two latencies overlap rather than add up
      RegTw<LOGN, ELOG, LO, EP> t;
      t.load(tws.table(), tid);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int m = 0; m < M; ++m) lds_to_regs<LOGN, ELOG, LO, EP>(v[m], lds + m * lds_words(LOGN), tid);
      inv_pass<LOGN, ELOG, LO, EP, PS, M, SC>(v, t, q, a, ap, b, bp);
    } else {
#pragma unroll
      for (int m = 0; m < M; ++m) lds_to_regs<LOGN, ELOG, LO, EP>(v[m], lds + m * lds_words(LOGN), tid);
      inv_pass<LOGN, ELOG, LO, EP, PS, M, SC>(v, tws.template pass<K>(), q, a, ap, b, bp);
    }
  }
};
template <int LOGN, int ELOG, int PS, int M, int PRE, bool SC>
struct InvPasses<LOGN, ELOG, 0, PS, M, PRE, SC> {
  // pass 0 (bits [PRE, PRE + EP)) expects its inputs already in registers
  template <class TWS>
  static __device__ __forceinline__ void run(uint32_t (&v)[M][1 << ELOG], uint32_t *, uint32_t, const TWS &tws,
                                             uint32_t q, uint32_t a, uint32_t ap, uint32_t b, uint32_t bp) {
    constexpr int LO = inv_lo(LOGN, ELOG, PRE, 0), EP = inv_ep(LOGN, ELOG, PRE, 0);
    inv_pass<LOGN, ELOG, LO, EP, PS, M, SC>(v, tws.template pass<0>(), q, a, ap, b, bp);
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

// ---------------------------------------------------------------- inverse NTT kernels
// PS: top stages pruned (see inv_pass); 0 for the whole transform. M
// polynomials src[m] of one limb, LDS of M * lds_words(LOGN) words. PRE:
// stages on bits below PRE already done (the first pass then reads its
// coefficients with coalesced 4-byte loads: lanes map to the low bits).
// The first inverse pass's registers from global memory: with PRE = 0 the
// pass covers bits [0, EP), 2^EP consecutive words per group (16-byte
// loads); otherwise lanes map to the low bits (coalesced 4-byte loads).
template <int LOGN, int ELOG, int PRE>
__device__ __forceinline__ void load_first(uint32_t (&v)[1 << ELOG], const uint32_t *src, uint32_t tid) {
  if constexpr (PRE == 0) {
    load_low_pass<LOGN, ELOG, pass_bits(LOGN, ELOG, 0)>(v, src, tid);
  } else {
    constexpr int LO = inv_lo(LOGN, ELOG, PRE, 0), EP = inv_ep(LOGN, ELOG, PRE, 0);
    const uint32_t *sb = src + gidx<LOGN, ELOG, LO, EP>(tid, 0);
#pragma unroll
    for (int u = 0; u < (1 << ELOG); ++u) v[u] = sb[gidx<LOGN, ELOG, LO, EP>(0, u)];
  }
}

// The inverse passes over registers already loaded (load_first), with
// twiddles from tws: the result is in registers, laid out for the last pass.
// SC: whether the last stage multiplies by N^-1 (see inv_pass).
template <int LOGN, int ELOG, int PS, int M, int PRE, bool SC = true, class TWS>
__device__ __forceinline__ void intt_passes(uint32_t (&v)[M][1 << ELOG], uint32_t *lds, uint32_t tid,
                                            const LimbConsts &c, const TWS &tws, uint32_t l) {
  InvPasses<LOGN, ELOG, inv_np(LOGN, ELOG, PRE) - 1, PS, M, PRE, SC>::run(v, lds, tid, tws, c.q[l], c.ninv[l],
                                                                          c.ninv_p[l], c.ninvw[l], c.ninvw_p[l]);
}

// PS: top stages pruned (see inv_pass); 0 for the whole transform. M
// polynomials src[m] of one limb, LDS of M * lds_words(LOGN) words. PRE:
// stages on bits below PRE already done.
template <int LOGN, int ELOG, int PS, int M, int PRE, bool SC = true>
__device__ __forceinline__ void intt_core(const uint32_t *const (&src)[M], uint32_t (&v)[M][1 << ELOG],
                                          uint32_t *lds, uint32_t tid, const LimbConsts &c, const uint2 *tw,
                                          uint32_t l) {
#pragma unroll
  for (int m = 0; m < M; ++m) load_first<LOGN, ELOG, PRE>(v[m], src[m], tid);
  // ELOG 5 keeps the per-use loads: its first two passes' twiddles would
  // cost it occupancy
  if constexpr (ELOG <= 4) {
    const EarlyTws<LOGN, ELOG, PRE> tws(tw, tid);
    intt_passes<LOGN, ELOG, PS, M, PRE, SC>(v, lds, tid, c, tws, l);
  } else {
    intt_passes<LOGN, ELOG, PS, M, PRE, SC>(v, lds, tid, c, MemTws<LOGN, ELOG, PRE>{tw, tid}, l);
  }
}

}  // namespace hc
