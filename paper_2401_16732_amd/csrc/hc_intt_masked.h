// The masked inverse NTT (A4 + A5) and its launch dispatch for one ring size.
// Its template instances are many (thread shape x pruned stages x
// polynomials per workgroup x stages done by the MAC), so they are compiled
// in one object per ring size: hc_intt_masked_<logn>.hip instantiates
// intt_masked_logn<LOGN>; the other objects only see the declaration.
#pragma once
#include "hc_device.h"

namespace hc {

template <int LOGN>
hipError_t intt_masked_logn(const ConvGeom &g, uint32_t elog, uint32_t npw, uint32_t pre, const uint32_t *y,
                            const uint32_t *m, uint32_t *c0, uint32_t *c1, uint32_t B, const LimbConsts &c,
                            const Twiddles &tw, const OutPtrs &out, hipStream_t st, bool c1_only);

#ifdef HC_INTT_MASKED_IMPL
// Output and mask buffers are global memory; table entries are plain
// integers, so their pointers are cast to the global address space (vector
// global accesses rather than flat ones, which also count as LDS accesses).
using gu32 = __attribute__((address_space(1))) uint32_t;

// Masked mode over Yhat [B][O][2][L][N]: c1 polynomials are written whole to
// c1_out [B][O][L][N]; c0 polynomials get the server mask added at the valid
// output coefficients, which are gathered into c0_ext [B][c_out][L][ho][wo].
// With pointer tables (out.n > 0) image b's mask, c0_ext and c1_out are
// separate buffers (out.mask[b], out.c0[b], out.c1[b]) laid out as for B = 1.
// PS: top stages of the c0 transform that are pruned (2^(LOGN - PS) must
// exceed every extracted coefficient index); c1 is always transformed whole.
// M: polynomials per workgroup, those of M consecutive (image, output
// ciphertext) indices bo with the same half p and limb l; workgroup w is
// ((pair 2 + p) L + l), bo = pair M + m, or (pair L + l) with p = 1 in the
// C1O form (c1 only; c0 finished elsewhere). Slots past B O compute a copy of
// slot 0 and store nothing. PRE: the stages on index bits below PRE were done
// by the multiply-accumulate (Yhat holds their output). Yhat carries the
// factor N^-1 already (the weights are stored scaled by it), so the last stage
// does not multiply by it.
template <int LOGN, int ELOG, int PS, int M, int PRE, bool C1O = false>
__global__ __launch_bounds__(1 << (LOGN - ELOG)) __attribute__((amdgpu_waves_per_eu(ntt_min_waves(ELOG, M)))) void k_intt_masked(const uint32_t *yhat, const uint32_t *mask,
                                                                     uint32_t *c0_ext, uint32_t *c1_out, ConvGeom g,
                                                                     uint32_t B, LimbConsts c, Twiddles tws,
                                                                     OutPtrs out) {
  constexpr int N = 1 << LOGN, E = 1 << ELOG, NT = 1 << (LOGN - ELOG), NP = inv_np(LOGN, ELOG, PRE);
  __shared__ uint32_t lds[M * lds_words(LOGN)];
  const uint32_t tid = threadIdx.x;
  const uint32_t wg = blockIdx.x;
  const uint32_t l = wg % g.L;
  const uint32_t p = C1O ? 1u : (wg / g.L) % 2;
  const size_t pair = wg / ((C1O ? 1u : 2u) * g.L);
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
    intt_core<LOGN, ELOG, 0, M, PRE, false>(src, v, lds, tid, c, tw, l);
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (!valid[m]) continue;
      const uint32_t o = (uint32_t)(bo[m] % g.O);
      const size_t b = bo[m] / g.O;
      gu32 *dst = out.n ? (gu32 *)out.c1[b] + ((size_t)o * g.L + l) * N : (gu32 *)c1_out + (bo[m] * g.L + l) * (size_t)N;
      gu32 *db = dst + gidx<LOGN, ELOG, LO, EP>(tid, 0);
#pragma unroll
      for (int u = 0; u < E; ++u) db[gidx<LOGN, ELOG, LO, EP>(0, u)] = csub(v[m][u], q);
    }
    return;
  }
  // c0 needs only its extracted coefficients
  intt_core<LOGN, ELOG, PS, M, PRE, false>(src, v, lds, tid, c, tw, l);
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
    const gu32 *mrow = out.n ? (const gu32 *)out.mask[b] + i * hw : (const gu32 *)mask + (b * g.c_out + i) * hw;
    gu32 *orow = out.n ? (gu32 *)out.c0[b] + ((size_t)i * g.L + l) * hw
                       : (gu32 *)c0_ext + ((b * g.c_out + i) * g.L + l) * hw;
    // Output idx of the tile (row oy0 + idx / wo, column idx % wo) is word
    // idx of the mask and output rows from row oy0, and coefficient
    // e = s w_pad (idx / wo) + s (idx % wo) of the polynomial (s oy0 is the
    // tile's first input row, tau r_o). A thread's outputs idx = tid + j NT
    // step their (row, column) by (NT / wo, NT % wo) with one carry, so no
    // division per output; their mask words are loaded U at a time, before
    // any of them is used.
    constexpr int U = 4;
    const gu32 *mr = mrow + (size_t)oy0 * g.wo;
    gu32 *orr = orow + (size_t)oy0 * g.wo;
    const uint32_t dy = NT / g.wo, dx = NT % g.wo, sw = g.s * g.w_pad;
    uint32_t ry = tid / g.wo, ox = tid % g.wo;
    for (uint32_t idx = tid; idx < count; idx += U * NT) {
      uint32_t rv[U];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const uint32_t ij = idx + j * NT;
        rv[j] = ij < count ? mr[ij] : 0u;
      }
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const uint32_t ij = idx + j * NT;
        if (ij < count) {
          const uint32_t e = sw * ry + g.s * ox;
          const uint32_t rc = rv[j] > half ? rv[j] - t + q : rv[j];  // centred lift of r, taken mod q
          const uint32_t add = csub(shoup_lazy(rc, dl, dlp, q), q);
          orr[ij] = csub(csub(lm[lpad(e)], q) + add, q);
        }
        ox += dx;
        ry += dy;
        if (ox >= g.wo) ox -= g.wo, ++ry;
      }
    }
  }
}

template <int LOGN, int ELOG, int PS, int M, int PRE>
static hipError_t invm_ps(const ConvGeom &g, const uint32_t *y, const uint32_t *m, uint32_t *c0, uint32_t *c1,
                          uint32_t B, const LimbConsts &c, const Twiddles &tw, const OutPtrs &out, hipStream_t st,
                          bool c1_only) {
  const size_t nbo = (size_t)B * g.O;
  const size_t nwg = (nbo + M - 1) / M * (c1_only ? 1 : 2) * g.L;
  if (nwg == 0) return hipSuccess;
  if (c1_only) {
    if constexpr (PS == 0 && PRE == 0)
      hipLaunchKernelGGL((k_intt_masked<LOGN, ELOG, 0, M, 0, true>), dim3((uint32_t)nwg), dim3(1 << (LOGN - ELOG)), 0,
                         st, y, m, c0, c1, g, B, c, tw, out);
    else
      return hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((k_intt_masked<LOGN, ELOG, PS, M, PRE>), dim3((uint32_t)nwg), dim3(1 << (LOGN - ELOG)), 0, st,
                       y, m, c0, c1, g, B, c, tw, out);
  }
  return hipGetLastError();
}
template <int LOGN, int ELOG, int M, int PRE>
static hipError_t invm_pm(const ConvGeom &g, const uint32_t *y, const uint32_t *m, uint32_t *c0, uint32_t *c1,
                          uint32_t B, const LimbConsts &c, const Twiddles &tw, const OutPtrs &out, hipStream_t st,
                          bool c1_only) {
  if (c1_only) return invm_ps<LOGN, ELOG, 0, M, PRE>(g, y, m, c0, c1, B, c, tw, out, st, true);
  const int ps = LOGN - (int)g.prune_bits;
  if (ps >= 7) return invm_ps<LOGN, ELOG, 7, M, PRE>(g, y, m, c0, c1, B, c, tw, out, st, c1_only);
  if (ps >= 5) return invm_ps<LOGN, ELOG, 5, M, PRE>(g, y, m, c0, c1, B, c, tw, out, st, c1_only);
  if (ps >= 3) return invm_ps<LOGN, ELOG, 3, M, PRE>(g, y, m, c0, c1, B, c, tw, out, st, c1_only);
  if (ps >= 2) return invm_ps<LOGN, ELOG, 2, M, PRE>(g, y, m, c0, c1, B, c, tw, out, st, c1_only);
  if (ps >= 1) return invm_ps<LOGN, ELOG, 1, M, PRE>(g, y, m, c0, c1, B, c, tw, out, st, c1_only);
  return invm_ps<LOGN, ELOG, 0, M, PRE>(g, y, m, c0, c1, B, c, tw, out, st, c1_only);
}
// Pruning fewer stages than allowed is always exact: take the largest
// instantiated count not above LOGN - prune_bits. Two polynomials per
// workgroup exist for ELOG <= 4 (the register and LDS budgets of ELOG 5);
// the forms that start at bit kMacPre exist for LOGN >= 12.
template <int LOGN, int ELOG>
static hipError_t invm_t(const ConvGeom &g, uint32_t npw, uint32_t pre, const uint32_t *y, const uint32_t *m,
                         uint32_t *c0, uint32_t *c1, uint32_t B, const LimbConsts &c, const Twiddles &tw,
                         const OutPtrs &out, hipStream_t st, bool c1_only) {
  if (pre == 0) {
    if (npw == 1) return invm_pm<LOGN, ELOG, 1, 0>(g, y, m, c0, c1, B, c, tw, out, st, c1_only);
    if constexpr (ELOG <= 4) {
      if (npw == 2) return invm_pm<LOGN, ELOG, 2, 0>(g, y, m, c0, c1, B, c, tw, out, st, c1_only);
    }
  }
  if constexpr (LOGN >= 12) {
    if (pre == kMacPre) {
      if (npw == 1) return invm_pm<LOGN, ELOG, 1, kMacPre>(g, y, m, c0, c1, B, c, tw, out, st, c1_only);
      if constexpr (ELOG <= 4) {
        if (npw == 2) return invm_pm<LOGN, ELOG, 2, kMacPre>(g, y, m, c0, c1, B, c, tw, out, st, c1_only);
      }
    }
  }
  return hipErrorInvalidValue;
}

template <int LOGN>
hipError_t intt_masked_logn(const ConvGeom &g, uint32_t elog, uint32_t npw, uint32_t pre, const uint32_t *y,
                            const uint32_t *m, uint32_t *c0, uint32_t *c1, uint32_t B, const LimbConsts &c,
                            const Twiddles &tw, const OutPtrs &out, hipStream_t st, bool c1_only) {
  if constexpr (LOGN <= 11) {
    if (elog == 3) return invm_t<LOGN, 3>(g, npw, pre, y, m, c0, c1, B, c, tw, out, st, c1_only);
    if (elog == 4) return invm_t<LOGN, 4>(g, npw, pre, y, m, c0, c1, B, c, tw, out, st, c1_only);
  } else if constexpr (LOGN <= 13) {
    if (elog == 3) return invm_t<LOGN, 3>(g, npw, pre, y, m, c0, c1, B, c, tw, out, st, c1_only);
    if (elog == 4) return invm_t<LOGN, 4>(g, npw, pre, y, m, c0, c1, B, c, tw, out, st, c1_only);
    if (elog == 5) return invm_t<LOGN, 5>(g, npw, pre, y, m, c0, c1, B, c, tw, out, st, c1_only);
  } else {
    if (elog == 4) return invm_t<LOGN, 4>(g, npw, pre, y, m, c0, c1, B, c, tw, out, st, c1_only);
    if (elog == 5) return invm_t<LOGN, 5>(g, npw, pre, y, m, c0, c1, B, c, tw, out, st, c1_only);
  }
  return hipErrorInvalidValue;
}
#endif

}  // namespace hc
