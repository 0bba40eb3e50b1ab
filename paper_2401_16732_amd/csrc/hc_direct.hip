// gfx950 kernel of Flash's own coefficient-domain convolution (Algorithm 1 as
// written: CMult of DRot-ed input ciphertexts, summed over taps and input
// channels), the alternative to the NTT path for layers whose c_n f^2 is
// small. It reads the int8 filters rather than the resident NTT-domain
// weights, so at one image it avoids the MAC's whole pass over W-hat.
//
// Output coefficient e of ciphertext i is
//   y_i[e] = sum_j sum_taps f[i][j][tap] * DRot(c_(g(j)), o_j + s_tap)[e],
// and DRot by k < N is a left shift with the sign flipped on wrap-around:
// DRot(c, k)[e] = c[e + k] for e + k < N, else -c[e + k - N] (the closed form of
// eq. drot proved in Appendix A). Products of a signed 8-bit weight and a
// 30-bit residue are summed exactly in signed 64 bits (the lazy reduction of
// "Employing Lazy Reduction in Convolution"), then reduced once.
#include "hc_device.h"

namespace hc {

// Grid: x = coefficient chunk of 256 (first the chunks of the extracted c0
// outputs, ho wo of them, then the N / 256 chunks of c1), y = group of IC
// output channels, z = b L + l. One thread per output coefficient, IC
// accumulators; the weights are wave-uniform (scalar loads).
template <int IC>
__global__ __launch_bounds__(256) void k_conv_direct(const uint32_t *__restrict__ ct, const int32_t *__restrict__ wt,
                                                      const uint32_t *__restrict__ mask, uint32_t *__restrict__ c0,
                                                      uint32_t *__restrict__ c1, ConvGeom g, uint32_t c0_chunks,
                                                      uint32_t wt_rows, DirectConsts d, LimbConsts c) {
  const uint32_t hw = g.ho * g.wo;
  const uint32_t b = blockIdx.z / g.L, l = blockIdx.z - b * g.L;
  const uint32_t i0 = blockIdx.y * IC;
  const bool comp0 = blockIdx.x < c0_chunks;
  uint32_t e, p = 0;
  if (comp0) {
    p = blockIdx.x * 256 + threadIdx.x;
    if (p >= hw) return;
    const uint32_t oy = p / g.wo, ox = p - oy * g.wo;
    e = g.s * oy * g.w_pad + g.s * ox;
  } else {
    e = (blockIdx.x - c0_chunks) * 256 + threadIdx.x;
  }
  const uint32_t comp = comp0 ? 0u : 1u;
  const uint32_t taps = g.f * g.f;
  int64_t acc[IC];
#pragma unroll
  for (int k = 0; k < IC; ++k) acc[k] = 0;
  for (uint32_t gi = 0; gi < g.G; ++gi) {
    const uint32_t *x = ct + (((size_t)b * g.G + gi) * 2 + comp) * g.L * g.N + (size_t)l * g.N;
    for (uint32_t slot = 0; slot < g.cn; ++slot) {
      const uint32_t j = gi * g.cn + slot;
      if (j >= g.c_in) break;
      const int32_t *wj = wt + ((size_t)i0 * g.c_in + j) * taps;
      for (uint32_t ky = 0; ky < g.f; ++ky)
        for (uint32_t kx = 0; kx < g.f; ++kx) {
          uint32_t idx = e + slot * g.F + ky * g.w_pad + kx;
          const bool wrap = idx >= g.N;
          if (wrap) idx -= g.N;
          const int32_t xv = (int32_t)x[idx];
          const int32_t sv = wrap ? -xv : xv;
          const uint32_t tap = ky * g.f + kx;
#pragma unroll
          for (int k = 0; k < IC; ++k) acc[k] += (int64_t)wj[(size_t)k * g.c_in * taps + tap] * sv;
        }
    }
  }
  const uint32_t q = c.q[l];
#pragma unroll
  for (int k = 0; k < IC; ++k) {
    const uint32_t i = i0 + k;
    if (i >= g.c_out || i >= wt_rows) break;
    // acc + bias is in [0, 2^57): one 64-bit fold to a canonical residue
    const uint32_t y = reduce64((uint64_t)(acc[k] + (int64_t)d.bias[l]), q, c.r2[l], c.r2_p[l], c.one_p[l]);
    if (comp0) {
      const uint32_t r = mask[((size_t)b * g.c_out + i) * hw + p];
      const uint32_t rc = r > c.t / 2 ? r - c.t + q : r;  // centred lift of r, taken mod q
      const uint32_t add = csub(shoup_lazy(rc, c.delta[l], c.delta_p[l], q), q);
      c0[(((size_t)b * g.c_out + i) * g.L + l) * hw + p] = csub(y + add, q);
    } else {
      c1[(((size_t)b * g.O + i) * g.L + l) * g.N + e] = y;
    }
  }
}

hipError_t launch_conv_direct(const ConvGeom &g, const uint32_t *ct, const int32_t *wt, uint32_t wt_rows,
                              const uint32_t *mask, uint32_t *c0, uint32_t *c1, uint32_t B, const DirectConsts &d,
                              const LimbConsts &c, hipStream_t st) {
  constexpr int IC = 16;
  if (g.tiled || g.N % 256 || wt_rows % IC || wt_rows < g.c_out) return hipErrorInvalidValue;
  const uint32_t c0_chunks = (g.ho * g.wo + 255) / 256;
  const uint64_t z = (uint64_t)B * g.L;
  const uint32_t ny = (g.c_out + IC - 1) / IC;
  if (B == 0) return hipSuccess;
  if (z > 65535 || ny > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_conv_direct<IC>), dim3(c0_chunks + g.N / 256, ny, (uint32_t)z), dim3(256), 0, st, ct, wt,
                     mask, c0, c1, g, c0_chunks, wt_rows, d, c);
  return hipGetLastError();
}

}  // namespace hc
