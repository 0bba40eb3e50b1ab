// gfx950 kernels of the steps around the convolution: on the client side the
// offline encryptions of zero, direct encoding with online encryption
// (Algorithm 2) of a layer's input and BFV decryption (eq. bfv_dec); on the
// server side the x^2 + x protocol's PMult helpers (plaintext lift and
// addition) and its final combination.
// All of them are elementwise and bound by HBM traffic: dword accesses that
// are consecutive across a wave's lanes, 2-D grids (ciphertext or channel x
// chunk) so that no thread divides a 64-bit index. The ring product c1 * s of
// decryption is hc_ntt.hip's k_ring_mul: forward NTT, product by NTT(s) and
// inverse NTT in one pass over HBM.
#include "hc_device.h"

namespace hc {

// ---------------------------------------------------------------- encryption
// Activation index [b][j][y][x] (into a [B][c_in][h][w] array) that coefficient
// k of input ciphertext gi of image b holds under the direct-encoding layout:
// zero padding, c_n channels per ciphertext at offsets (j mod c_n) F, or row
// tiles with f - 1 halo rows when F > N; with client subsampling the encoded
// pixel (y, x) is [j][sub y][sub x]. kNone for padding and empty slots.
constexpr size_t kNone = ~(size_t)0;
__device__ __forceinline__ size_t encoded_index(const ConvGeom &g, const EncGeom &e, size_t b, uint32_t gi,
                                                uint32_t k) {
  uint32_t j, y, x;
  if (!g.tiled) {
    const uint32_t slot = k / g.F;
    j = gi * g.cn + slot;
    if (slot >= g.cn || j >= g.c_in) return kNone;
    const uint32_t pos = k - slot * g.F;
    y = pos / g.w_pad;
    x = pos - y * g.w_pad;
  } else {
    j = gi / g.T;
    const uint32_t tau = gi - j * g.T;
    const uint32_t yl = k / g.w_pad;
    if (yl >= e.rows_per_ct) return kNone;
    x = k - yl * g.w_pad;
    y = tau * g.r_o + yl;
    if (y >= e.h_pad) return kNone;
  }
  if (y < e.pad || x < e.pad) return kNone;
  const uint32_t ya = y - e.pad, xa = x - e.pad;
  if (ya >= e.h_enc || xa >= e.w_enc) return kNone;
  return ((b * g.c_in + j) * e.h + (size_t)ya * e.sub) * e.w + (size_t)xa * e.sub;
}

// Delta_l * (m mod q_l) for the centred plaintext value of m in [0, t)
// (m <= t/2: m itself; else m - t + q, which t < 2 q_l keeps in [0, q_l)).
__device__ __forceinline__ uint32_t delta_times(uint32_t m, const LimbConsts &c, uint32_t l) {
  const uint32_t q = c.q[l];
  const uint32_t mc = m > c.t / 2 ? m - c.t + q : m;
  return csub(shoup_lazy(mc, c.delta[l], c.delta_p[l], q), q);
}

// Grid: x = input ciphertext (b * G + gi), y = chunk of 1024 coefficients;
// each thread takes 4 coefficients 256 apart, so every access instruction of a
// wave covers 256 consecutive bytes. c0_l += Delta_l (m mod q_l) for the
// centred plaintext m in (-t/2, t/2], every limb.
__global__ __launch_bounds__(256) void k_encrypt_online(const uint32_t *__restrict__ act,
                                                         const uint32_t *__restrict__ ct0,
                                                         uint32_t *__restrict__ ct, ConvGeom g, EncGeom e,
                                                         uint32_t copy_c1, LimbConsts c) {
  const uint32_t ctn = blockIdx.x;
  const uint32_t b = ctn / g.G, gi = ctn - b * g.G;
  const uint32_t k0 = blockIdx.y * 1024 + threadIdx.x;
  uint32_t m[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const size_t idx = encoded_index(g, e, b, gi, k0 + 256 * j);
    m[j] = idx == kNone ? 0u : act[idx];
  }
  const size_t base = (size_t)ctn * 2 * g.L * g.N + k0;
  for (uint32_t l = 0; l < g.L; ++l) {
    const uint32_t q = c.q[l];
    const size_t w0 = base + (size_t)l * g.N, w1 = w0 + (size_t)g.L * g.N;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      ct[w0 + 256 * j] = csub(ct0[w0 + 256 * j] + delta_times(m[j], c, l), q);
      if (copy_c1) ct[w1 + 256 * j] = ct0[w1 + 256 * j];
    }
  }
}

// ---------------------------------------------------------------- x^2 + x protocol, server steps
// out[c][l][k] = centred(mult * p[c][k] mod t) mod q_l (p in [0, t), mult 1 or 2).
// Grid: x = plaintext, y = chunk of 256 coefficients.
__global__ __launch_bounds__(256) void k_lift_plain(const uint32_t *__restrict__ p, uint32_t *__restrict__ out,
                                                     uint32_t N, uint32_t mult, LimbConsts c) {
  const size_t cn = blockIdx.x;
  const uint32_t k = blockIdx.y * 256 + threadIdx.x;
  uint32_t v = p[cn * N + k];
  if (mult == 2) v = csub(2 * v, c.t);
  for (uint32_t l = 0; l < c.L; ++l)
    out[(cn * c.L + l) * N + k] = v > c.t / 2 ? v - c.t + c.q[l] : v;
}

// c0 of ct[c] += Delta_l (centred p[c][k] mod q_l): plaintext addition.
__global__ __launch_bounds__(256) void k_add_plain(uint32_t *__restrict__ ct, const uint32_t *__restrict__ p,
                                                    uint32_t N, LimbConsts c) {
  const size_t cn = blockIdx.x;
  const uint32_t k = blockIdx.y * 256 + threadIdx.x;
  const uint32_t m = p[cn * N + k];
  for (uint32_t l = 0; l < c.L; ++l) {
    const size_t w0 = ((cn * 2) * c.L + l) * N + k;
    ct[w0] = csub(ct[w0] + delta_times(m, c, l), c.q[l]);
  }
}

// ct = ct_x - ct_y + Delta * enc(r^2 - r + v mod t), direct encoding of the
// layer's input. Grid as k_encrypt_online.
__global__ __launch_bounds__(256) void k_act_combine(const uint32_t *ct_x, const uint32_t *ct_y,
                                                      const uint32_t *__restrict__ r, const uint32_t *__restrict__ v,
                                                      uint32_t *ct, ConvGeom g, EncGeom e, LimbConsts c) {
  const uint32_t ctn = blockIdx.x;
  const uint32_t b = ctn / g.G, gi = ctn - b * g.G;
  const uint32_t k0 = blockIdx.y * 1024 + threadIdx.x;
  uint32_t w[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const size_t idx = encoded_index(g, e, b, gi, k0 + 256 * j);
    if (idx == kNone) {
      w[j] = 0;
    } else {
      const uint64_t rr = r[idx];
      w[j] = (uint32_t)((rr * (rr ? rr - 1 : 0) + v[idx]) % c.t);
    }
  }
  const size_t base = (size_t)ctn * 2 * g.L * g.N + k0;
  for (uint32_t l = 0; l < g.L; ++l) {
    const uint32_t q = c.q[l];
    const size_t w0 = base + (size_t)l * g.N, w1 = w0 + (size_t)g.L * g.N;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t d0 = csub(ct_x[w0 + 256 * j] + q - ct_y[w0 + 256 * j], q);
      const uint32_t d1 = csub(ct_x[w1 + 256 * j] + q - ct_y[w1 + 256 * j], q);
      ct[w0 + 256 * j] = csub(d0 + delta_times(w[j], c, l), q);
      ct[w1 + 256 * j] = d1;
    }
  }
}

// Offline encryption of zero (private-key form): ct[c][0][l] = -(as[c][l] + e[c]) mod q_l,
// ct[c][1][l] = a[c][l], with as = a * s already computed and e small signed integers.
// Grid: x = ciphertext, y = chunk of 256 coefficients.
__global__ __launch_bounds__(256) void k_encrypt_zero(const uint32_t *__restrict__ a,
                                                       const uint32_t *__restrict__ as,
                                                       const int32_t *__restrict__ e, uint32_t *__restrict__ ct,
                                                       uint32_t N, LimbConsts c) {
  const size_t cn = blockIdx.x;
  const uint32_t k = blockIdx.y * 256 + threadIdx.x;
  const int32_t ek = e[cn * N + k];
  for (uint32_t l = 0; l < c.L; ++l) {
    const uint32_t q = c.q[l];
    // e mod q_l for |e| < q_l
    const uint32_t el = ek < 0 ? q - (uint32_t)(-(int64_t)ek) : (uint32_t)ek;
    const uint32_t sum = csub(as[(cn * c.L + l) * N + k] + csub(el, q), q);
    const size_t w0 = ((cn * 2) * c.L + l) * N + k;
    ct[w0] = sum == 0 ? 0 : q - sum;
    ct[w0 + (size_t)c.L * N] = a[(cn * c.L + l) * N + k];
  }
}

// ---------------------------------------------------------------- decryption
__global__ void k_gather_c1(const uint32_t *__restrict__ ct, uint32_t *__restrict__ c1, size_t n_ct, size_t ln) {
  const size_t total = n_ct * ln;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < total; id += stride)
    c1[id] = ct[(2 * (id / ln) + 1) * ln + id % ln];
}

// round(t v / q) mod t for the phase with residues v[0..L) (canonical).
__device__ __forceinline__ uint32_t decode_phase(const uint32_t (&v)[kMaxLimbs], const LimbConsts &c,
                                                 const DecodeConsts &d) {
  uint64_t whole = 0;                       // sum_l x_l a_l
  uint32_t f0 = 0, f1 = 0, f2 = 0, f3 = 0;  // sum_l x_l phi_l: 160 fraction bits in f0..f4,
  uint32_t f4 = 0, top = 0;                 // the integer part (< 2^32) in top
#pragma unroll
  for (uint32_t l = 0; l < (uint32_t)kMaxLimbs; ++l) {
    if (l < c.L) {
      const uint32_t q = c.q[l];
      const uint32_t x = csub(shoup_lazy(v[l], d.qt[l], d.qt_p[l], q), q);
      whole += (uint64_t)x * d.a[l];
      uint64_t p = (uint64_t)x * d.phi[l][0] + f0;
      f0 = (uint32_t)p;
      p = (uint64_t)x * d.phi[l][1] + f1 + (p >> 32);
      f1 = (uint32_t)p;
      p = (uint64_t)x * d.phi[l][2] + f2 + (p >> 32);
      f2 = (uint32_t)p;
      p = (uint64_t)x * d.phi[l][3] + f3 + (p >> 32);
      f3 = (uint32_t)p;
      p = (uint64_t)x * d.phi[l][4] + f4 + (p >> 32);
      f4 = (uint32_t)p;
      top += (uint32_t)(p >> 32);
    }
  }
  top += (uint32_t)(((uint64_t)f4 + 0x80000000u) >> 32);  // + 1/2, then floor
  return (uint32_t)((whole + top) % c.t);
}

// Grid: x = (b, i) output channel of an image, y = chunk of 256 output pixels.
__global__ __launch_bounds__(256) void k_decrypt_extracted(const uint32_t *__restrict__ c0_ext,
                                                            const uint32_t *__restrict__ c1s,
                                                            uint32_t *__restrict__ m, ConvGeom g, LimbConsts c,
                                                            DecodeConsts d) {
  const uint32_t hw = g.ho * g.wo;
  const uint32_t p = blockIdx.y * 256 + threadIdx.x;
  if (p >= hw) return;
  const uint32_t bi = blockIdx.x;  // b * c_out + i
  const uint32_t b = bi / g.c_out, i = bi - b * g.c_out;
  const uint32_t oy = p / g.wo, ox = p - oy * g.wo;
  const uint32_t Y = g.s * oy;
  const uint32_t tau = Y / g.r_o;
  const uint32_t e = (Y - tau * g.r_o) * g.w_pad + g.s * ox;
  const size_t o = (size_t)b * g.O + (size_t)i * g.T + tau;
  uint32_t v[kMaxLimbs] = {};
#pragma unroll
  for (uint32_t l = 0; l < (uint32_t)kMaxLimbs; ++l)
    if (l < c.L)
      v[l] = csub(c0_ext[((size_t)bi * g.L + l) * hw + p] + c1s[(o * g.L + l) * g.N + e], c.q[l]);
  m[(size_t)bi * hw + p] = decode_phase(v, c, d);
}

// Grid: x = ciphertext, y = chunk of 256 coefficients.
__global__ __launch_bounds__(256) void k_decrypt_full(const uint32_t *__restrict__ ct,
                                                       const uint32_t *__restrict__ c1s, uint32_t *__restrict__ m,
                                                       uint32_t N, LimbConsts c, DecodeConsts d) {
  const size_t cn = blockIdx.x;
  const uint32_t k = blockIdx.y * 256 + threadIdx.x;
  uint32_t v[kMaxLimbs] = {};
#pragma unroll
  for (uint32_t l = 0; l < (uint32_t)kMaxLimbs; ++l)
    if (l < c.L)
      v[l] = csub(ct[((cn * 2) * c.L + l) * N + k] + c1s[(cn * c.L + l) * N + k], c.q[l]);
  m[cn * N + k] = decode_phase(v, c, d);
}

// ---------------------------------------------------------------- launchers
namespace {
uint32_t grid_for(size_t total) {
  size_t blocks = (total + 255) / 256;
  return (uint32_t)(blocks > 65536 ? 65536 : blocks);
}
}  // namespace

// Grid x dimensions are below 2^31 (checked by the callers' sizes: B * G, B * c_out and
// ciphertext counts are 32-bit); y is at most N / 256 = 64.
hipError_t launch_encrypt_online(const ConvGeom &g, const EncGeom &e, const uint32_t *act, const uint32_t *ct0,
                                 uint32_t *ct, uint32_t B, bool copy_c1, const LimbConsts &c, hipStream_t st) {
  const uint64_t n_ct = (uint64_t)B * g.G;
  if (n_ct == 0) return hipSuccess;
  if (n_ct >= (1ull << 31) || g.N % 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_encrypt_online, dim3((uint32_t)n_ct, g.N / 1024), dim3(256), 0, st, act, ct0, ct, g, e,
                     copy_c1 ? 1u : 0u, c);
  return hipGetLastError();
}
hipError_t launch_lift_plain(const uint32_t *p, uint32_t *out, size_t n, uint32_t N, uint32_t mult,
                             const LimbConsts &c, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (n >= (1ull << 31) || N % 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lift_plain, dim3((uint32_t)n, N / 256), dim3(256), 0, st, p, out, N, mult, c);
  return hipGetLastError();
}
hipError_t launch_add_plain(uint32_t *ct, const uint32_t *p, size_t n, uint32_t N, const LimbConsts &c,
                            hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (n >= (1ull << 31) || N % 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_add_plain, dim3((uint32_t)n, N / 256), dim3(256), 0, st, ct, p, N, c);
  return hipGetLastError();
}
hipError_t launch_act_combine(const ConvGeom &g, const EncGeom &e, const uint32_t *ct_x, const uint32_t *ct_y,
                              const uint32_t *r, const uint32_t *v, uint32_t *ct, uint32_t B, const LimbConsts &c,
                              hipStream_t st) {
  const uint64_t n_ct = (uint64_t)B * g.G;
  if (n_ct == 0) return hipSuccess;
  if (n_ct >= (1ull << 31) || g.N % 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_act_combine, dim3((uint32_t)n_ct, g.N / 1024), dim3(256), 0, st, ct_x, ct_y, r, v, ct, g, e,
                     c);
  return hipGetLastError();
}
hipError_t launch_encrypt_zero(const uint32_t *a, const uint32_t *as, const int32_t *e, uint32_t *ct, size_t n_ct,
                               uint32_t N, const LimbConsts &c, hipStream_t st) {
  if (n_ct == 0) return hipSuccess;
  if (n_ct >= (1ull << 31) || N % 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_encrypt_zero, dim3((uint32_t)n_ct, N / 256), dim3(256), 0, st, a, as, e, ct, N, c);
  return hipGetLastError();
}
hipError_t launch_gather_c1(const uint32_t *ct, uint32_t *c1, size_t n_ct, uint32_t L, uint32_t N, hipStream_t st) {
  const size_t ln = (size_t)L * N;
  if (n_ct * ln == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_c1, dim3(grid_for(n_ct * ln)), dim3(256), 0, st, ct, c1, n_ct, ln);
  return hipGetLastError();
}
hipError_t launch_decrypt_extracted(const ConvGeom &g, const uint32_t *c0_ext, const uint32_t *c1s, uint32_t *m,
                                    uint32_t B, const LimbConsts &c, const DecodeConsts &d, hipStream_t st) {
  const uint64_t rows = (uint64_t)B * g.c_out, hw = (uint64_t)g.ho * g.wo;
  if (rows == 0 || hw == 0) return hipSuccess;
  if (rows >= (1ull << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_decrypt_extracted, dim3((uint32_t)rows, (uint32_t)((hw + 255) / 256)), dim3(256), 0, st,
                     c0_ext, c1s, m, g, c, d);
  return hipGetLastError();
}
hipError_t launch_decrypt_full(const uint32_t *ct, const uint32_t *c1s, uint32_t *m, size_t n_ct, uint32_t N,
                               const LimbConsts &c, const DecodeConsts &d, hipStream_t st) {
  if (n_ct == 0) return hipSuccess;
  if (n_ct >= (1ull << 31) || N % 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_decrypt_full, dim3((uint32_t)n_ct, N / 256), dim3(256), 0, st, ct, c1s, m, N, c, d);
  return hipGetLastError();
}

}  // namespace hc
