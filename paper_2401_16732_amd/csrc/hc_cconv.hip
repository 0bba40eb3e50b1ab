// gfx950 kernels of the conventional convolution (batch encoding, HRot with
// key switching, PMult): the section "Conventional Convolution" and the HRot
// procedure of "Background: Homomorphic Encryption" (eq. keySwitching), built
// for comparison with the DRot path. Everything stays in the NTT domain
// between the input's forward transform and the output's inverse transform:
// the automorphism x -> x^g permutes NTT-domain values, key switching and
// PMult are pointwise.
#include "hc_device.h"

namespace hc {

// Index of the evaluation point omega_k^g among the forward NTT's outputs
// (omega_k = psi^(2 brv(k) + 1)): NTT(a(x^g))[k] = NTT(a)[galois_index(k, g)].
__device__ __forceinline__ uint32_t galois_index(uint32_t k, uint32_t g, uint32_t logn) {
  const uint32_t mask2n = (2u << logn) - 1u;
  const uint32_t e = 2u * (__builtin_bitreverse32(k) >> (32 - logn)) + 1u;  // odd exponent of omega_k
  const uint32_t eg = (e * g) & mask2n;
  return __builtin_bitreverse32((eg - 1u) >> 1) >> (32 - logn);
}

// dig[c][l D + d][l'][k] = bits [T d, T d + T) of c1 of ciphertext c, limb l,
// coefficient k, for every limb l' (a value below 2^T is the same residue in
// every limb). ct: [n_ct][2][L][N] coefficient domain. Grid (n_ct * L * D, N / 256).
__global__ __launch_bounds__(256) void k_cc_digits(const uint32_t *__restrict__ ct, uint32_t *__restrict__ dig,
                                                   uint32_t N, uint32_t L, uint32_t T, uint32_t D) {
  const uint32_t LD = L * D;
  const size_t cj = blockIdx.x;  // (ciphertext, digit)
  const size_t c = cj / LD;
  const uint32_t j = (uint32_t)(cj % LD), l = j / D, d = j % D;
  const uint32_t k = blockIdx.y * 256 + threadIdx.x;
  const uint32_t v = (ct[((c * 2 + 1) * L + l) * N + k] >> (T * d)) & ((1u << T) - 1u);
  uint32_t *o = dig + (c * LD + j) * (size_t)L * N + k;
  for (uint32_t lp = 0; lp < L; ++lp) o[(size_t)lp * N] = v;
}

// Key switching after the automorphism, in the NTT domain, for ciphertext c
// and rotation r with Galois element gal[r]:
//   out0[k] = x0[pi(k)] + sum_i dig_i[pi(k)] key[r][i][0][k]
//   out1[k] = sum_i dig_i[pi(k)] key[r][i][1][k]
// (pi = galois_index), or out = x (no key switch) when gal[r] = 1. Sums are
// 64-bit, folded (hi 2^32 + lo) every 8 terms, reduced once.
// xh [n_ct][2][L][N], dh [n_ct][LD][L][N], keys [R][LD][2][L][N], out [n_ct][R][2][L][N].
// Grid (n_ct * R * L, N / 256).
__global__ __launch_bounds__(256) void k_cc_keyswitch(const uint32_t *__restrict__ xh, const uint32_t *__restrict__ dh,
                                                      const uint32_t *__restrict__ keys,
                                                      const uint32_t *__restrict__ gal, uint32_t *__restrict__ out,
                                                      uint32_t R, uint32_t LD, uint32_t logn, LimbConsts c) {
  const uint32_t N = 1u << logn, L = c.L;
  const size_t id = blockIdx.x;
  const uint32_t l = (uint32_t)(id % L);
  const uint32_t r = (uint32_t)((id / L) % R);
  const size_t ci = id / ((size_t)L * R);
  const uint32_t k = blockIdx.y * 256 + threadIdx.x;
  const uint32_t g = gal[r];
  const size_t LN = (size_t)L * N;
  const uint32_t *x0 = xh + (ci * 2) * LN + (size_t)l * N;
  uint32_t *o = out + ((ci * R + r) * 2) * LN + (size_t)l * N + k;
  if (g == 1u) {
    o[0] = x0[k];
    o[LN] = x0[LN + k];
    return;
  }
  const uint32_t q = c.q[l], r2 = c.r2[l];
  const uint32_t pk = galois_index(k, g, logn);
  const uint32_t *dd = dh + ci * LD * LN + (size_t)l * N + pk;
  const uint32_t *kk = keys + (size_t)r * LD * 2 * LN + (size_t)l * N + k;
  uint64_t a0 = x0[pk], a1 = 0;
  for (uint32_t i = 0; i < LD; ++i) {
    const uint64_t dv = dd[(size_t)i * LN];
    a0 += dv * kk[(size_t)i * 2 * LN];
    a1 += dv * kk[(size_t)i * 2 * LN + LN];
    if ((i & 7u) == 7u) {
      a0 = (uint64_t)(uint32_t)(a0 >> 32) * r2 + (uint32_t)a0;
      a1 = (uint64_t)(uint32_t)(a1 >> 32) * r2 + (uint32_t)a1;
    }
  }
  o[0] = reduce64(a0, q, r2, c.r2_p[l], c.one_p[l]);
  o[LN] = reduce64(a1, q, r2, c.r2_p[l], c.one_p[l]);
}

// Plaintext slot values of the weights for plaintexts P = p0 .. p0 + gridDim.x
// - 1, P = (o_g G_in + g) R + rot, written in the batch encoding's slot order
// (slot k at psi^(2 brv(k) + 1)), ready for the inverse transform modulo t:
// slot (row r, column c) is the point psi^(+-3^c) (pow3[c] = 3^c mod 2N) and
// holds f[o][j][ky][kx] mod t when output pixel (y, x) of block k = c / bsz
// reads a pixel inside the image, else 0 (the layout of oracle/hrot.CLayout).
// rot_tab: [R][4] = (swap, d, ky, kx). filt: int8 [c_out][c_in][f][f].
// Grid (n_pt, N / 256).
__global__ __launch_bounds__(256) void k_cc_weight_slots(const int8_t *__restrict__ filt,
                                                         const uint32_t *__restrict__ rot_tab,
                                                         const uint32_t *__restrict__ pow3, uint32_t *__restrict__ z,
                                                         CcGeom cg, size_t p0, uint32_t t) {
  const size_t P = p0 + blockIdx.x;
  const uint32_t rot = (uint32_t)(P % cg.R);
  const size_t og_g = P / cg.R;
  const uint32_t g = (uint32_t)(og_g % cg.g_in), o_g = (uint32_t)(og_g / cg.g_in);
  const uint32_t idx = blockIdx.y * 256 + threadIdx.x;  // slot in row-major rotation order
  const uint32_t half = cg.N / 2;
  const uint32_t row = idx / half, col = idx % half;
  const uint32_t swap = rot_tab[rot * 4], d = rot_tab[rot * 4 + 1], ky = rot_tab[rot * 4 + 2],
                 kx = rot_tab[rot * 4 + 3];
  uint32_t val = 0;
  const uint32_t blk = col / cg.bsz, pos = col % cg.bsz;
  if (pos < cg.h * cg.w) {
    const uint32_t y = pos / cg.w, x = pos % cg.w;
    const uint32_t o = o_g * cg.c_n + row * cg.c_r + blk;
    const uint32_t j = g * cg.c_n + (row ^ swap) * cg.c_r + (blk + d) % cg.c_r;
    const int sy = (int)y + (int)ky - (int)cg.p, sx = (int)x + (int)kx - (int)cg.p;
    if (o < cg.c_out && j < cg.c_in && sy >= 0 && sy < (int)cg.h && sx >= 0 && sx < (int)cg.w) {
      const int fv = filt[(((size_t)o * cg.c_in + j) * cg.f + ky) * cg.f + kx];
      val = fv < 0 ? t - (uint32_t)(-fv) : (uint32_t)fv;
    }
  }
  const uint32_t e = row == 0 ? pow3[col] : (2u * cg.N - pow3[col]);
  const uint32_t kb = __builtin_bitreverse32((e - 1u) >> 1) >> (32 - cg.logn);
  z[(size_t)blockIdx.x * cg.N + kb] = val;
}

// Rotation-order slots <-> the batch encoding's slot order, for n vectors of N:
// dir 0: out[v][brv((e(r, c) - 1) / 2)] = in[v][r N/2 + c]; dir 1: the inverse.
// Grid (n, N / 256).
__global__ __launch_bounds__(256) void k_cc_slot_perm(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                      const uint32_t *__restrict__ pow3, uint32_t logn, int dir) {
  const uint32_t N = 1u << logn, half = N / 2;
  const size_t v = blockIdx.x;
  const uint32_t idx = blockIdx.y * 256 + threadIdx.x;
  const uint32_t row = idx / half, col = idx % half;
  const uint32_t e = row == 0 ? pow3[col] : (2u * N - pow3[col]);
  const uint32_t kb = __builtin_bitreverse32((e - 1u) >> 1) >> (32 - logn);
  if (dir == 0)
    out[v * N + kb] = in[v * N + idx];
  else
    out[v * N + idx] = in[v * N + kb];
}

// Switching keys in the NTT domain from NTT(a_i), NTT(e_i) and NTT(s):
//   key[r][i][0][l][k] = eh[r][i][l][k] - ah[r][i][l][k] sh[l][k] + [l = l_i] 2^(T d_i) sh[l][pi_r(k)]
//   key[r][i][1][l][k] = ah[r][i][l][k]
// for digit i = (l_i, d_i) = (i / D, i % D) (the CRT weight of digit i is
// 2^(T d_i) in limb l_i and 0 in the others). Grid (R * LD * L, N / 256).
__global__ __launch_bounds__(256) void k_cc_keygen(const uint32_t *__restrict__ ah, const uint32_t *__restrict__ eh,
                                                   const uint32_t *__restrict__ sh, const uint32_t *__restrict__ gal,
                                                   uint32_t *__restrict__ keys, uint32_t LD, uint32_t D, uint32_t T,
                                                   uint32_t logn, LimbConsts c) {
  const uint32_t N = 1u << logn, L = c.L;
  const size_t id = blockIdx.x;
  const uint32_t l = (uint32_t)(id % L);
  const size_t ri = id / L;  // r LD + i
  const uint32_t i = (uint32_t)(ri % LD);
  const uint32_t r = (uint32_t)(ri / LD);
  const uint32_t k = blockIdx.y * 256 + threadIdx.x;
  const uint32_t q = c.q[l];
  const size_t LN = (size_t)L * N;
  const uint32_t a = ah[ri * LN + (size_t)l * N + k];
  uint64_t acc = (uint64_t)eh[ri * LN + (size_t)l * N + k] + (uint64_t)(q - a) * sh[(size_t)l * N + k];
  if (i / D == l) {
    uint64_t wpow = 1;
    for (uint32_t b = 0; b < T * (i % D); ++b) wpow = (wpow * 2) % q;
    acc += wpow * sh[(size_t)l * N + galois_index(k, gal[r], logn)];
  }
  keys[(ri * 2) * LN + (size_t)l * N + k] = (uint32_t)(acc % q);
  keys[(ri * 2 + 1) * LN + (size_t)l * N + k] = a;
}

// e [n][N] int32 (|e| < q_l) -> residues [n][L][N]. Grid (n, N / 256).
__global__ __launch_bounds__(256) void k_cc_lift_signed(const int32_t *__restrict__ e, uint32_t *__restrict__ out,
                                                        uint32_t N, LimbConsts c) {
  const size_t v = blockIdx.x;
  const uint32_t k = blockIdx.y * 256 + threadIdx.x;
  const int32_t x = e[v * N + k];
  for (uint32_t l = 0; l < c.L; ++l) out[(v * c.L + l) * N + k] = x < 0 ? c.q[l] - (uint32_t)(-x) : (uint32_t)x;
}

// ---------------------------------------------------------------- launchers
static bool grid_ok(size_t gx, uint32_t N) { return gx > 0 && gx < (1ull << 31) && N % 256 == 0; }

hipError_t launch_cc_digits(const uint32_t *ct, uint32_t *dig, size_t n_ct, uint32_t N, uint32_t L, uint32_t T,
                            uint32_t D, hipStream_t st) {
  const size_t gx = n_ct * L * D;
  if (n_ct == 0) return hipSuccess;
  if (!grid_ok(gx, N) || T == 0 || T * D < 30 || T > 16) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cc_digits, dim3((uint32_t)gx, N / 256), dim3(256), 0, st, ct, dig, N, L, T, D);
  return hipGetLastError();
}

hipError_t launch_cc_keyswitch(const uint32_t *xh, const uint32_t *dh, const uint32_t *keys, const uint32_t *gal,
                               uint32_t *out, size_t n_ct, uint32_t R, uint32_t LD, uint32_t logn,
                               const LimbConsts &c, hipStream_t st) {
  const uint32_t N = 1u << logn;
  const size_t gx = n_ct * R * c.L;
  if (n_ct == 0 || R == 0) return hipSuccess;
  if (!grid_ok(gx, N)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cc_keyswitch, dim3((uint32_t)gx, N / 256), dim3(256), 0, st, xh, dh, keys, gal, out, R, LD,
                     logn, c);
  return hipGetLastError();
}

hipError_t launch_cc_weight_slots(const int8_t *filt, const uint32_t *rot_tab, const uint32_t *pow3, uint32_t *z,
                                  const CcGeom &cg, size_t p0, size_t n_pt, uint32_t t, hipStream_t st) {
  if (n_pt == 0) return hipSuccess;
  if (!grid_ok(n_pt, cg.N)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cc_weight_slots, dim3((uint32_t)n_pt, cg.N / 256), dim3(256), 0, st, filt, rot_tab, pow3, z,
                     cg, p0, t);
  return hipGetLastError();
}

hipError_t launch_cc_slot_perm(const uint32_t *in, uint32_t *out, const uint32_t *pow3, size_t n, uint32_t logn,
                               int dir, hipStream_t st) {
  const uint32_t N = 1u << logn;
  if (n == 0) return hipSuccess;
  if (!grid_ok(n, N)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cc_slot_perm, dim3((uint32_t)n, N / 256), dim3(256), 0, st, in, out, pow3, logn, dir);
  return hipGetLastError();
}

hipError_t launch_cc_keygen(const uint32_t *ah, const uint32_t *eh, const uint32_t *sh, const uint32_t *gal,
                            uint32_t *keys, uint32_t R, uint32_t LD, uint32_t D, uint32_t T, uint32_t logn,
                            const LimbConsts &c, hipStream_t st) {
  const uint32_t N = 1u << logn;
  const size_t gx = (size_t)R * LD * c.L;
  if (R == 0) return hipSuccess;
  if (!grid_ok(gx, N)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cc_keygen, dim3((uint32_t)gx, N / 256), dim3(256), 0, st, ah, eh, sh, gal, keys, LD, D, T,
                     logn, c);
  return hipGetLastError();
}

hipError_t launch_cc_lift_signed(const int32_t *e, uint32_t *out, size_t n, uint32_t N, const LimbConsts &c,
                                 hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (!grid_ok(n, N)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cc_lift_signed, dim3((uint32_t)n, N / 256), dim3(256), 0, st, e, out, N, c);
  return hipGetLastError();
}

}  // namespace hc
