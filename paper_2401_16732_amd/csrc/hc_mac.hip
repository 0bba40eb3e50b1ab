// gfx950 multiply-accumulate kernels of the homomorphic convolution (A3): the
// register-tiled and the LDS-staged form, with their launcher.
#include "hc_device.h"

namespace hc {

// ---------------------------------------------------------------- multiply-accumulate
// reduce64_lazy of sums pp of a register tile, with the first multiply-add of
// every sum issued before the second ones (no multiply-add waits on the one
// just before it); the same values as reduce64_lazy
template <int CT, int BT>
__device__ __forceinline__ void reduce_tile_lazy(uint64_t (&acc)[CT][BT][2], int pp, uint32_t (&out)[CT][BT],
                                                 uint32_t q, uint32_t r2, uint32_t r2p, uint32_t onep) {
  uint32_t Q[CT][BT];
#pragma unroll
  for (int cc = 0; cc < CT; ++cc)
#pragma unroll
    for (int bb = 0; bb < BT; ++bb) {
      const uint64_t a = acc[cc][bb][pp];
      const uint32_t hi = (uint32_t)(a >> 32), lo = (uint32_t)a;
      Q[cc][bb] = __umulhi(hi, r2p) + __umulhi(lo, onep);
      acc[cc][bb][pp] = mad64_s(hi, r2, a);
    }
#pragma unroll
  for (int cc = 0; cc < CT; ++cc)
#pragma unroll
    for (int bb = 0; bb < BT; ++bb) out[cc][bb] = csub(mad_lo_s(Q[cc][bb], 0u - q, acc[cc][bb][pp]), 2 * q);
}

// A wave's tile of sums leaves as Yhat values in [0, 2q) (the inverse NTT's
// input range): nc channels x nb images x 2 polynomials, 64 coefficients from
// kb 64, lane `lane4 / 4` storing one. Each polynomial segment is a raw buffer
// store whose base (wave-uniform, scalar registers) is the segment and whose
// lane offset is lane4, so the stores need no vector address arithmetic.
template <int CT, int BT>
__device__ __forceinline__ void store_tile(const uint64_t (&acc)[CT][BT][2], uint32_t *Y, const ConvGeom &g,
                                           uint32_t b0, uint32_t i0, uint32_t tau, uint32_t l, uint32_t kb,
                                           uint32_t nc, uint32_t nb, uint32_t lane4, uint32_t q, uint32_t r2,
                                           uint32_t r2p, uint32_t onep) {
  const size_t LN = (size_t)g.L * g.N;
#pragma unroll
  for (int cc = 0; cc < CT; ++cc) {
    if ((uint32_t)cc >= nc) continue;
    const uint32_t o = (i0 + cc) * g.T + tau;
#pragma unroll
    for (int bb = 0; bb < BT; ++bb) {
      if ((uint32_t)bb >= nb) continue;
      uint32_t *y = Y + (((size_t)(b0 + bb) * g.O + o) * 2) * LN + (size_t)l * g.N + (size_t)kb * 64;
      const __amdgpu_buffer_rsrc_t yr =
          __builtin_amdgcn_make_buffer_rsrc((void *)y, (short)0, (int)0xffffffffu, (int)kBufferWord3);
      __builtin_amdgcn_raw_buffer_store_b32(reduce64_lazy(acc[cc][bb][0], q, r2, r2p, onep), yr, lane4, 0, 0);
      __builtin_amdgcn_raw_buffer_store_b32(reduce64_lazy(acc[cc][bb][1], q, r2, r2p, onep), yr, lane4,
                                            (uint32_t)(LN * 4), 0);
    }
  }
}

// Yhat[b][o][p][l][k] = sum_{gw < G_w} What[i][gw][l][k] * Xhat[b][gw T + tau][p][l][k]  mod q_l,
// o = i T + tau. The weights are stored blocked, What[l][k / 64][gw][i][k mod 64]
// with g.w_ld channels per block (launch_weight_block): the 64 coefficients of
// a tile's consecutive channels for one input ciphertext are one run.
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
  // the host guarantees BT*G*2*L*N*4 < 2^32; in the weights' block a channel
  // is the next 256 bytes), and every lane the same 4 * lane.
  const char *xbase = (const char *)(X + ((size_t)b0 * g.G + tau) * 2 * LN + (size_t)l * g.N + (size_t)kb * 64);
  const char *wbase = (const char *)(Wt + (((size_t)l * nkb + kb) * g.G_w * g.w_ld + i0) * 64);
  const size_t xstep = (size_t)8 * LN * g.T, wstep = (size_t)256 * g.w_ld;  // bytes
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
    wo[cc] = __builtin_amdgcn_readfirstlane(((uint32_t)cc < nc ? (uint32_t)cc : 0u) * 256u);
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
  // loads in flight. The last partial chunk needs no fold: the final reduction takes any
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
  store_tile<CT, BT>(acc, Y, g, b0, i0, tau, l, kb, nc, nb, lane4, q, r2, r2p, onep);
}

// Epilogue of the LDS- and DMA-staged MACs with PRE (= 5) inverse stages:
// the wave's 64 sums (one polynomial per lane slot: 2 BT CT = 64) leave in
// [0, 2q) after the inverse NTT's stages on index bits 0 .. PRE-1, which act
// within the tile's block of 64 coefficients. In two rounds, one per half of
// the block, each wave moves its 64 polynomials x 32 coefficients through its
// LDS region (64 x 36 words from `stage`) so that a lane holds 32 consecutive
// coefficients of one polynomial, runs the stages in registers with twiddles
// that are the same for every lane (scalar loads), and goes back through LDS
// so that every store writes two whole 128-byte runs. Every wave of the
// workgroup calls it (its barriers), also one whose tile is absent (it stores
// nothing).
template <int CT, int BT, int PRE>
__device__ __forceinline__ void pre_epilogue(const uint64_t (&acc)[CT][BT][2], uint32_t *stage, uint32_t wave,
                                             uint32_t lane, uint32_t *Y, const ConvGeom &g, uint32_t B,
                                             uint32_t b0, uint32_t i0, uint32_t tau, uint32_t l, uint32_t kb,
                                             uint32_t q, uint32_t r2, uint32_t r2p, uint32_t onep,
                                             const uint2 *__restrict__ twinv) {
  static_assert(PRE == 5 && 2 * BT * CT == 64, "epilogue stages need one polynomial per lane");
  constexpr uint32_t RWW = 64 * 36;  // words per wave (64 x (32 + 4 pad))
  const size_t LN = (size_t)g.L * g.N;
  uint32_t val[CT][BT][2];
#pragma unroll
  for (int cc = 0; cc < CT; ++cc)
#pragma unroll
    for (int bb = 0; bb < BT; ++bb)
#pragma unroll
      for (int pp = 0; pp < 2; ++pp) val[cc][bb][pp] = reduce64_lazy(acc[cc][bb][pp], q, r2, r2p, onep);
  // polynomial P = (cc BT + bb) 2 + pp of the wave's tile is row P of the
  // wave's LDS region
  uint32_t *region = stage + wave * RWW;
  const uint32_t q2 = 2 * q, nq = 0u - q;
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
      // the stage's 16 butterflies side by side, one operation at a time
      // (pair k is (u, u + 2^b), u = k with a zero inserted at bit b)
      uint32_t d[16], hi[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int u = ((k >> b) << (b + 1)) | (k & ((1 << b) - 1)), u2 = u | (1 << b);
        const uint32_t X = v[u], Yv = v[u2];
        d[k] = X - Yv + q2;
        v[u] = csub(X + Yv, q2);
      }
      uint64_t dw[16];  // (the products first: no multiply waits on the one before it)
#pragma unroll
      for (int k = 0; k < 16; ++k) hi[k] = __umulhi(d[k], (uint32_t)(tw[k >> b] >> 32));
#pragma unroll
      for (int k = 0; k < 16; ++k) dw[k] = mul64<true>(d[k], (uint32_t)tw[k >> b]);
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int u = ((k >> b) << (b + 1)) | (k & ((1 << b) - 1)), u2 = u | (1 << b);
        v[u2] = mad_lo_s(hi[k], nq, dw[k]);  // Shoup: in [0, 2q)
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
// storing, the epilogue (pre_epilogue) applies the inverse NTT's first PRE
// Gentleman-Sande stages (index bits 0 .. PRE-1); the masked inverse NTT then
// starts at bit PRE.
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
    woff[k] = (cc < ncw ? cc : 0u) * 256u + (e & 255u);
  }
  const char *xbase = (const char *)(X + ((size_t)bw * g.G + tau) * 2 * LN + (size_t)l * g.N + (size_t)kb * 64);
  const char *wbase = (const char *)(Wt + (((size_t)l * nkb + kb) * g.G_w * g.w_ld + iw) * 64);
  const size_t xstep = (size_t)8 * LN * g.T, wstep = (size_t)256 * g.w_ld;  // bytes
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
    store_tile<CT, BT>(acc, Y, g, b0, i0, tau, l, kb, nc, nb, lane * 4u, q, r2, r2p, onep);
  } else {
    pre_epilogue<CT, BT, PRE>(acc, (uint32_t *)stage, wave, lane, Y, g, B, b0, i0, tau, l, kb, q, r2, r2p, onep,
                              twinv);
  }
}

// s_waitcnt that waits until at most n vector memory operations of this wave
// are outstanding and leaves the other counters alone (gfx9 encoding: vmcnt
// in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
template <int n>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(n >= 0 && n < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14));
}

// One buffer load of `W` bytes per lane into LDS: lane i's bytes land at the
// wave-uniform LDS address `lds` + i W. (Device pass only: the host pass
// sees an empty body, since the host target has no such builtin.)
template <int W>
__device__ __forceinline__ void load_to_lds(__amdgpu_buffer_rsrc_t r, char *lds, uint32_t voff) {
  static_assert(W == 4 || W == 16, "4- or 16-byte lanes");
#if defined(__HIP_DEVICE_COMPILE__)
  using lds_ptr = __attribute__((address_space(3))) void *;
  if constexpr (W == 16)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr)lds, 16, voff, 0, 0, 0);
  else
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr)lds, 4, voff, 0, 0, 0);
#else
  (void)r, (void)lds, (void)voff;
#endif
}

// DMA-staged form of the same register tile. The step's segments (as in
// k_mac_lds) go from global memory straight into LDS: buffer loads with the
// LDS flag, which write lane i's 4 or 16 bytes at a wave-uniform LDS base
// + i * width, the position the LDS-staged form stores them at. S stages deep:
// S - 1 steps are in flight and none of them occupies registers. Per step g:
// wait until this thread's loads of step g have landed (its later steps'
// loads may stay outstanding), one barrier (then every thread's have, and
// every wave has finished reading the stage that the next loads refill),
// issue the loads of step g + S - 1, read the operands from stage g mod S
// and multiply-accumulate.
// The grid may be smaller than the ntiles tiles: each workgroup then loops
// over its share, so that a capped launch leaves room on every compute unit
// for the workgroups of a kernel running beside it on another stream. With
// the grid and ntiles multiples of 8, workgroup w (on XCD w mod 8) takes the
// tiles (w mod 8) ntiles/8 + w/8 + k grid/8: the workgroups of one XCD work
// on consecutive tiles, as the full launch's remap arranges.
// PRE: as in k_mac_lds (pre_epilogue; its region reuses the stages).
template <int BT, int CT, int RG, int CG, int S, int PRE>
__global__ __launch_bounds__(64 * RG * CG) void k_mac_dma(const uint32_t *__restrict__ X,
                                                          const uint32_t *__restrict__ Wt,
                                                          uint32_t *__restrict__ Y, ConvGeom g, uint32_t B,
                                                          uint32_t nib, uint32_t nkb, LimbConsts c,
                                                          uint32_t ntiles, const uint2 *__restrict__ twinv) {
  constexpr int NT = 64 * RG * CG;
  constexpr int NX = RG * BT * 2, NW = CG * CT;          // segments per step
  constexpr int XB = NX * 256 / NT, WB = NW * 256 / NT;  // bytes per thread per step
  static_assert(NX * 256 % NT == 0 && NW * 256 % NT == 0 && XB % 4 == 0 && WB % 4 == 0, "shares must be whole");
  constexpr int XW = XB % 16 == 0 ? 16 : 4, WWD = WB % 16 == 0 ? 16 : 4;  // access widths
  constexpr int KX = XB / XW, KW = WB / WWD;                              // accesses per thread per step
  constexpr int LPS = KX + KW;
  static_assert(S >= 2 && (S - 1) * LPS <= 63, "loads in flight beyond the vector memory counter");
  constexpr uint32_t BUFB = (NX + NW) * 256;  // bytes per stage
  constexpr uint32_t BUFW = BUFB / 4;
  static_assert(PRE == 0 || (PRE == 5 && 2 * BT * CT == 64), "epilogue stages need one polynomial per lane");
  constexpr uint32_t EPB = PRE ? RG * CG * 64 * 36 * 4 : 0;  // pre_epilogue's regions
  __shared__ uint4 stage4[(S * BUFB > EPB ? S * BUFB : EPB) / 16];
  char *stage = (char *)stage4;
  const uint32_t G = gridDim.x;
  const bool xcd = (ntiles & 7u) == 0 && (G & 7u) == 0;
  const uint32_t tid = threadIdx.x;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t lane = tid & 63u;
  const uint32_t rg = wave % RG, cg = wave / RG;
  const uint32_t LN = g.L * g.N;
  const uint32_t G_w = g.G_w, last = G_w - 1;
  const size_t xstep = (size_t)8 * LN * g.T, wstep = (size_t)256 * g.w_ld;  // bytes
  // this wave's operands inside a stage (words)
  const uint32_t *xs0 = (const uint32_t *)stage + (rg * BT * 2) * 64 + lane;
  const uint32_t *ws0 = (const uint32_t *)stage + (NX + cg * CT) * 64 + lane;
  for (uint32_t it = 0;; ++it) {
    uint32_t wg;
    if (xcd) {
      const uint32_t m = (blockIdx.x >> 3) + it * (G >> 3);
      if (m >= (ntiles >> 3)) break;
      wg = (blockIdx.x & 7u) * (ntiles >> 3) + m;
    } else {
      wg = blockIdx.x + it * G;
      if (wg >= ntiles) break;
    }
    // image tiles vary fastest (as in k_mac_lds)
    const uint32_t nbt = (B + RG * BT - 1) / (RG * BT);
    const uint32_t bt = wg % nbt;
    uint32_t r = wg / nbt;
    const uint32_t ib = r % nib;
    r /= nib;
    const uint32_t tau = r % g.T;
    r /= g.T;
    const uint32_t kb = r % nkb;
    const uint32_t l = r / nkb;
    const uint32_t bw = bt * RG * BT, iw = ib * CG * CT;
    if (bw >= B || iw >= g.c_out) continue;  // uniform over the workgroup
    const uint32_t nbw = min((uint32_t)(RG * BT), B - bw), ncw = min((uint32_t)(CG * CT), g.c_out - iw);
    // per-thread global byte offsets of its accesses, fixed for the tile
    // (absent images and channels read image / channel 0 of the tile)
    uint32_t xoff[KX], woff[KW];
#pragma unroll
    for (int k = 0; k < KX; ++k) {
      const uint32_t e = (tid + k * NT) * XW, seg = e >> 8, i = seg >> 1;
      xoff[k] = (((i < nbw ? i : 0u) * g.G * 2 + (seg & 1u)) * LN) * 4u + (e & 255u);
    }
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      const uint32_t e = (tid + k * NT) * WWD, cc = e >> 8;
      woff[k] = (cc < ncw ? cc : 0u) * 256u + (e & 255u);
    }
    const char *xbase = (const char *)(X + ((size_t)bw * g.G + tau) * 2 * LN + (size_t)l * g.N + (size_t)kb * 64);
    const char *wbase = (const char *)(Wt + (((size_t)l * nkb + kb) * g.G_w * g.w_ld + iw) * 64);
    // step gw into stage st: access k of this thread lands at byte (tid + k NT) width
    // of its operand's part of the stage = wave-uniform (wave 64 + k NT) width + lane width
    auto issue = [&](uint32_t gw, uint32_t st) {
      const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
          (void *)(xbase + gw * xstep), (short)0, (int)0xffffffffu, (int)kBufferWord3);
      const __amdgpu_buffer_rsrc_t wr = __builtin_amdgcn_make_buffer_rsrc(
          (void *)(wbase + gw * wstep), (short)0, (int)0xffffffffu, (int)kBufferWord3);
      char *sb = stage + st * BUFB;
#pragma unroll
      for (int k = 0; k < KX; ++k) load_to_lds<XW>(xr, sb + (wave * 64 + k * NT) * XW, xoff[k]);
#pragma unroll
      for (int k = 0; k < KW; ++k) load_to_lds<WWD>(wr, sb + NX * 256 + (wave * 64 + k * NT) * WWD, woff[k]);
    };
    const uint32_t q = c.q[l], r2 = c.r2[l], fold = c.fold[l];
    // (without epilogue stages the first step sets the accumulators: no
    // zeroing pass per tile; with them the registers are too tight for two
    // forms of the step)
    uint64_t acc[CT][BT][2];
    if constexpr (PRE != 0) {
#pragma unroll
      for (int cc = 0; cc < CT; ++cc)
#pragma unroll
        for (int bb = 0; bb < BT; ++bb) acc[cc][bb][0] = acc[cc][bb][1] = 0;
    }
#pragma unroll
    for (int j = 0; j < S - 1; ++j) issue(min((uint32_t)j, last), (uint32_t)j);
    uint32_t since_fold = 0;
    for (uint32_t g0 = 0; g0 < G_w; g0 += S) {
#pragma unroll
      for (int j = 0; j < S; ++j) {
        const uint32_t gw = g0 + j;
        if (gw >= G_w) break;  // uniform
        wait_vmcnt<(S - 2) * LPS>();
        asm volatile("s_barrier" ::: "memory");
        issue(min(gw + S - 1, last), (uint32_t)((j + S - 1) % S));
        const uint32_t *xs = xs0 + j * BUFW, *wsp = ws0 + j * BUFW;
        uint32_t w[CT], x[BT][2];
#pragma unroll
        for (int cc = 0; cc < CT; ++cc) w[cc] = wsp[cc * 64];
#pragma unroll
        for (int bb = 0; bb < BT; ++bb) {
          x[bb][0] = xs[(bb * 2) * 64];
          x[bb][1] = xs[(bb * 2 + 1) * 64];
        }
        if (PRE == 0 && j == 0 && gw == 0) {
#pragma unroll
          for (int cc = 0; cc < CT; ++cc)
#pragma unroll
            for (int bb = 0; bb < BT; ++bb) {
              acc[cc][bb][0] = (uint64_t)w[cc] * x[bb][0];
              acc[cc][bb][1] = (uint64_t)w[cc] * x[bb][1];
            }
        } else {
#pragma unroll
          for (int cc = 0; cc < CT; ++cc)
#pragma unroll
            for (int bb = 0; bb < BT; ++bb) {
              acc[cc][bb][0] += (uint64_t)w[cc] * x[bb][0];
              acc[cc][bb][1] += (uint64_t)w[cc] * x[bb][1];
            }
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
      }
    }
    // the redundant loads past the last step must land, and every wave must
    // be done with the stages, before the next tile's loads (or the release
    // of the workgroup's LDS)
    wait_vmcnt<0>();
    asm volatile("s_barrier" ::: "memory");
    const uint32_t i0 = iw + cg * CT, b0 = bw + rg * BT;
    if constexpr (PRE == 0) {
      if (i0 < g.c_out && b0 < B) {
        const uint32_t nc = min((uint32_t)CT, g.c_out - i0), nb = min((uint32_t)BT, B - b0);
        store_tile<CT, BT>(acc, Y, g, b0, i0, tau, l, kb, nc, nb, lane * 4u, q, r2, c.r2_p[l], c.one_p[l]);
      }
    } else {
      pre_epilogue<CT, BT, PRE>(acc, (uint32_t *)stage, wave, lane, Y, g, B, b0, i0, tau, l, kb, q, r2, c.r2_p[l],
                                c.one_p[l], twinv);
      // the regions overlap the stages that the next tile's loads refill
      __syncthreads();
    }
  }
}

// Multiply-accumulate that also carries out c0's masked inverse transform up
// to its final sum (MacShape pre = kMacC0; layers with mac_c0_ok). With every
// extracted c0 coefficient below 64, the pruned transform is the
// Gentleman-Sande stages on index bits 0..5 inside each 64-coefficient block,
// then the plain sum of the blocks (the top stages' sum halves). The tile is
// k_mac_dma's (4 images x 8 channels per thread, RG x CG waves, S stages), but
// a workgroup owns (image tile, channel tile, limb, split sp) and walks the
// blocks kb of its split, nkb / nsplit of them. Per block: the steps over the
// input ciphertexts as in k_mac_dma; c1's sums go to Yhat; c0's 32 sums per
// lane (one coefficient of 32 polynomials) go through the wave's LDS region
// so that lane (P, h) = (lane mod 32, lane / 32) holds coefficients 2 u + h,
// u < 32, of polynomial P; the stage on bit 0 pairs lane L with L xor 32
// (swaps of the wave's halves, one butterfly per lane, per-lane twiddles), the
// stages on bits 1..5 run in registers (every twiddle the same in all lanes,
// scalar loads), and the block's result is added to the lane's running sums
// in [0, 2q). At the end every lane writes its 32 sums to
// Yhat[b][i][0][l][64 sp + 32 h + u], the unused c0 slot of its polynomial
// (coefficient 2 u + h of the split's partial sum).
template <int RG, int CG, int S>
__global__ __launch_bounds__(64 * RG * CG) void k_mac_c0x(const uint32_t *__restrict__ X,
                                                          const uint32_t *__restrict__ Wt,
                                                          uint32_t *__restrict__ Y, ConvGeom g, uint32_t B,
                                                          uint32_t nib, uint32_t nkb, LimbConsts c,
                                                          uint32_t nsplit, const uint2 *__restrict__ twinv) {
  constexpr int BT = 4, CT = 8;
  constexpr int NT = 64 * RG * CG;
  constexpr int NX = RG * BT * 2, NW = CG * CT;          // segments per step
  constexpr int XB = NX * 256 / NT, WB = NW * 256 / NT;  // bytes per thread per step
  static_assert(NX * 256 % NT == 0 && NW * 256 % NT == 0 && XB % 4 == 0 && WB % 4 == 0, "shares must be whole");
  constexpr int XW = XB % 16 == 0 ? 16 : 4, WWD = WB % 16 == 0 ? 16 : 4;  // access widths
  constexpr int KX = XB / XW, KW = WB / WWD;                              // accesses per thread per step
  constexpr int LPS = KX + KW;
  static_assert(S >= 2 && (S - 1) * LPS <= 63, "loads in flight beyond the vector memory counter");
  constexpr uint32_t BUFB = (NX + NW) * 256;  // bytes per stage
  constexpr uint32_t BUFW = BUFB / 4;
  constexpr uint32_t RS = 68;                          // region row: 64 coefficients + 4 pad (words)
  constexpr uint32_t EPB = RG * CG * 32 * RS * 4;      // the waves' regions (32 rows each)
  __shared__ uint4 stage4[(S * BUFB > EPB ? S * BUFB : EPB) / 16];
  char *stage = (char *)stage4;
  const uint32_t tid = threadIdx.x;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t lane = tid & 63u;
  const uint32_t rg = wave % RG, cg = wave / RG;
  const uint32_t LN = g.L * g.N;
  const uint32_t G_w = g.G_w, last = G_w - 1;
  const uint32_t LOGN = 31 - __builtin_clz(g.N);
  const size_t xstep = (size_t)8 * LN, wstep = (size_t)256 * g.w_ld;  // bytes (one row tile)
  const uint32_t *xs0 = (const uint32_t *)stage + (rg * BT * 2) * 64 + lane;
  const uint32_t *ws0 = (const uint32_t *)stage + (NX + cg * CT) * 64 + lane;
  // workgroup -> (image tile, channel tile, split, limb), image tiles fastest;
  // the workgroups of one XCD take consecutive ones
  const uint32_t nwg = gridDim.x;
  uint32_t wg = blockIdx.x;
  if ((nwg & 7u) == 0) wg = (wg & 7u) * (nwg >> 3) + (wg >> 3);
  const uint32_t nbt = (B + RG * BT - 1) / (RG * BT);
  const uint32_t bt = wg % nbt;
  uint32_t r = wg / nbt;
  const uint32_t ib = r % nib;
  r /= nib;
  const uint32_t sp = r % nsplit;
  const uint32_t l = r / nsplit;
  const uint32_t bw = bt * RG * BT, iw = ib * CG * CT;
  const uint32_t nbw = min((uint32_t)(RG * BT), B - bw), ncw = min((uint32_t)(CG * CT), g.c_out - iw);
  uint32_t xoff[KX], woff[KW];
#pragma unroll
  for (int k = 0; k < KX; ++k) {
    const uint32_t e = (tid + k * NT) * XW, seg = e >> 8, i = seg >> 1;
    xoff[k] = (((i < nbw ? i : 0u) * g.G * 2 + (seg & 1u)) * LN) * 4u + (e & 255u);
  }
#pragma unroll
  for (int k = 0; k < KW; ++k) {
    const uint32_t e = (tid + k * NT) * WWD, cc = e >> 8;
    woff[k] = (cc < ncw ? cc : 0u) * 256u + (e & 255u);
  }
  const uint32_t q = c.q[l], r2 = c.r2[l], fold = c.fold[l], r2p = c.r2_p[l], onep = c.one_p[l];
  const uint32_t q2 = 2 * q, nq = 0u - q;
  const uint32_t i0 = iw + cg * CT, b0 = bw + rg * BT;
  const bool tile_on = i0 < g.c_out && b0 < B;  // uniform over the wave
  const uint32_t nc = tile_on ? min((uint32_t)CT, g.c_out - i0) : 0u, nb = tile_on ? min((uint32_t)BT, B - b0) : 0u;
  // this lane's polynomial and half in the epilogue
  const uint32_t P = lane & 31u, h = lane >> 5;
  const uint32_t pcc = P / BT, pbb = P % BT;
  uint32_t *region = (uint32_t *)stage + wave * 32 * RS;
  uint32_t sum[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) sum[j] = 0;
  const uint32_t kbs = nkb / nsplit, kb0 = sp * kbs;
  for (uint32_t kb = kb0; kb < kb0 + kbs; ++kb) {
    const char *xbase = (const char *)(X + (size_t)bw * g.G * 2 * LN + (size_t)l * g.N + (size_t)kb * 64);
    const char *wbase = (const char *)(Wt + (((size_t)l * nkb + kb) * g.G_w * g.w_ld + iw) * 64);
    auto issue = [&](uint32_t gw, uint32_t st) {
      const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
          (void *)(xbase + gw * xstep), (short)0, (int)0xffffffffu, (int)kBufferWord3);
      const __amdgpu_buffer_rsrc_t wr = __builtin_amdgcn_make_buffer_rsrc(
          (void *)(wbase + gw * wstep), (short)0, (int)0xffffffffu, (int)kBufferWord3);
      char *sb = stage + st * BUFB;
#pragma unroll
      for (int k = 0; k < KX; ++k) load_to_lds<XW>(xr, sb + (wave * 64 + k * NT) * XW, xoff[k]);
#pragma unroll
      for (int k = 0; k < KW; ++k) load_to_lds<WWD>(wr, sb + NX * 256 + (wave * 64 + k * NT) * WWD, woff[k]);
    };
    // (the first step sets the accumulators: no zeroing pass per block)
    uint64_t acc[CT][BT][2];
#pragma unroll
    for (int j = 0; j < S - 1; ++j) issue(min((uint32_t)j, last), (uint32_t)j);
    uint32_t since_fold = 0;
    for (uint32_t g0 = 0; g0 < G_w; g0 += S) {
#pragma unroll
      for (int j = 0; j < S; ++j) {
        const uint32_t gw = g0 + j;
        if (gw >= G_w) break;  // uniform
        wait_vmcnt<(S - 2) * LPS>();
        asm volatile("s_barrier" ::: "memory");
        issue(min(gw + S - 1, last), (uint32_t)((j + S - 1) % S));
        const uint32_t *xs = xs0 + j * BUFW, *wsp = ws0 + j * BUFW;
        uint32_t w[CT], x[BT][2];
#pragma unroll
        for (int cc = 0; cc < CT; ++cc) w[cc] = wsp[cc * 64];
#pragma unroll
        for (int bb = 0; bb < BT; ++bb) {
          x[bb][0] = xs[(bb * 2) * 64];
          x[bb][1] = xs[(bb * 2 + 1) * 64];
        }
        if (j == 0 && gw == 0) {
#pragma unroll
          for (int cc = 0; cc < CT; ++cc)
#pragma unroll
            for (int bb = 0; bb < BT; ++bb) {
              acc[cc][bb][0] = (uint64_t)w[cc] * x[bb][0];
              acc[cc][bb][1] = (uint64_t)w[cc] * x[bb][1];
            }
        } else {
#pragma unroll
          for (int cc = 0; cc < CT; ++cc)
#pragma unroll
            for (int bb = 0; bb < BT; ++bb) {
              acc[cc][bb][0] += (uint64_t)w[cc] * x[bb][0];
              acc[cc][bb][1] += (uint64_t)w[cc] * x[bb][1];
            }
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
      }
    }
    // the loads past the last step have landed and every wave is done with
    // the stages: they become the waves' regions
    wait_vmcnt<0>();
    asm volatile("s_barrier" ::: "memory");
    // c1: the block's sums as k_mac_dma stores them
    uint32_t red[CT][BT];
    reduce_tile_lazy<CT, BT>(acc, 1, red, q, r2, r2p, onep);
    if (tile_on) {
#pragma unroll
      for (int cc = 0; cc < CT; ++cc) {
        if ((uint32_t)cc >= nc) continue;
#pragma unroll
        for (int bb = 0; bb < BT; ++bb) {
          if ((uint32_t)bb >= nb) continue;
          uint32_t *y = Y + (((size_t)(b0 + bb) * g.O + i0 + cc) * 2 + 1) * LN + (size_t)l * g.N + (size_t)kb * 64;
          const __amdgpu_buffer_rsrc_t yr =
              __builtin_amdgcn_make_buffer_rsrc((void *)y, (short)0, (int)0xffffffffu, (int)kBufferWord3);
          __builtin_amdgcn_raw_buffer_store_b32(red[cc][bb], yr, lane * 4u, 0, 0);
        }
      }
    }
    // the stage on bit 0's twiddles for this lane's butterflies, index
    // 2^(LOGN-1) + 32 kb + 16 h + u for u < 16 ({w, w'} of u = 2k, 2k + 1 in w4[k])
    uint4 w4[8];
    {
      const uint4 *tw4 = (const uint4 *)(twinv + (size_t)l * g.N + (1u << (LOGN - 1)) + kb * 32 + h * 16);
#pragma unroll
      for (int k = 0; k < 8; ++k) w4[k] = tw4[k];
    }
    // c0: row P of the region holds the block of polynomial P = cc BT + bb,
    // deinterleaved (coefficient k at column 32 (k mod 2) + k / 2), so that
    // lane (P, h) reads coefficients 2 u + h, u < 32, as one run
    const uint32_t col = (lane & 1u) * 32u + (lane >> 1);
    reduce_tile_lazy<CT, BT>(acc, 0, red, q, r2, r2p, onep);
#pragma unroll
    for (int cc = 0; cc < CT; ++cc)
#pragma unroll
      for (int bb = 0; bb < BT; ++bb) region[(cc * BT + bb) * RS + col] = red[cc][bb];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint32_t v[32];
    const uint4 *r4 = (const uint4 *)(region + P * RS + h * 32);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint4 t4 = r4[k];
      v[4 * k] = t4.x, v[4 * k + 1] = t4.y, v[4 * k + 2] = t4.z, v[4 * k + 3] = t4.w;
    }
    // stage on bit 0: (2u, 2u + 1) sit in lanes (P, 0) and (P, 1) of v[u]. A
    // swap of the wave's halves between v[u] and v[u + 16] (u < 16) gives lane
    // (P, 0) the pair of u and lane (P, 1) the pair of u + 16, so every lane
    // computes one whole butterfly; a second swap restores the layout
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const auto p = __builtin_amdgcn_permlane32_swap(v[u], v[u + 16], false, false);
      const uint32_t e = p[0], o = p[1];
      const uint4 w2 = w4[u >> 1];
      const uint32_t w = (u & 1) ? w2.z : w2.x, wp = (u & 1) ? w2.w : w2.y;
      const uint32_t s = csub(e + o, q2);
      const uint32_t t = shoup_mad<false>(e - o + q2, w, wp, nq);
      const auto r = __builtin_amdgcn_permlane32_swap(s, t, false, false);
      v[u] = r[0];
      v[u + 16] = r[1];
    }
    // stages on bits 1..5 of j = 64 kb + 2u + h, bits 0..4 of u, in registers:
    // twiddle index 2^(LOGN-1-b) + (j >> (b+1)) = 2^(LOGN-1-b) + 2^(5-b) kb +
    // (u >> b) for bit b, the same in every lane
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      const_u64 *tw = (const_u64 *)(twinv + (size_t)l * g.N + (1u << (LOGN - 2 - b)) + ((kb * 64) >> (b + 2)));
      uint32_t d[16], hi[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int u = ((k >> b) << (b + 1)) | (k & ((1 << b) - 1)), u2 = u | (1 << b);
        const uint32_t A = v[u], Bv = v[u2];
        d[k] = A - Bv + q2;
        v[u] = csub(A + Bv, q2);
      }
      uint64_t dw[16];  // (the products first: no multiply waits on the one before it)
#pragma unroll
      for (int k = 0; k < 16; ++k) hi[k] = __umulhi(d[k], (uint32_t)(tw[k >> b] >> 32));
#pragma unroll
      for (int k = 0; k < 16; ++k) dw[k] = mul64<true>(d[k], (uint32_t)tw[k >> b]);
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int u = ((k >> b) << (b + 1)) | (k & ((1 << b) - 1)), u2 = u | (1 << b);
        v[u2] = mad_lo_s(hi[k], nq, dw[k]);  // Shoup: in [0, 2q)
      }
    }
#pragma unroll
    for (int u = 0; u < 32; ++u) sum[u] = csub(sum[u] + v[u], q2);
    // every wave is done with its region (the stages of the next block)
    __syncthreads();
  }
  if (tile_on && pcc < nc && pbb < nb) {
    uint4 *dst = (uint4 *)(Y + (((size_t)(b0 + pbb) * g.O + i0 + pcc) * 2) * LN + (size_t)l * g.N + sp * 64 + h * 32);
#pragma unroll
    for (int k = 0; k < 8; ++k) dst[k] = make_uint4(sum[4 * k], sum[4 * k + 1], sum[4 * k + 2], sum[4 * k + 3]);
  }
}

template <int BT, int CT, int RG, int CG, int NS, int LDS, int PRE>
static hipError_t mac_t(const ConvGeom &g, const uint32_t *x, const uint32_t *w, uint32_t *y, uint32_t B,
                        const LimbConsts &c, const Twiddles &tw, hipStream_t st, uint32_t max_wgs) {
  if (!mac_offsets_fit(g, MacShape{BT, CT, RG, CG, NS, LDS, PRE})) return hipErrorInvalidValue;
  const uint32_t nkb = g.N / 64;
  const uint32_t nib = (g.c_out + CG * CT - 1) / (CG * CT);
  const uint32_t nbt = (B + RG * BT - 1) / (RG * BT);
  const size_t nwg = (size_t)nib * g.T * nkb * g.L * nbt;
  if (nwg == 0) return hipSuccess;
  if constexpr (PRE == (int)kMacC0) {
    static_assert(LDS == 2 && BT == 4 && CT == 8, "c0's transform in the MAC: the DMA-staged 4 x 8 tile");
    // one workgroup per (image tile, channel tile, split, limb); no cap
    const uint32_t ns = c0_splits(g);
    hipLaunchKernelGGL((k_mac_c0x<RG, CG, NS>), dim3((uint32_t)((size_t)nib * nbt * ns * g.L)), dim3(64 * RG * CG),
                       0, st, x, w, y, g, B, nib, nkb, c, ns, tw.inv);
  } else if constexpr (LDS == 2) {
    // a cap (a multiple of 8, so that the XCD arrangement holds) turns the
    // launch into workgroups that loop over the tiles
    const size_t cap = max_wgs >= 8 ? (size_t)(max_wgs & ~7u) : nwg;
    hipLaunchKernelGGL((k_mac_dma<BT, CT, RG, CG, NS, PRE>), dim3((uint32_t)std::min(nwg, cap)), dim3(64 * RG * CG),
                       0, st, x, w, y, g, B, nib, nkb, c, (uint32_t)nwg, tw.inv);
  }
  else if constexpr (LDS == 1)
    hipLaunchKernelGGL((k_mac_lds<BT, CT, RG, CG, NS, PRE>), dim3((uint32_t)nwg), dim3(64 * RG * CG), 0, st, x, w,
                       y, g, B, nib, nkb, c, tw.inv);
  else
    hipLaunchKernelGGL((k_mac_tiled<BT, CT, RG, CG, NS>), dim3((uint32_t)nwg), dim3(64 * RG * CG), 0, st, x, w, y,
                       g, B, nib, nkb, c);
  return hipGetLastError();
}

// The register tile's 32-bit input offsets span BT images; the LDS-staged
// form's span the workgroup's RG BT images. (The weight offsets stay inside
// one block of channels.)
bool mac_offsets_fit(const ConvGeom &g, const MacShape &m) {
  const uint64_t ln = (uint64_t)g.L * g.N * 4;
  const uint64_t bi = m.lds ? (uint64_t)m.rg * m.bt : m.bt;
  if (m.pre == kMacC0 && !mac_c0_ok(g)) return false;
  return bi * g.G * 2 * ln < (1ull << 32) && g.w_ld >= g.c_out;
}

// c0's transform fits the MAC where every extracted coefficient lies in the
// first block of 64 and the layer is one row tile (its output polynomials are
// (image, channel), with c0 slots of N words for the partial sums).
bool mac_c0_ok(const ConvGeom &g) { return g.T == 1 && g.prune_bits <= 6 && g.N >= 1024; }

// Splits of the 64-coefficient blocks over workgroups: enough workgroups
// (channel tiles of 16 x 2 image tiles x limbs x splits >= 1024), at most a
// quarter of the blocks per split count. Depends on the layer only, so that
// the MAC and the finishing pass agree for any group of its images.
uint32_t c0_splits(const ConvGeom &g) {
  const uint32_t nkb = g.N / 64;
  const uint64_t base = (uint64_t)((g.c_out + 15) / 16) * 2 * g.L;
  uint32_t s = 1;
  while (s * 4 < nkb && base * s < 1024) s *= 2;
  return s;
}

// (images per thread, channels per thread, image groups, channel groups,
//  loads in flight (register sets; LDS stages for the DMA-staged form),
//  0 register tile / 1 LDS-staged / 2 DMA-staged, inverse stages in the epilogue)
#define HC_MAC_VARIANTS(X)                                                                                      \
  X(1, 8, 1, 4, 2, 0, 0) X(1, 4, 1, 4, 2, 0, 0) X(2, 4, 1, 4, 2, 0, 0) X(4, 4, 1, 4, 2, 0, 0)                   \
  X(4, 2, 1, 4, 2, 0, 0) X(8, 2, 1, 4, 2, 0, 0) X(4, 4, 4, 2, 2, 0, 0) X(4, 8, 4, 2, 2, 0, 0)                   \
  X(2, 8, 4, 2, 2, 0, 0) X(4, 4, 2, 4, 2, 0, 0) X(2, 4, 4, 4, 2, 0, 0) X(1, 8, 2, 4, 2, 0, 0)                   \
  X(4, 8, 4, 2, 3, 0, 0) X(2, 8, 4, 2, 4, 0, 0) X(4, 4, 4, 2, 4, 0, 0) X(4, 4, 2, 4, 4, 0, 0)                   \
  X(1, 8, 2, 4, 4, 0, 0) X(2, 4, 4, 4, 4, 0, 0) X(1, 8, 1, 4, 4, 0, 0) X(4, 8, 4, 2, 2, 1, 0)                   \
  X(4, 8, 4, 2, 3, 1, 0) X(4, 8, 2, 2, 2, 1, 0) X(4, 8, 2, 2, 3, 1, 0) X(2, 8, 4, 2, 3, 1, 0)                   \
  X(4, 4, 4, 2, 3, 1, 0) X(2, 8, 2, 2, 3, 1, 0) X(4, 8, 4, 2, 2, 1, 5) X(4, 8, 2, 2, 2, 1, 5)                   \
  X(4, 8, 2, 2, 3, 1, 5) X(4, 8, 2, 2, 3, 2, 0) X(4, 8, 2, 2, 4, 2, 0) X(4, 8, 2, 2, 6, 2, 0)                   \
  X(4, 8, 4, 2, 3, 2, 0) X(4, 8, 4, 2, 4, 2, 0) X(2, 8, 4, 2, 4, 2, 0) X(4, 4, 4, 2, 4, 2, 0)                   \
  X(2, 8, 2, 2, 4, 2, 0) X(4, 4, 2, 2, 4, 2, 0) X(4, 8, 2, 2, 3, 2, 5) X(4, 8, 2, 2, 4, 2, 5)                   \
  X(4, 8, 4, 2, 4, 2, 5) X(4, 8, 2, 2, 3, 2, 6) X(4, 8, 2, 2, 4, 2, 6) X(4, 8, 4, 2, 3, 2, 6)                   \
  X(4, 8, 4, 2, 4, 2, 6)

bool mac_variant_ok(const MacShape &m) {
#define HC_MAC_OK(B_, C_, R_, G_, S_, D_, P_)                                                                 \
  if (m.bt == B_ && m.ct == C_ && m.rg == R_ && m.cg == G_ && m.depth == S_ && m.lds == D_ && m.pre == P_) \
    return true;
  HC_MAC_VARIANTS(HC_MAC_OK)
#undef HC_MAC_OK
  return false;
}

hipError_t launch_mac(const ConvGeom &g, const MacShape &m, const uint32_t *x, const uint32_t *w, uint32_t *y,
                      uint32_t B, const LimbConsts &c, const Twiddles &tw, hipStream_t st, uint32_t max_wgs) {
  if (m.pre == kMacPre && g.N < 4096) return hipErrorInvalidValue;  // the epilogue's twiddle layout needs N >= 4096
#define HC_MAC_CASE(B_, C_, R_, G_, S_, D_, P_)                                                               \
  if (m.bt == B_ && m.ct == C_ && m.rg == R_ && m.cg == G_ && m.depth == S_ && m.lds == D_ && m.pre == P_) \
    return mac_t<B_, C_, R_, G_, S_, D_, P_>(g, x, w, y, B, c, tw, st, max_wgs);
  HC_MAC_VARIANTS(HC_MAC_CASE)
#undef HC_MAC_CASE
  return hipErrorInvalidValue;
}

}  // namespace hc
