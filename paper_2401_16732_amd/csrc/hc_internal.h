// Internal declarations shared by the host library (hc_host.cpp, hc_server.cpp,
// hc_client.cpp) and the gfx950 kernels (hc_ntt.hip, hc_mac.hip,
// hc_intt_masked_*.hip, hc_client.hip). Not part of the ABI.
#pragma once
#include <cstddef>
#include <cstdint>
#include <hip/hip_runtime.h>

namespace hc {

constexpr int kMaxLimbs = 4;

// Per-limb constants handed to every kernel by value (scalar registers).
// Shoup pairs: for a constant w < q, wp = floor(w * 2^32 / q); then for any
// a < 2^32, a*w - floor(a*wp / 2^32)*q lies in [0, 2q).
struct LimbConsts {
  uint32_t q[kMaxLimbs];
  uint32_t ninv[kMaxLimbs], ninv_p[kMaxLimbs];     // N^-1
  uint32_t ninvw[kMaxLimbs], ninvw_p[kMaxLimbs];   // N^-1 * psi^-brv(1): last inverse stage
  uint32_t r2[kMaxLimbs];                          // 2^32 mod q (64-bit accumulator fold)
  uint32_t r2_p[kMaxLimbs];
  uint32_t one_p[kMaxLimbs];                       // floor(2^32 / q): Shoup constant of 1
  uint32_t delta[kMaxLimbs], delta_p[kMaxLimbs];   // Delta mod q
  uint32_t fold[kMaxLimbs];                        // MAC terms between two accumulator folds
  uint32_t t;                                      // plaintext modulus
  uint32_t L;
};

// Twiddles: per limb N entries {w, floor(w 2^32 / q)} in the order the
// butterflies read them: fwd[k] = psi^brv(k), inv[k] = psi^-brv(k).
struct Twiddles {
  const uint2 *fwd;
  const uint2 *inv;
};

// Geometry of one convolution as the kernels need it.
struct ConvGeom {
  uint32_t N, L;
  uint32_t c_in, c_out, f, s;        // s: stride on the encoded grid
  uint32_t cn, tiled, T, r_o;
  uint32_t G, G_w, O;
  uint32_t w_pad, F;
  uint32_t ho, wo;
  uint32_t prune_bits;  // every extracted c0 coefficient index is below 2^prune_bits
  uint32_t w_ld;        // NTT-domain weights: channels per (limb, coefficient block, input ciphertext) block
};

// Per-image buffer tables (kernel arguments by value) for groups of up to
// kMaxTab images whose buffers are not one strided array (the server).
constexpr uint32_t kMaxTab = 16;
struct ImgPtrs {
  uint64_t p[kMaxTab];
  uint32_t n;  // 0: not used
};
struct OutPtrs {
  uint64_t mask[kMaxTab], c0[kMaxTab], c1[kMaxTab];
  uint32_t n;  // 0: not used
};

// Launchers (the kernel sources). Each enqueues on `st` and returns the launch status.
// Launch-shape variants: an NTT uses 2^(logn - elog) threads per polynomial;
// the MAC gives each thread bt images x ct output channels, and a workgroup
// rg x cg such threads per coefficient (image groups x channel groups); depth
// input ciphertexts are in flight, in registers or (lds) staged through LDS.
// pre: inverse NTT stages (index bits 0 .. pre-1) applied by the MAC before
// it stores (0, or kMacPre for LDS-staged tiles with 2 bt ct = 64).
struct MacShape {
  uint32_t bt, ct, rg, cg, depth, lds, pre;
};
bool ntt_variant_ok(uint32_t logn, uint32_t elog);
// Inverse stages (index bits 0 .. kMacPre-1) the LDS-staged MAC can apply to
// its outputs before storing them, for the masked inverse NTT to skip.
constexpr uint32_t kMacPre = 5;
// mac pre = kMacC0: the MAC carries out c0's whole masked inverse transform
// up to the final sum (layers whose extracted c0 coefficients all lie below
// 64, in one row tile: mac_c0_ok): per 64-coefficient block the stages on
// index bits 0..5, then the sum over the blocks, which is all the pruned
// top stages leave of c0. It writes c0_splits(g) partial sums per (image,
// channel, limb) into the unused c0 slot of Yhat, coefficient j of split s at
// Yhat[b][i][0][l][64 s + 32 (j mod 2) + j / 2],
// and the masked inverse NTT then transforms c1 only and finishes c0 (adds
// the splits, the mask, and extracts).
constexpr uint32_t kMacC0 = 6;
bool mac_c0_ok(const ConvGeom &g);
uint32_t c0_splits(const ConvGeom &g);
// The masked inverse NTT with npw polynomials per workgroup (1, or 2 for
// elog <= 4) that starts at index bit pre (0, or kMacPre for logn >= 12), or
// that follows a MAC with pre = kMacC0.
bool intt_masked_ok(uint32_t logn, uint32_t elog, uint32_t npw, uint32_t pre);
bool mac_variant_ok(const MacShape &m);
// The MAC addresses its image and channel tiles with 32-bit byte offsets.
bool mac_offsets_fit(const ConvGeom &g, const MacShape &m);

// tab: optional input table (npolys == tab->n * ppi); input polynomials then
// come from tab->p[poly / ppi] + (poly % ppi) * N.
hipError_t launch_ntt_fwd(uint32_t logn, uint32_t elog, const uint32_t *in, uint32_t *out, size_t npolys,
                          const LimbConsts &c, const Twiddles &tw, hipStream_t st, const ImgPtrs *tab = nullptr,
                          uint32_t ppi = 0);
// out[p] = in[p] * s mod (x^N + 1, q_(p mod L)) over [P][N], where s is row
// p / mul_div (row 0 for all p when mul_div is 0; mul_div a multiple of L) of
// mul [..][L][N], which holds NTT(s) per limb as launch_ntt_fwd writes it
// (canonical, 16-byte aligned): forward NTT, product and inverse NTT in one
// kernel (in place allowed). keep_bits < logn: only outputs below 2^keep_bits
// are computed and stored (the rest of out is left as it was). addp: the
// polynomials are whole ciphertexts [..][2][L][N], and c0 of ciphertext r
// gains Delta (centred addp[r] mod q_l), addp [..][N] in [0, t) (no pruning).
hipError_t launch_ring_mul(uint32_t logn, uint32_t elog, const uint32_t *in, uint32_t *out, size_t npolys,
                           const uint32_t *mul, uint32_t mul_div, const LimbConsts &c, const Twiddles &tw,
                           hipStream_t st, uint32_t keep_bits = 32, const uint32_t *addp = nullptr);
// Full mode: in [P][N] -> out [P][N] (in place allowed). scale = false for
// inputs that carry the factor N^-1 already (the convolution's sums).
hipError_t launch_intt_full(uint32_t logn, uint32_t elog, const uint32_t *in, uint32_t *out, size_t npolys,
                            const LimbConsts &c, const Twiddles &tw, hipStream_t st, bool scale = true);
// p [..][L][N] (n words) *= N^-1 mod q_l, canonical.
hipError_t launch_scale_ninv(uint32_t *p, size_t n, uint32_t N, const LimbConsts &c, hipStream_t st);
// Masked mode: in = Yhat [B][O][2][L][N]; c1 polys go to c1_out [B][O][L][N],
// c0 polys are extracted with the mask into c0_ext [B][c_out][L][ho][wo].
// tab: optional per-image output tables (tab->n == B). npw: polynomials per
// workgroup; pre: stages already applied by the MAC (0 or kMacPre).
hipError_t launch_intt_masked(const ConvGeom &g, uint32_t logn, uint32_t elog, uint32_t npw, uint32_t pre,
                              const uint32_t *yhat,
                              const uint32_t *mask, uint32_t *c0_ext, uint32_t *c1_out, uint32_t B,
                              const LimbConsts &c, const Twiddles &tw, hipStream_t st, const OutPtrs *tab = nullptr);
// what: weights in the blocked layout of launch_weight_block, g.w_ld channels
// per block (a launch over channels [i0, i0 + g.c_out) of a larger layer
// passes what + 64 i0 and keeps the layer's w_ld). max_wgs > 0 caps the grid
// of the DMA-staged form (its workgroups then loop over the tiles); the other
// forms ignore it.
hipError_t launch_mac(const ConvGeom &g, const MacShape &m, const uint32_t *xhat, const uint32_t *what,
                      uint32_t *yhat, uint32_t B, const LimbConsts &c, const Twiddles &tw, hipStream_t st,
                      uint32_t max_wgs = 0);
hipError_t launch_weight_scatter(const ConvGeom &g, const int8_t *filters, uint32_t *w, const LimbConsts &c,
                                 hipStream_t st);
// NTT-domain weights from [c][g][l][N] (c_out channels, G_w polynomials each)
// to the multiply-accumulate's blocked layout [l][kb][g][c][64] (kb < N / 64;
// w_ld = c_out): per input ciphertext, the 64-coefficient blocks of
// consecutive channels are one run. dst must not overlap src.
hipError_t launch_weight_block(const uint32_t *src, uint32_t *dst, uint32_t c_out, uint32_t G_w, uint32_t L,
                               uint32_t N, hipStream_t st);
hipError_t launch_fill_zero(uint32_t *p, size_t n, hipStream_t st);
hipError_t launch_mask_extract(const ConvGeom &g, const uint32_t *ct_out, const uint32_t *mask, uint32_t *c0_ext,
                               uint32_t *c1_out, uint32_t B, const LimbConsts &c, hipStream_t st);
// Adds to *count (device) the number of words of np polynomials [..][L][N]
// that are >= the prime of their limb.
hipError_t launch_count_noncanonical(const uint32_t *p, size_t np, uint32_t N, const LimbConsts &k,
                                     unsigned long long *count, hipStream_t st);
// Register-only VALU probe `kind` (0 simple add/sub, 1 mul_lo/mul_hi, 2
// mad_u64_u32, 3 inverse butterflies) over nwg workgroups of 256 threads.
hipError_t launch_probe(int kind, uint32_t nwg, uint32_t iters, uint32_t q, const uint2 *tw, uint32_t *out,
                        hipStream_t st);
hipError_t launch_pointwise_mul(const uint32_t *a, const uint32_t *b, uint32_t *c, size_t npolys, uint32_t N,
                                const LimbConsts &k, hipStream_t st);

// ---------------------------------------------------------------- client side (hc_client.hip)
// Exact BFV decoding m = round(t v / q) mod t of a phase v in [0, q) given by
// its residues v_l. With x_l = v_l (q / q_l)^-1 mod q_l, v = sum_l x_l q / q_l
// minus a multiple of q, so t v / q equals sum_l x_l t / q_l up to a multiple
// of t; t / q_l = a_l + tau_l / q_l with a_l an integer and tau_l = t mod q_l.
// The fractions x_l tau_l / q_l are summed in 160-bit fixed point (phi_l =
// floor(tau_l 2^160 / q_l)): the sum is low by less than 2^-128, while the
// exact sum plus 1/2 is at least 1 / (2q) > 2^-121 away from an integer
// (2q does not divide an odd numerator), so the rounding is exact.
struct DecodeConsts {
  uint32_t qt[kMaxLimbs], qt_p[kMaxLimbs];  // (q / q_l)^-1 mod q_l and its Shoup constant
  uint32_t a[kMaxLimbs];                    // floor(t / q_l) mod t
  uint32_t phi[kMaxLimbs][5];               // floor(tau_l 2^160 / q_l), least significant word first
};
// Input geometry of a layer's direct encoding beyond ConvGeom.
struct EncGeom {
  uint32_t h, w;          // activation size as given
  uint32_t sub;           // client-side subsampling factor (1 if none)
  uint32_t pad;           // (f - 1) / 2
  uint32_t h_enc, w_enc;  // encoded (subsampled) size
  uint32_t h_pad;         // h_enc + 2 pad
  uint32_t rows_per_ct;   // padded rows one input ciphertext holds (h_pad, or R_o + f - 1 when tiled)
};
// ct[b][g] = ct_zero[b][g] + Delta * m_(b,g): c0 gains Delta times the
// direct-encoded, centred activations act [B][c_in][h][w]; c1 is copied
// unless copy_c1 is false (ct == ct_zero).
hipError_t launch_encrypt_online(const ConvGeom &g, const EncGeom &e, const uint32_t *act, const uint32_t *ct_zero,
                                 uint32_t *ct, uint32_t B, bool copy_c1, const LimbConsts &c, hipStream_t st);
// ct [n_ct][2][L][N] <- (-(as + e) mod q_l, a) from a, as = a * s ([n_ct][L][N])
// and e [n_ct][N] (signed, |e| < q_l).
hipError_t launch_encrypt_zero(const uint32_t *a, const uint32_t *as, const int32_t *e, uint32_t *ct, size_t n_ct,
                               uint32_t N, const LimbConsts &c, hipStream_t st);
// Batch encoding helpers (x^2 + x protocol). lift: out[c][l][k] = centred(mult * p[c][k] mod t)
// mod q_l for plaintexts p [n][N] in [0, t) (mult 1 or 2). add_plain: c0 of ct [n][2][L][N]
// += Delta_l (centred p[c] mod q_l).
hipError_t launch_lift_plain(const uint32_t *p, uint32_t *out, size_t n, uint32_t N, uint32_t mult,
                             const LimbConsts &c, hipStream_t st);
hipError_t launch_add_plain(uint32_t *ct, const uint32_t *p, size_t n, uint32_t N, const LimbConsts &c,
                            hipStream_t st);
// Server step 2 of the x^2 + x protocol: ct = ct_x - ct_y + Delta * enc(r^2 - r + v mod t)
// under the layer's direct encoding, r and v [B][c_in][h][w] in [0, t) (ct may be ct_x or ct_y).
hipError_t launch_act_combine(const ConvGeom &g, const EncGeom &e, const uint32_t *ct_x, const uint32_t *ct_y,
                              const uint32_t *r, const uint32_t *v, uint32_t *ct, uint32_t B, const LimbConsts &c,
                              hipStream_t st);
// ---------------------------------------------------------------- coefficient-domain conv (hc_direct.hip)
// bias[l] = q_l ceil(2^55 / q_l): added to a signed 64-bit sum |acc| < 2^54 it
// gives a value in [0, 2^57) with the same residue.
struct DirectConsts {
  uint64_t bias[kMaxLimbs];
};
// Algorithm 1 in the coefficient domain for an untiled layer, with the mask
// add and extraction: c0_ext and c1_out as launch_intt_masked writes them.
// wt: int32 filters [wt_rows][c_in][f f], wt_rows a multiple of 16 >= c_out,
// rows beyond c_out zero. Needs c_in f f <= 2^17 (the sum bound).
hipError_t launch_conv_direct(const ConvGeom &g, const uint32_t *ct, const int32_t *wt, uint32_t wt_rows,
                              const uint32_t *mask, uint32_t *c0, uint32_t *c1, uint32_t B, const DirectConsts &d,
                              const LimbConsts &c, hipStream_t st);
// c1[c][l][:] = ct[c][1][l][:] for n_ct ciphertexts [n_ct][2][L][N].
hipError_t launch_gather_c1(const uint32_t *ct, uint32_t *c1, size_t n_ct, uint32_t L, uint32_t N, hipStream_t st);
// m[b][i][oy][ox] = decode(c0_ext[b][i][:][oy][ox] + c1s[b][(i, tau)][:][e]).
hipError_t launch_decrypt_extracted(const ConvGeom &g, const uint32_t *c0_ext, const uint32_t *c1s, uint32_t *m,
                                    uint32_t B, const LimbConsts &c, const DecodeConsts &d, hipStream_t st);
// m[c][k] = decode(ct[c][0][:][k] + c1s[c][:][k]).
hipError_t launch_decrypt_full(const uint32_t *ct, const uint32_t *c1s, uint32_t *m, size_t n_ct, uint32_t N,
                               const LimbConsts &c, const DecodeConsts &d, hipStream_t st);

// ---------------------------------------------------------------- conventional convolution (hc_cconv.hip)
// Slot layout of the conventional (batch-encoded) convolution: images of h w
// <= N/2 pixels in blocks of bsz = (N/2)/c_r slots of one slot row, c_r
// channels per row, c_n = 2 c_r per ciphertext; R = c_n f^2 rotations.
struct CcGeom {
  uint32_t N, logn, c_in, c_out, h, w, f, p;
  uint32_t c_r, bsz, c_n, g_in, R;
};
// dig [n_ct][L D][L][N] <- the T-bit digits of c1 of ct [n_ct][2][L][N]
// (coefficient domain), each digit polynomial repeated in every limb.
hipError_t launch_cc_digits(const uint32_t *ct, uint32_t *dig, size_t n_ct, uint32_t N, uint32_t L, uint32_t T,
                            uint32_t D, hipStream_t st);
// out [n_ct][R][2][L][N] <- the automorphism x -> x^gal[r] and key switching
// of each ciphertext (NTT domain: xh its forward NTT, dh its digits' forward
// NTTs) with keys [R][LD][2][L][N]; gal[r] = 1 copies the ciphertext.
hipError_t launch_cc_keyswitch(const uint32_t *xh, const uint32_t *dh, const uint32_t *keys, const uint32_t *gal,
                               uint32_t *out, size_t n_ct, uint32_t R, uint32_t LD, uint32_t logn,
                               const LimbConsts &c, hipStream_t st);
// z [n_pt][N] <- the weight slot values (mod t) of plaintexts p0 .. p0 + n_pt
// - 1, in the batch encoding's slot order.
hipError_t launch_cc_weight_slots(const int8_t *filt, const uint32_t *rot_tab, const uint32_t *pow3, uint32_t *z,
                                  const CcGeom &cg, size_t p0, size_t n_pt, uint32_t t, hipStream_t st);
// Rotation-order slots (dir 0) to the batch encoding's order, or back (dir 1).
hipError_t launch_cc_slot_perm(const uint32_t *in, uint32_t *out, const uint32_t *pow3, size_t n, uint32_t logn,
                               int dir, hipStream_t st);
// keys [R][LD][2][L][N] (NTT domain) from ah, eh [R][LD][L][N] and sh [L][N].
hipError_t launch_cc_keygen(const uint32_t *ah, const uint32_t *eh, const uint32_t *sh, const uint32_t *gal,
                            uint32_t *keys, uint32_t R, uint32_t LD, uint32_t D, uint32_t T, uint32_t logn,
                            const LimbConsts &c, hipStream_t st);
// out [n][L][N] <- signed e [n][N] (|e| < q_l) as residues.
hipError_t launch_cc_lift_signed(const int32_t *e, uint32_t *out, size_t n, uint32_t N, const LimbConsts &c,
                                 hipStream_t st);

}  // namespace hc
