/*
 * hc.h - C ABI of the MI355X homomorphic-convolution library (libhconv.so).
 *
 * The library computes the homomorphic convolution of Flash (arXiv 2401.16732,
 * section "Convolution with Direct Encoding", Algorithm 1) on one gfx950 GPU:
 * a server holding integer filters receives BFV ciphertexts of direct-encoded
 * (eq. de), zero-padded, channel-packed activations and returns one ciphertext
 * per output channel (Algorithm 1's output vector y), masked with its own random
 * share r (HAdd([[a]], [[r]]) in "Proposed Secure Computation of Polynomial
 * Activation Function").
 *
 * Algorithm 1 is a ring computation: DRot is multiplication by x^(-step) in
 * R_q = Z_q[x]/(x^n + 1) (eq. drot) and CMult is multiplication by a scalar, so
 * for output channel i its result is y_i = sum_g c_g * W_{i,g} with the sparse
 * weight polynomial W_{i,g}(x) = sum_{j in g} sum_taps f[i][j][tap] x^(-(o_j + s_tap)).
 * The library evaluates that same product as a negacyclic NTT of the inputs,
 * a pointwise multiply-accumulate over input ciphertexts against resident
 * NTT-domain weights, and an inverse NTT. Results are the canonical residues
 * of Algorithm 1's output, coefficient for coefficient.
 *
 * Arithmetic: RNS, q = prod_l q_l with L <= 4 primes q_l < 2^30, q_l = 1 mod 2n;
 * plaintext modulus t <= 2^30 (the paper's p); Delta = floor(q / t) (Notation
 * table). All values are uint32 residues; nothing is floating point.
 *
 * Layout of one convolution (fixed by hc_plan, public like the architecture):
 *   padding p = (f - 1) / 2, padded image h' x w' = (h + 2p) x (w + 2p), F = h' w'.
 *   F <= n: c_n = floor(n / F) channels per ciphertext; channel j sits in input
 *           ciphertext floor(j / c_n) at offset (j mod c_n) F, padded pixel (y, x)
 *           at that offset + y w' + x; one output ciphertext per output channel.
 *   F >  n: row tiles: tile tau of channel j holds padded rows
 *           [tau R_o, tau R_o + R_o + f - 1) at coefficient (y - tau R_o) w' + x,
 *           where R_o = stride * floor((floor(n / w') - f + 1) / stride);
 *           input ciphertext j T + tau, output ciphertext i T + tau.
 *   stride s > 1, f > 1: the stride-1 grid is computed; output pixel (oy, ox)
 *           is at coefficient (s oy - tau R_o) w' + s ox of output ciphertext (i, tau).
 *   f = 1, s > 1: the client encodes the subsampled input a[j][s y][s x] and the
 *           layer is the 1x1 stride-1 layer on the ceil(h/s) x ceil(w/s) grid.
 *
 * Device buffers (all uint32, contiguous, row-major, owned by the caller):
 *   ciphertexts      [B][cts][2][L][n]   (poly 0 = c0, poly 1 = c1; limb-major)
 *   mask r           [B][c_out][ho][wo]  values in [0, t)
 *   c0_ext           [B][c_out][L][ho][wo]
 *   c1_out           [B][out_cts][L][n]
 * Inputs must be canonical residues (in [0, q_l)); outputs always are. The
 * library trusts them, unless the environment variable HC_CHECK_INPUTS=1 is
 * set when a context is created: hc_conv and hc_conv_masked on its layers
 * then count the input ciphertexts' non-canonical words first (a device pass
 * and a wait for the stream, on a counter the context allocated; checks on one
 * context run one at a time) and return HC_EINVAL if there are any. That wait
 * cannot be recorded into a graph: with the check on, these calls return
 * HC_ESTATE on a stream under capture. hc_check_residues does the same count
 * on demand.
 *
 * Errors: every call returns hc_status. Argument and shape errors are
 * synchronous (HC_EINVAL / HC_EUNSUPPORTED); kernel faults are asynchronous and
 * surface from a later call or hc_sync as HC_EDEVICE. Nothing throws across
 * the ABI. A context and its layers are immutable after creation; calls on
 * different streams may run concurrently as long as their output and
 * workspace buffers are distinct.
 */
#ifndef HC_H
#define HC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HC_OK = 0,
    HC_EINVAL = -1,        /* bad argument (null pointer, size, value out of range) */
    HC_EUNSUPPORTED = -2,  /* valid request outside the supported shapes */
    HC_ENOMEM = -3,        /* device or host allocation failed */
    HC_EDEVICE = -4,       /* HIP runtime error, including an earlier asynchronous fault */
    HC_ESTATE = -5         /* object used in the wrong state (e.g. mismatched context) */
} hc_status;

typedef struct hc_ctx hc_ctx;
typedef struct hc_layer hc_layer;
typedef struct hc_batch hc_batch;

/* One convolution: c_in -> c_out channels on an h x w input, odd filter
 * width f, stride, 'same' zero padding (f - 1) / 2. */
typedef struct {
    uint32_t c_in, c_out, h, w, f, stride;
} hc_conv_shape;

/* The direct-encoding layout of one convolution (see the header comment). */
typedef struct {
    uint32_t sub;               /* client-side subsampling factor (f = 1, stride > 1), else 1 */
    uint32_t s;                 /* stride applied on the encoded grid */
    uint32_t h_enc, w_enc;      /* encoded input size (after subsampling) */
    uint32_t pad;               /* (f - 1) / 2 */
    uint32_t h_pad, w_pad;      /* h_enc + 2 pad, w_enc + 2 pad */
    uint32_t footprint;         /* F = h_pad * w_pad */
    uint32_t tiled;             /* 1 when F > n */
    uint32_t cn;                /* channels per input ciphertext */
    uint32_t tiles;             /* T: row tiles per channel (1 when untiled) */
    uint32_t rows_out_per_tile; /* R_o: stride-1 output rows per tile */
    uint32_t in_cts;            /* G: input ciphertexts per image */
    uint32_t w_cts;             /* weight polynomials per output channel (G, or c_in when tiled) */
    uint32_t out_cts;           /* O = c_out * T output ciphertexts per image */
    uint32_t ho, wo;            /* output size */
} hc_layout;

/* Launch-shape choices of a context (the autotuner's knobs). They change
 * speed only, never results: every supported value produces the same bits.
 * 0 selects the library default for that field. */
typedef struct {
    uint32_t fwd_elog;   /* forward NTT: 2^fwd_elog coefficients per thread */
    uint32_t inv_elog;   /* inverse NTT: 2^inv_elog coefficients per thread */
    uint32_t mac_rows;   /* multiply-accumulate: images per thread */
    uint32_t mac_cols;   /* multiply-accumulate: output channels per thread */
    uint32_t mac_row_groups;  /* waves per workgroup along images */
    uint32_t mac_col_groups;  /* waves per workgroup along output channels */
    uint32_t mac_depth;       /* input ciphertexts whose loads are in flight (2..4 as the tile
                                 allows; 0 = 2); with mac_lds = 2 the LDS stages (3, 4 or 6) */
    uint32_t mac_lds;         /* 1: the workgroup stages each input ciphertext's tile through LDS
                                 with 16-byte loads into registers; 2: the same tile loaded
                                 straight into LDS (buffer loads to LDS, no staging registers);
                                 0: every wave loads its operands itself */
    uint32_t inv_polys;       /* masked inverse NTT: polynomials per workgroup, sharing each twiddle
                                 load (1, or 2 when inv_elog <= 4; 0 = 1) */
    uint32_t mac_pre;         /* masked conv: inverse NTT stages the LDS- or DMA-staged MAC applies to its
                                 outputs before storing them (0, or 5 for 4x8 tiles, N >= 4096); 6
                                 (DMA-staged 4x8 tiles): the MAC carries out c0's whole pruned
                                 inverse transform (the stages inside each 64-coefficient block, then
                                 the sum over blocks, in splits) and the inverse NTT transforms c1
                                 only, then adds the splits and the mask - only on layers in one row
                                 tile whose extracted c0 coefficients all lie below 64 (the paper's
                                 small late feature maps); elsewhere it acts as 0. Same outputs. */
} hc_tuning;

/* Create a context on HIP device `hip_device`: ring degree N (power of two,
 * 1024..16384), L RNS primes (1..4), plaintext modulus t (2..2^30, below
 * 2 q_l for every prime, so centred plaintext values are residues).
 * primes: L distinct primes < 2^30 with q = 1 mod 2N, or NULL to choose the
 * L largest such primes, in descending order. Builds the NTT twiddle tables
 * on the device. The caller destroys it with hc_ctx_destroy. */
hc_status hc_ctx_create(uint32_t N, uint32_t L, const uint32_t *primes, uint64_t t, int hip_device,
                        hc_ctx **out);

/* Copy out the primes (L values) and Delta mod q_l (L values); either pointer may be NULL. */
hc_status hc_ctx_info(const hc_ctx *ctx, uint32_t *primes_out, uint32_t *delta_mod_q_out);
void hc_ctx_destroy(hc_ctx *ctx);

/* Set / read the context's launch shapes. Unsupported combinations return
 * HC_EUNSUPPORTED and leave the tuning unchanged. Not thread-safe against
 * calls in flight on the same context from other host threads. */
hc_status hc_ctx_set_tuning(hc_ctx *ctx, const hc_tuning *tuning);
hc_status hc_ctx_get_tuning(const hc_ctx *ctx, hc_tuning *out);

/* The layout of `shape` in this context (pure host computation). */
hc_status hc_plan(const hc_ctx *ctx, const hc_conv_shape *shape, hc_layout *out);

/* Host-only forms (no device needed): the layout for ring degree N, and the
 * parameters hc_ctx_create would choose (primes == NULL): the L largest primes
 * < 2^30 with q = 1 mod 2N in descending order, and Delta mod q_l. */
hc_status hc_plan_ring(uint32_t N, const hc_conv_shape *shape, hc_layout *out);
hc_status hc_ring_params(uint32_t N, uint32_t L, uint64_t t, uint32_t *primes_out, uint32_t *delta_mod_q_out);

/* Offline weight encoding (Algorithm 1's filters as W_{i,g}, then the forward
 * NTT, stored times N^-1 so that the convolution's inverse NTT needs no final
 * scaling). filters_host: int8 [c_out][c_in][f][f] in host memory, read during
 * the call. The NTT-domain weights stay resident in device memory owned by the
 * layer until hc_layer_destroy. `stream` is a hipStream_t (NULL = default);
 * the call returns after the encoding has been enqueued and the filters copied. */
hc_status hc_layer_create(hc_ctx *ctx, const hc_conv_shape *shape, const int8_t *filters_host, void *stream,
                          hc_layer **out);
void hc_layer_destroy(hc_layer *layer);
hc_status hc_layer_plan(const hc_layer *layer, hc_layout *out);

/* Bytes of device workspace hc_conv (masked = 0) or hc_conv_masked (masked = 1)
 * needs for a batch of B images. */
hc_status hc_workspace_size(const hc_layer *layer, uint32_t B, int masked, size_t *bytes);

/* Algorithm 1 for B images: ct_in [B][in_cts][2][L][N] -> ct_out
 * [B][out_cts][2][L][N], coefficient domain, canonical. ws: device workspace of
 * at least hc_workspace_size(layer, B, 0) bytes. Asynchronous on `stream`. */
hc_status hc_conv(const hc_layer *layer, const uint32_t *ct_in, uint32_t *ct_out, uint32_t B, void *ws,
                  size_t ws_bytes, void *stream);

/* Share conversion and extraction of hc_conv's output: for every output pixel
 * (b, i, oy, ox) at coefficient e of output ciphertext (i, tau):
 *   c0_ext[b][i][l][oy][ox] = ct_out[b][(i,tau)][0][l][e] + (Delta mod q_l) * (r_c mod q_l)  mod q_l
 * where r_c is mask[b][i][oy][ox] lifted to (-t/2, t/2]; and
 *   c1_out[b][o][l][:] = ct_out[b][o][1][l][:].
 * This adds the trivial ciphertext (Delta r, 0): the server cannot encrypt
 * (it has no key), so HAdd with [[r]] is a plaintext add to c0.
 * ct_out and c1_out must be 16-byte aligned. */
hc_status hc_mask_extract(const hc_layer *layer, const uint32_t *ct_out, const uint32_t *mask, uint32_t *c0_ext,
                          uint32_t *c1_out, uint32_t B, void *stream);

/* hc_conv followed by hc_mask_extract, fused into the inverse-NTT epilogue;
 * the full c0 of each output ciphertext is never written. ws: at least
 * hc_workspace_size(layer, B, 1) bytes. */
hc_status hc_conv_masked(const hc_layer *layer, const uint32_t *ct_in, const uint32_t *mask, uint32_t *c0_ext,
                         uint32_t *c1_out, uint32_t B, void *ws, size_t ws_bytes, void *stream);

/* Batched execution of several layers on B images each (all layers of a
 * network): the per-layer work (forward NTT, multiply-accumulate, inverse NTT
 * with mask and extraction) is recorded once into a HIP graph and replayed by
 * hc_batch_run. The layers must outlive the batch. The batch owns its
 * workspace (allocated here). */
hc_status hc_batch_create(hc_ctx *ctx, const hc_layer *const *layers, uint32_t n_layers, uint32_t B,
                          hc_batch **out);
hc_status hc_batch_workspace_bytes(const hc_batch *batch, size_t *bytes);

/* Run the batch: per layer k, ct_in[k], mask[k], c0_ext[k], c1_out[k] have
 * the hc_conv_masked shapes for B images. The graph is re-recorded when the
 * pointers differ from the previous call's. Asynchronous on `stream`. */
hc_status hc_batch_run(hc_batch *batch, const uint32_t *const *ct_in, const uint32_t *const *mask,
                       uint32_t *const *c0_ext, uint32_t *const *c1_out, void *stream);

/* Same work as hc_batch_run but launched kernel by kernel in stream order
 * (no graph); the reference for the graph path. */
hc_status hc_batch_run_eager(hc_batch *batch, const uint32_t *const *ct_in, const uint32_t *const *mask,
                             uint32_t *const *c0_ext, uint32_t *const *c1_out, void *stream);
void hc_batch_destroy(hc_batch *batch);

/* The batch's work as a two-stream pipeline over chunks of output channels,
 * launched kernel by kernel (no graph): per layer, the forward NTT, then for
 * each chunk of about chunk_bytes of multiply-accumulate output (a multiple of
 * the MAC's channel tile) the MAC on one stream and the inverse NTT with mask
 * and extraction of that chunk on a second stream, which waits for it; nbuf
 * (2..8) chunk buffers rotate, so the MAC of the next chunks (and layers) runs
 * beside the inverse NTT of earlier ones and a chunk's products can still be
 * in the last-level cache when they are read. Same outputs as hc_batch_run.
 * Allocates its own workspace on first use (and when a larger one is needed);
 * `stream` waits for the whole batch. Not for graph capture. */
hc_status hc_batch_run_pipelined(hc_batch *batch, const uint32_t *const *ct_in, const uint32_t *const *mask,
                                 uint32_t *const *c0_ext, uint32_t *const *c1_out, uint64_t chunk_bytes,
                                 uint32_t nbuf, void *stream);

/* Autotuner: for every layer of the batch, time each supported launch shape
 * of each stage (forward NTT threads per polynomial, MAC tile, inverse NTT
 * threads per polynomial) on the batch's own buffers (B images) and keep the
 * fastest per stage as the layer's shapes for B images. Results never change
 * (every shape gives the same bits). cache_path (may be NULL): a text file of
 * earlier results keyed by device, ring, B and layer shape; hits skip the
 * timing and new results are appended. Synchronous; the next hc_batch_run
 * re-records its graph. The buffers are overwritten. */
hc_status hc_batch_autotune(hc_batch *batch, const uint32_t *const *ct_in, const uint32_t *const *mask,
                            uint32_t *const *c0_ext, uint32_t *const *c1_out, void *stream, const char *cache_path);
/* Grid cap of the batch graph's multiply-accumulate launches (DMA-staged form,
 * mac_lds = 2; other forms ignore it): 0 launches one workgroup per tile;
 * cap >= 8 launches at most cap workgroups (rounded down to a multiple of 8),
 * each looping over its tiles, which leaves room on every compute unit for
 * the other chains' kernels. A new batch starts at 0. Same outputs either
 * way. The next hc_batch_run re-records its graph.
 * Set returns HC_EINVAL for 1..7. */
hc_status hc_batch_get_mac_cap(const hc_batch *batch, uint32_t *cap);
hc_status hc_batch_set_mac_cap(hc_batch *batch, uint32_t cap);
/* A layer's autotuned shapes and the batch size they apply to (0: none); clearing
 * removes every stored set and returns the layer to the context's shapes. */
hc_status hc_layer_get_tuning(const hc_layer *layer, uint32_t *batch_size, hc_tuning *out);
/* A layer keeps up to 4 autotuned shape sets, one per batch size (e.g. the
 * batched graph's and a single image's); runs of B images use the set tuned
 * for B, if any, else the context's. hc_layer_get_tuning gives the set stored
 * last; hc_layer_get_tuning_for the one for `batch_size` (HC_ESTATE and an
 * all-zero *out when there is none). */
hc_status hc_layer_get_tuning_for(const hc_layer *layer, uint32_t batch_size, hc_tuning *out);
hc_status hc_layer_clear_tuning(hc_layer *layer);

/* hc_batch_run_eager with a HIP event recorded on `stream` before and after
 * every kernel launch; waits for completion and adds the elapsed milliseconds
 * of each stage to stage_ms[0] (forward NTT of the inputs), stage_ms[1]
 * (multiply-accumulate) and stage_ms[2] (inverse NTT with mask and
 * extraction). For measurement; the events serialise the launches. */
hc_status hc_batch_run_timed(hc_batch *batch, const uint32_t *const *ct_in, const uint32_t *const *mask,
                             uint32_t *const *c0_ext, uint32_t *const *c1_out, void *stream, double *stage_ms);

/* ---------------------------------------------------------------- serving
 * Continuous batching of requests. A request is one image through every
 * convolution layer of one registered network. The server owns an HBM arena
 * of arena_bytes; a request is admitted, first come first served, when its
 * footprint (per layer: input ciphertexts, mask, c0_ext, c1_out of one image)
 * fits, and its inputs are then copied into the arena (from device or host
 * memory, which must stay valid until the request completes). Each
 * hc_server_step groups the next layer of every admitted request whose
 * previous layer has finished by (network, layer) and launches every group of
 * at most max_batch images as one batched forward NTT -> multiply-accumulate
 * -> masked inverse NTT, round robin over `streams` streams. Layers of one
 * request run in order. Steps never block. The results of a request do not
 * depend on which other requests it was grouped with. The server is not
 * thread-safe; drive it from one host thread. */
typedef struct hc_server hc_server;
typedef struct {
    uint64_t arena_bytes;  /* HBM for admitted requests */
    uint32_t max_batch;    /* images per launch group, 1..16 */
    uint32_t streams;      /* concurrent launch streams, 1..8 */
    uint32_t max_inflight; /* launch groups queued on the GPU at once (0: no limit). While the
                              limit is reached, ready requests wait and can join larger groups;
                              the largest ready group (then the oldest) launches first. */
} hc_server_config;
typedef struct {
    uint64_t submitted, admitted, completed, groups, images;  /* cumulative */
    uint64_t queued;       /* waiting for arena space */
    uint64_t arena_used, arena_bytes;
    uint64_t direct_groups;  /* cumulative: groups of one image run by the coefficient-domain conv */
} hc_server_stats;

hc_status hc_server_create(hc_ctx *ctx, const hc_server_config *cfg, hc_server **out);
/* Register a network (its layers must outlive the server); call before submitting. */
hc_status hc_server_add_net(hc_server *s, const hc_layer *const *layers, uint32_t n_layers, uint32_t *net_id);
hc_status hc_server_request_bytes(const hc_server *s, uint32_t net_id, size_t *bytes);
/* Queue a request: ct_in[k] / mask[k] are layer k's inputs for one image
 * ([in_cts][2][L][N] and [c_out][ho][wo]). */
hc_status hc_server_submit(hc_server *s, uint32_t net_id, const uint32_t *const *ct_in, const uint32_t *const *mask,
                           uint64_t *req_id);
hc_status hc_server_step(hc_server *s);
/* Ids of requests completed since the last poll (at most cap; *n returned). */
hc_status hc_server_poll(hc_server *s, uint64_t *ids, uint32_t cap, uint32_t *n);
/* Device pointers of a completed (or admitted) request's outputs for one layer:
 * c0_ext [c_out][L][ho][wo], c1_out [out_cts][L][N]; valid until release. */
hc_status hc_server_outputs(const hc_server *s, uint64_t req_id, uint32_t layer, uint32_t **c0_ext, uint32_t **c1_out);
/* Return a completed request's arena space. */
hc_status hc_server_release(hc_server *s, uint64_t req_id);
hc_status hc_server_get_stats(const hc_server *s, hc_server_stats *out);
/* Wait for all launched work. */
hc_status hc_server_sync(hc_server *s);
void hc_server_destroy(hc_server *s);

/* Negacyclic products c_k = a_k * b_k mod (x^N + 1, q_l) of `count` pairs of
 * polynomials laid out [count][L][N] (canonical residues), through the same
 * forward NTT, pointwise product and inverse NTT kernels as the convolution.
 * ws: at least 2 * count * L * N * 4 bytes. Exposes the NTT for testing. */
hc_status hc_poly_mul(const hc_ctx *ctx, const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t count,
                      void *ws, size_t ws_bytes, void *stream);

/* Count the words of npolys polynomials laid out [..][L][N] (device memory,
 * e.g. ciphertexts [B][cts][2][L][N] with npolys = B * cts * 2 * L) that are
 * not canonical, i.e. not below the prime of their limb, into *n_bad (host).
 * Enqueued on `stream`; the call waits for the stream. The input-validation
 * step of the interface (the same count HC_CHECK_INPUTS=1 runs in the conv
 * calls). */
hc_status hc_check_residues(const hc_ctx *ctx, const uint32_t *polys, size_t npolys, void *stream,
                            uint64_t *n_bad);

/* ------------------------------------------------------------ client side
 * The steps on either side of the convolution, for a client that runs on the
 * GPU (or for checking the server's outputs at full size). Plaintext values
 * are in [0, t) and are lifted to (-t/2, t/2] before Delta scales them
 * (plaintext coefficients of R_p, Background: Homomorphic Encryption).
 *
 * Direct encoding (eq. de) plus online encryption (Algorithm 2, section
 * "Moving Data-independent Operations to Offline Phase"): for each image b and
 * input ciphertext g of the layer, ct_in[b][g] = [[0]]_(b,g) + Delta * m_(b,g),
 * where m_(b,g) is the plaintext polynomial that the layout (header comment)
 * gives ciphertext g from act[b] (zero padding, channel packing, row tiles,
 * client-side subsampling); only c0 changes.
 *   act      [B][c_in][h][w] values in [0, t) (device; other values give a
 *            well-formed but meaningless ciphertext)
 *   ct_zero  [B][G][2][L][N] canonical encryptions of zero, one per ciphertext,
 *            made offline (c0 = -(a s + e), c1 = a; Table 2's private-key form)
 *   ct_in    [B][G][2][L][N] output, the conv's input; may be ct_zero itself
 *            (then only c0 is written), must not otherwise overlap it or act.
 * Enqueued on `stream`; no allocation. */
hc_status hc_encrypt_online(const hc_layer *layer, const uint32_t *act, const uint32_t *ct_zero, uint32_t *ct_in,
                            uint32_t B, void *stream);

/* The offline half of Algorithm 2: `count` private-key encryptions of zero
 * (Table 2's private-key form with m = 0), ct_zero[c] = (-(a_c s + e_c) mod q, a_c).
 * The random polynomials are inputs, drawn by the caller:
 *   a   [count][L][N]  uniform residues (canonical, device)
 *   sk  [L][N]         secret key residues s mod q_l (canonical, device)
 *   e   [count][N]     int32 error coefficients, |e| < q_l (device)
 *   ct_zero [count][2][L][N] output, must not overlap a or ws.
 * a * s is the negacyclic product through the NTT (the kernel decryption uses).
 * ws: at least (count + 1) L N words, 16-byte aligned. */
hc_status hc_encrypt_zero(const hc_ctx *ctx, const uint32_t *a, const uint32_t *sk, const int32_t *e,
                          uint32_t *ct_zero, uint32_t count, void *ws, size_t ws_bytes, void *stream);

/* BFV decryption (eq. bfv_dec): m = round(t [c1 s + c0]_q / q) mod t, rounded
 * half up and exact for every phase (the RNS rounding carries 160 fraction bits;
 * q < 2^120). The secret key sk is given as its residues [L][N] (s mod q_l,
 * canonical, device); c1 s is the negacyclic product through the forward NTT,
 * a pointwise product and the inverse NTT.
 *
 * hc_decrypt_extracted decrypts the masked conv's outputs (hc_conv_masked):
 * output pixel (i, oy, ox) has phase c0_ext[b][i][:][oy][ox] + (c1_out[b][(i,tau)] s)[e]
 * at its coefficient e (header comment); m [B][c_out][ho][wo] receives values in
 * [0, t), i.e. conv(a) + r mod t for a fresh encryption of a under mask r.
 * ws: hc_decrypt_workspace_size bytes, (B out_cts + 1) L N words, 16-byte aligned. */
hc_status hc_decrypt_workspace_size(const hc_layer *layer, uint32_t B, size_t *bytes);
hc_status hc_decrypt_extracted(const hc_layer *layer, const uint32_t *c0_ext, const uint32_t *c1_out,
                               const uint32_t *sk, uint32_t *m, uint32_t B, void *ws, size_t ws_bytes,
                               void *stream);
/* Decrypts `count` whole ciphertexts ct [count][2][L][N] into m [count][N]
 * (every coefficient, values in [0, t)). ws: at least (count + 1) L N words, 16-byte
 * aligned. */
hc_status hc_decrypt(const hc_ctx *ctx, const uint32_t *ct, const uint32_t *sk, uint32_t *m, uint32_t count,
                     void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ x^2 + x protocol
 * Section "Proposed Secure Computation of Polynomial Activation Function": the
 * client returns [[a + r]] under batch encoding, the server multiplies it slot
 * by slot with 2r and hides the product with v (step 1); the client returns
 * that vector re-encrypted under direct encoding, and the server combines it
 * with [[a^2 + 2ar + r^2 + a + r]] into [[a^2 + a]] (step 2). r, v are the
 * server's random vectors (inputs, drawn offline).
 *
 * Batch (slot) encoding needs a context whose t is a prime = 1 mod 2N (below
 * 2^30); other contexts return HC_EUNSUPPORTED. R_t = Z_t[x]/(x^N + 1) splits
 * into N slots, the evaluations at the roots of x^N + 1. Slot order (public, a
 * convention the paper leaves open): slot k is the evaluation at
 * psi^(2 brv(k) + 1), brv = bit reversal over log2 N bits, psi = the first
 * x^((t-1)/2N), x = 2, 3, ..., whose N-th power is -1.
 *
 * hc_batch_encode: p [n][N] <- the plaintext polynomials with slots z [n][N]
 *   (values in [0, t)); hc_batch_decode: z <- slots of p (z 16-byte aligned).
 * hc_encrypt_plain: ct = ct_zero + Delta * p for plaintext polynomials p
 *   [n][N] in [0, t) (Algorithm 2 for a batch-encoded message); ct_zero, ct
 *   [n][2][L][N]; ct may be ct_zero, must not otherwise overlap it.
 * Enqueued on `stream`; no allocation. */
hc_status hc_batch_encode(const hc_ctx *ctx, const uint32_t *z, uint32_t *p, uint32_t n, void *stream);
hc_status hc_batch_decode(const hc_ctx *ctx, const uint32_t *p, uint32_t *z, uint32_t n, void *stream);
hc_status hc_encrypt_plain(const hc_ctx *ctx, const uint32_t *p, const uint32_t *ct_zero, uint32_t *ct, uint32_t n,
                           void *stream);

/* Step 1: ct_out = PMult(ct_batch, encode(2r)) + encode(v), i.e. [[2r (a + r) + v]]
 * under batch encoding, for n_ct ciphertexts ct_batch [n_ct][2][L][N] with slot
 * vectors r, v [n_ct][N] in [0, t). PMult multiplies both components by the
 * centred plaintext polynomial in R_q (forward NTT, product, inverse NTT in one
 * kernel). ct_out may be ct_batch, must not otherwise overlap it.
 * ws: hc_act_workspace_size bytes ((L + 2) n_ct N words), 16-byte aligned. */
hc_status hc_act_workspace_size(const hc_ctx *ctx, uint32_t n_ct, size_t *bytes);
hc_status hc_act_pmult(const hc_ctx *ctx, const uint32_t *ct_batch, const uint32_t *r, const uint32_t *v,
                       uint32_t *ct_out, uint32_t n_ct, void *ws, size_t ws_bytes, void *stream);
/* Step 2, for the layer whose input the activation map is: ct_out = ct_x - ct_y
 * + Delta * enc(r^2 - r + v mod t), where ct_x, ct_y [B][G][2][L][N] are the
 * layer's direct-encoded input ciphertexts of a^2 + 2ar + r^2 + a + r and of
 * 2ar + 2r^2 + v, enc is the layer's direct encoding (header comment) and r, v
 * are [B][c_in][h][w] in [0, t); the result encrypts a^2 + a. ct_out may be
 * ct_x or ct_y, must not otherwise overlap them. Any t; no allocation. */
hc_status hc_act_combine(const hc_layer *layer, const uint32_t *ct_x, const uint32_t *ct_y, const uint32_t *r,
                         const uint32_t *v, uint32_t *ct_out, uint32_t B, void *stream);

/* Flash's own coefficient-domain convolution (Algorithm 1 as written: CMult of
 * DRot-ed inputs summed over taps and channels, in exact signed 64-bit sums,
 * section "Employing Lazy Reduction in Convolution"), with the same outputs as
 * hc_conv_masked, bit for bit. It reads the int8 filters instead of the
 * resident NTT-domain weights and needs no workspace, so it pays where c_n f^2
 * is small and the batch is small. Untiled layers with c_in f^2 <= 2^17
 * (HC_EUNSUPPORTED otherwise). Enqueued on `stream`; no allocation. */
hc_status hc_conv_masked_direct(const hc_layer *layer, const uint32_t *ct_in, const uint32_t *mask, uint32_t *c0_ext,
                                uint32_t *c1_out, uint32_t B, void *stream);

/* ------------------------------------------------------------ conventional convolution
 * The convolution the paper compares Flash's against (section "Conventional
 * Convolution"; HRot and eq. keySwitching in "Background: Homomorphic
 * Encryption"), for measuring that comparison (Table 9) on this GPU: batch
 * encoding, slot rotations by automorphism plus key switching, PMult by
 * plaintexts of weights, HAdd. Needs a context whose t is a prime = 1 mod 2N
 * (below 2^30), stride 1 and h w <= N/2 (HC_EUNSUPPORTED otherwise).
 *
 * Slots in rotation order (a convention the paper leaves open): two rows of
 * N/2; slot (r, c) is the evaluation at psi^(3^c) (row 0) or psi^(-3^c)
 * (row 1), psi as for hc_batch_encode; vectors are [2][N/2], row 0 first.
 * The automorphism x -> x^(3^k) shifts both rows left by k (the paper's
 * left-cyclic HRot), x -> x^(-1) exchanges them.
 *
 * Layout: c_r = the largest power of two with c_r h w <= N/2 channels per slot
 * row, each in a block of `block` = (N/2)/c_r slots (row-major pixels, the
 * rest zero); c_n = 2 c_r channels per ciphertext (input channel j of
 * ciphertext j / c_n at row (j mod c_n) / c_r, block (j mod c_n) mod c_r);
 * the output ciphertexts hold the output channels the same way (packed).
 * Rotations r = 0 .. c_n f^2 - 1 in the order (swap, d, ky, kx), swap slowest:
 * exchange the rows when swap, then shift left by d block + (ky - p) w + (kx - p)
 * (mod N/2); its Galois element is hc_cconv_info's galois[r]. Output ciphertext
 * o = sum over input ciphertexts g and rotations r of PMult(HRot(in_g, r),
 * pt(o, g, r)), where pt holds at each output slot the weight that the
 * rotated input's channel and pixel there carry (0 where the tap reads the
 * zero padding or a channel is absent). A rotation with element 1 is the
 * identity (no key switch).
 *
 * Key switching: c1 is split into D = ceil(30 / decomp_bits) digits of
 * decomp_bits bits per RNS limb (L D digits, digit (l, d) weighted by the CRT
 * basis element of limb l times 2^(decomp_bits d)); the digits go through the
 * automorphism and are multiplied by the switching keys (swk0, swk1) of the
 * rotation: c0' = c0(x^g) + sum_i swk0_i c1^(i)(x^g), c1' = sum_i swk1_i c1^(i)(x^g).
 * Keys are made on the client from the secret: swk0_i = -a_i s + e_i +
 * w_i s(x^g), swk1_i = a_i (hc_cconv_keygen).
 *
 * Buffers (uint32 residues unless stated, device, caller-owned):
 *   keys     [rotations][L D][2][L][N]  NTT domain (hc_cconv_keygen's output)
 *   ct_in    [B][g_in][2][L][N]   batch-encoded inputs, coefficient domain, canonical
 *   ct_out   [B][g_out][2][L][N]  coefficient domain, canonical
 * The layer owns its weight plaintexts (g_out g_in rotations L N words, NTT
 * domain) until hc_cconv_destroy. */
typedef struct hc_cconv hc_cconv;
typedef struct {
    uint32_t c_r, block, c_n;   /* channels per slot row, slots per channel block, channels per ciphertext */
    uint32_t g_in, g_out;       /* input / output ciphertexts per image */
    uint32_t rotations;         /* c_n f^2 */
    uint32_t decomp_bits, digits; /* bits per digit; digits per key (L D) */
} hc_cconv_layout;
hc_status hc_cconv_create(hc_ctx *ctx, const hc_conv_shape *shape, const int8_t *filters_host, uint32_t decomp_bits,
                          void *stream, hc_cconv **out);
void hc_cconv_destroy(hc_cconv *layer);
/* galois: NULL, or room for `rotations` values. */
hc_status hc_cconv_info(const hc_cconv *layer, hc_cconv_layout *out, uint32_t *galois);
hc_status hc_cconv_keys_size(const hc_cconv *layer, size_t *bytes);
hc_status hc_cconv_keygen_workspace_size(const hc_cconv *layer, size_t *bytes);
/* Client side: keys from the secret's residues sk [L][N], uniform residues
 * a [rotations][L D][L][N] and int32 errors e [rotations][L D][N] (|e| < q_l),
 * all drawn by the caller. ws: hc_cconv_keygen_workspace_size bytes. */
hc_status hc_cconv_keygen(const hc_cconv *layer, const uint32_t *sk, const uint32_t *a, const int32_t *e,
                          uint32_t *keys, void *ws, size_t ws_bytes, void *stream);
hc_status hc_cconv_workspace_size(const hc_cconv *layer, uint32_t B, size_t *bytes);
/* The convolution of B images. ws: hc_cconv_workspace_size bytes. Enqueued on
 * `stream`; no allocation. */
hc_status hc_cconv_run(const hc_cconv *layer, const uint32_t *keys, const uint32_t *ct_in, uint32_t *ct_out,
                       uint32_t B, void *ws, size_t ws_bytes, void *stream);
/* Rotation-order batch encoding of n slot vectors z [n][N] (values in [0, t))
 * into plaintext polynomials p [n][N], and decoding back (ws: n N words,
 * 16-byte aligned). z and p must not overlap. These two calls allocate a small
 * table and wait for the stream. */
hc_status hc_rot_encode(const hc_ctx *ctx, const uint32_t *z, uint32_t *p, uint32_t n, void *stream);
hc_status hc_rot_decode(const hc_ctx *ctx, const uint32_t *p, uint32_t *z, uint32_t n, void *ws, size_t ws_bytes,
                        void *stream);

/* ------------------------------------------------------------ measurement
 * Register-only VALU rate probes on HIP device `hip_device`, the ceilings the
 * kernels' roofline is priced against: independent chains of one instruction
 * class in registers, no memory traffic in the timed loop, 8 four-wave
 * workgroups per compute unit; one warm-up launch, then one launch timed with
 * HIP events. Rates are lane-operations (or butterflies) per second over the
 * whole device:
 *   simple_ops_per_s   32-bit integer add / sub
 *   mul_ops_per_s      32-bit integer multiply, low and high halves
 *   mad64_ops_per_s    v_mad_u64_u32 (the multiply-accumulate's instruction)
 *   butterflies_per_s  the inverse NTT's butterfly (Gentleman-Sande, Shoup
 *                      twiddle, lazy [0, 2q) range), compiled from the same
 *                      code as the inverse NTT kernels
 * compute_units and clock_hz are the device's reported unit count and peak
 * engine clock; measured_clock_hz is the engine clock during the simple-op
 * probe (shader cycle counter of its longest workgroup over the launch's
 * duration; every workgroup is resident for the whole launch). Synchronous;
 * allocates and frees a few kilobytes of device memory. */
typedef struct {
    double simple_ops_per_s, mul_ops_per_s, mad64_ops_per_s, butterflies_per_s;
    uint32_t compute_units;
    double clock_hz;
    double measured_clock_hz;
} hc_valu_rates;
hc_status hc_valu_probe(int hip_device, hc_valu_rates *out);

/* ------------------------------------------------------------ no allocation
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * hc_conv_masked without a workspace argument. Its scratch (the NTT-domain
 * inputs and products of one call, hc_workspace_size(layer, B, 1) bytes) is a
 * fixed device array of HC_NOALLOC_SCRATCH_BYTES per device, held by the
 * library until the process ends; the call allocates nothing and returns
 * HC_EINVAL when the layer needs more for B images (call it with fewer images,
 * or use hc_conv_masked). Every call on one device shares that device's array
 * and overwrites it completely before reading it: calls that overlap in time
 * on one device (other streams, other host threads) race and give wrong
 * results; order them on one stream. Same outputs as hc_conv_masked, bit for
 * bit. Asynchronous on `stream`. */
#define HC_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
hc_status hc_conv_masked_noalloc(const hc_layer *layer, const uint32_t *ct_in, const uint32_t *mask,
                                 uint32_t *c0_ext, uint32_t *c1_out, uint32_t B, void *stream);

/* Wait for all work on the context's device; reports earlier asynchronous faults. */
hc_status hc_sync(hc_ctx *ctx);
const char *hc_status_string(hc_status s);
/* Text of the last error on the calling thread (empty if none). */
const char *hc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HC_H */
