/*
 * Algorithm 1 (Proposed convolution) of Flash, arXiv 2401.16732, in plain C.
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle. Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg load it. It shares no code with
 * the GPU library.
 *
 * For output channel i and row tile tau (one polynomial p of the ciphertext,
 * one RNS limb q):
 *     partial = 0
 *     for each input channel j:
 *         c = x[ciphertext holding (j, tau)]
 *         t = sum over taps k of DRot(c, s_k) * f[i][j][k]      (CMult + DRot)
 *         partial += DRot(t, o_j)
 *     y = partial mod q                                          (one reduction)
 * DRot(c, step) is c(x) * x^(-step) mod x^n + 1 (eq. drot); coefficient m of
 * the result is (-1)^floor((m + step) / n) * c[(m + step) mod n] (closed form
 * in the Appendix A proof). Sums are kept unreduced in int64, the paper's lazy
 * reduction (Employing Lazy Reduction in Convolution): |c| < 2^31, |f| <= 128,
 * at most 49 taps and 2^12 channels keep |partial| below 2^57.
 *
 * The layout (tap shifts s_k, channel offsets o_j, which ciphertext holds
 * (j, tau)) is supplied by the caller.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the OpenMP loops below will use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* dst += DRot(src, step) * w  (w = 1 for the channel alignment). */
static void drot_axpy(int64_t *dst, const int64_t *src, uint32_t n, uint32_t step, int64_t w)
{
    for (uint32_t m = 0; m < n; ++m) {
        uint32_t k = m + step;
        if (k < n)
            dst[m] += w * src[k];
        else
            dst[m] -= w * src[k - n];
    }
}

static void drot_axpy_u32(int64_t *dst, const uint32_t *src, uint32_t n, uint32_t step, int64_t w)
{
    for (uint32_t m = 0; m < n; ++m) {
        uint32_t k = m + step;
        if (k < n)
            dst[m] += w * (int64_t)src[k];
        else
            dst[m] -= w * (int64_t)src[k - n];
    }
}

/*
 * One layer on one image.
 *   x        : input ciphertexts [G][2][L][n]
 *   in_ct    : [c_i * T]   in_ct[j*T + tau] = index of the ciphertext holding (j, tau)
 *   chan_off : [c_i]       o_j
 *   tap_off  : [n_taps]    s_k
 *   filters  : [c_o][c_i][n_taps] int8
 *   outs     : [n_out]     output channels to compute
 *   y        : [n_out * T][2][L][n]
 * Returns 0, or -1 on allocation failure.
 */
int oracle_alg1_layer(uint32_t n, uint32_t L, const uint32_t *q, uint32_t c_i, uint32_t T,
                      uint32_t n_taps, const uint32_t *tap_off, const uint32_t *chan_off,
                      const uint32_t *in_ct, const int8_t *filters, const uint32_t *x,
                      uint32_t n_out, const uint32_t *outs, uint32_t *y)
{
    int64_t jobs = (int64_t)n_out * T * 2 * L;
    int err = 0;
#pragma omp parallel
    {
        int64_t *t = (int64_t *)malloc(sizeof(int64_t) * n);
        int64_t *partial = (int64_t *)malloc(sizeof(int64_t) * n);
        if (!t || !partial) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t job = 0; job < jobs; ++job) {
            if (!t || !partial) continue;
            uint32_t l = (uint32_t)(job % L);
            uint32_t p = (uint32_t)((job / L) % 2);
            uint32_t tau = (uint32_t)((job / (2 * L)) % T);
            uint32_t oi = (uint32_t)(job / (2 * (int64_t)L * T));
            uint32_t i = outs[oi];
            memset(partial, 0, sizeof(int64_t) * n);
            for (uint32_t j = 0; j < c_i; ++j) {
                const uint32_t *c = x + (((size_t)in_ct[(size_t)j * T + tau] * 2 + p) * L + l) * n;
                const int8_t *fk = filters + ((size_t)i * c_i + j) * n_taps;
                memset(t, 0, sizeof(int64_t) * n);
                for (uint32_t k = 0; k < n_taps; ++k)
                    if (fk[k] != 0)
                        drot_axpy_u32(t, c, n, tap_off[k], (int64_t)fk[k]);
                drot_axpy(partial, t, n, chan_off[j], 1);
            }
            uint32_t *out = y + (((size_t)oi * T + tau) * 2 + p) * L * n + (size_t)l * n;
            int64_t ql = (int64_t)q[l];
            for (uint32_t m = 0; m < n; ++m) {
                int64_t r = partial[m] % ql;
                out[m] = (uint32_t)(r < 0 ? r + ql : r);
            }
        }
        free(t);
        free(partial);
    }
    return err ? -1 : 0;
}

/*
 * Selected coefficients of Algorithm 1's output, by the closed form of the
 * composed rotations: with e = o_j + s_k (< n),
 *     y[m] = sum_j sum_k f[i][j][k] * (-1)^floor((m + e) / n) * c_(j,tau)[(m + e) mod n]  mod q.
 * Point r asks for (output channel pt_i[r], tile pt_tau[r], poly pt_p[r],
 * limb pt_l[r], coefficient pt_m[r]); the answer goes to val[r].
 */
void oracle_alg1_points(uint32_t n, uint32_t L, const uint32_t *q, uint32_t c_i, uint32_t T,
                        uint32_t n_taps, const uint32_t *tap_off, const uint32_t *chan_off,
                        const uint32_t *in_ct, const int8_t *filters, const uint32_t *x,
                        uint64_t n_pts, const uint32_t *pt_i, const uint32_t *pt_tau,
                        const uint32_t *pt_p, const uint32_t *pt_l, const uint32_t *pt_m,
                        uint32_t *val)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < (int64_t)n_pts; ++r) {
        uint32_t i = pt_i[r], tau = pt_tau[r], p = pt_p[r], l = pt_l[r], m = pt_m[r];
        int64_t acc = 0;
        for (uint32_t j = 0; j < c_i; ++j) {
            const uint32_t *c = x + (((size_t)in_ct[(size_t)j * T + tau] * 2 + p) * L + l) * n;
            const int8_t *fk = filters + ((size_t)i * c_i + j) * n_taps;
            for (uint32_t k = 0; k < n_taps; ++k) {
                uint32_t idx = m + chan_off[j] + tap_off[k];
                int64_t v = (int64_t)c[idx % n];
                if ((idx / n) % 2 == 1) v = -v;
                acc += (int64_t)fk[k] * v;
            }
        }
        int64_t ql = (int64_t)q[l];
        int64_t rr = acc % ql;
        val[r] = (uint32_t)(rr < 0 ? rr + ql : rr);
    }
}

/*
 * Freivalds combination of one layer's outputs over output channels, for one
 * image: for each tile tau, poly p and limb l,
 *     z[tau][p][l][m] = sum_i rho[l][i] y_(i,tau)[p][l][m]   mod q_l.
 * The tap positions e = o_j + s_k do not depend on i, so this equals the
 * closed form above with the combined filter f'[j][k] = sum_i rho[l][i] f[i][j][k]
 * mod q_l in place of f[i] (n a power of two):
 *     z[m] = sum_j sum_k f'[j][k] (-1)^floor((m + e) / n) c_(j,tau)[(m + e) mod n]  mod q_l,
 * which costs 1 / c_o of the layer. f' is no longer small, so products
 * (< 2^60) are summed in uint64 and reduced every 8 terms.
 *   rho : [L][c_o] residues
 *   z   : [T][2][L][n]
 */
void oracle_freivalds(uint32_t n, uint32_t L, const uint32_t *q, uint32_t c_i, uint32_t c_o, uint32_t T,
                      uint32_t n_taps, const uint32_t *tap_off, const uint32_t *chan_off,
                      const uint32_t *in_ct, const int8_t *filters, const uint32_t *x,
                      const uint32_t *rho, uint32_t *z)
{
    size_t nf = (size_t)c_i * n_taps;
    uint64_t *fc = (uint64_t *)malloc(sizeof(uint64_t) * nf * L);
    if (!fc)
        abort();
    for (uint32_t l = 0; l < L; ++l) {
        uint64_t ql = q[l];
        for (size_t jk = 0; jk < nf; ++jk) {
            uint64_t acc = 0;
            for (uint32_t i = 0; i < c_o; ++i) {
                int64_t f = filters[(size_t)i * nf + jk];
                uint64_t fm = f < 0 ? ql - (uint64_t)(-f) : (uint64_t)f;
                acc = (acc + (uint64_t)rho[(size_t)l * c_o + i] % ql * fm) % ql;
            }
            fc[(size_t)l * nf + jk] = acc;
        }
    }
    uint32_t logn = 0;
    while ((1u << logn) < n)
        ++logn;
    const uint32_t MB = 256;  /* coefficients per work item */
    int64_t blocks = (int64_t)((n + MB - 1) / MB);
    int64_t items = (int64_t)T * 2 * L * blocks;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t it = 0; it < items; ++it) {
        uint32_t mb = (uint32_t)(it % blocks);
        uint32_t l = (uint32_t)((it / blocks) % L);
        uint32_t p = (uint32_t)((it / (blocks * L)) % 2);
        uint32_t tau = (uint32_t)(it / (blocks * L * 2));
        uint64_t ql = q[l];
        const uint64_t *fl = fc + (size_t)l * nf;
        uint32_t m0 = mb * MB, m1 = m0 + MB < n ? m0 + MB : n;
        uint64_t acc[256];
        memset(acc, 0, sizeof(acc));
        uint32_t terms = 0;
        for (uint32_t j = 0; j < c_i; ++j) {
            const uint32_t *c = x + (((size_t)in_ct[(size_t)j * T + tau] * 2 + p) * L + l) * n;
            for (uint32_t k = 0; k < n_taps; ++k) {
                uint64_t w = fl[(size_t)j * n_taps + k];
                uint32_t e = chan_off[j] + tap_off[k];
                for (uint32_t m = m0; m < m1; ++m) {
                    uint32_t idx = m + e;
                    uint64_t v = c[idx & (n - 1)];
                    if (v >= ql)
                        v %= ql;
                    if (((idx >> logn) & 1u) && v != 0)
                        v = ql - v;
                    acc[m - m0] += w * v;
                }
                if (++terms == 8) {
                    for (uint32_t m = m0; m < m1; ++m)
                        acc[m - m0] %= ql;
                    terms = 0;
                }
            }
        }
        for (uint32_t m = m0; m < m1; ++m)
            z[(((size_t)tau * 2 + p) * L + l) * n + m] = (uint32_t)(acc[m - m0] % ql);
    }
    free(fc);
}

/* Cap the OpenMP threads of the calls above (n >= 1); returns the new count. */
int oracle_set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads >= 1)
        omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/*
 * Schoolbook negacyclic product c = a b mod (x^n + 1, q) of residue vectors
 * (a[i], b[j] < q < 2^31): c_k = sum_{i+j=k} a_i b_j - sum_{i+j=k+n} a_i b_j,
 * summed in unsigned 128-bit integers (positive and negative parts apart) and
 * reduced once per coefficient.
 */
void oracle_negacyclic_mul(uint32_t n, uint64_t q, const uint64_t *a, const uint64_t *b, uint64_t *c)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < (int64_t)n; ++k) {
        unsigned __int128 pos = 0, neg = 0;
        for (uint32_t i = 0; i <= (uint32_t)k; ++i)
            pos += (unsigned __int128)a[i] * b[k - i];
        for (uint32_t i = (uint32_t)k + 1; i < n; ++i)
            neg += (unsigned __int128)a[i] * b[(uint32_t)k + n - i];
        uint64_t p = (uint64_t)(pos % q), m = (uint64_t)(neg % q);
        c[k] = p >= m ? p - m : p + q - m;
    }
}
