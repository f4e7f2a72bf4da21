/*
 * Plain CPU oracle for the X-engine cross-multiply-accumulate (CMAC).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * What it computes (paper: Section 2.3 "X-engine" defines the X-engine as the
 * conjugate multiplication and accumulation of channelised voltages; Eq. 2 in
 * Section 3.2 "Phase testing" defines a visibility as the time average of
 * S1* . S2):
 *
 *   for every channel f, every input i and every input j <= i,
 *     V_ij[f] = sum over t of  x_i[f,t] * conj(x_j[f,t])
 *     Re V_ij = sum (re_i re_j + im_i im_j)
 *     Im V_ij = sum (im_i re_j - re_i im_j)
 *
 * stored at pair index p = i(i+1)/2 + j (row-major lower triangle, autos
 * included).  The lower-triangle entry equals <S1* S2> of Eq. 2 with
 * S1 = x_j and S2 = x_i.
 *
 * Input formats (Section 2.1 "F-engine": the channelised data are truncated
 * to 4-bit real + 4-bit imaginary; Section 2.3: the fluff step widens them to
 * 8-bit + 8-bit):
 *   bits = 4 : one byte per (t, f, input); high nibble = real part, low
 *              nibble = imaginary part, each 4-bit two's complement [-8, 7].
 *   bits = 8 : two bytes per (t, f, input): int8 real then int8 imaginary.
 * Layout: time-major [T][F][N] (the corner-turned order in which blocks
 * arrive), so sample (t, f, i) starts at byte ((t*F + f)*N + i) * bytes.
 *
 * Accumulation is in int64 (exact for any T that fits memory) or in double
 * (exact while every partial sum is an integer below 2^53).  The int64
 * result is not narrowed here: the caller checks it against the int32 range.
 */
#include <stdint.h>
#include <stdlib.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

/* Sign-extend a 4-bit two's-complement field. */
static int sext4(unsigned v)
{
    v &= 15u;
    return (v & 8u) ? (int)v - 16 : (int)v;
}

/* Decode channel f of the input into re[i*T + t], im[i*T + t]. */
static void decode_channel(const uint8_t *v, int bits, int64_t T, int64_t F,
                           int64_t N, int64_t f, int *re, int *im)
{
    for (int64_t t = 0; t < T; ++t) {
        for (int64_t i = 0; i < N; ++i) {
            if (bits == 4) {
                uint8_t b = v[(t * F + f) * N + i];
                re[i * T + t] = sext4(b >> 4);
                im[i * T + t] = sext4(b);
            } else {
                const int8_t *s = (const int8_t *)v + ((t * F + f) * N + i) * 2;
                re[i * T + t] = s[0];
                im[i * T + t] = s[1];
            }
        }
    }
}

static int check_args(const uint8_t *v, int bits, int64_t T, int64_t F,
                      int64_t N, const int64_t *chans, int64_t n_sel,
                      const void *out)
{
    if (!v || !out || (bits != 4 && bits != 8) || T < 0 || F < 1 || N < 1 ||
        n_sel < 0)
        return ORACLE_EINVAL;
    for (int64_t s = 0; s < n_sel; ++s) {
        int64_t f = chans ? chans[s] : s;
        if (f < 0 || f >= F)
            return ORACLE_EINVAL;
    }
    return ORACLE_OK;
}

/*
 * Integer oracle.  chans lists the channels to correlate (NULL = channels
 * 0..n_sel-1).  out is [n_sel][P][2] int64 with P = N(N+1)/2, (re, im).
 */
int oracle_xcorr_i64(const uint8_t *v, int bits, int64_t T, int64_t F,
                     int64_t N, const int64_t *chans, int64_t n_sel,
                     int64_t *out)
{
    int rc = check_args(v, bits, T, F, N, chans, n_sel, out);
    if (rc)
        return rc;
    const int64_t P = N * (N + 1) / 2;
    int *re = malloc(sizeof(int) * (size_t)(N * (T ? T : 1)));
    int *im = malloc(sizeof(int) * (size_t)(N * (T ? T : 1)));
    if (!re || !im) {
        free(re);
        free(im);
        return ORACLE_ENOMEM;
    }
    for (int64_t s = 0; s < n_sel; ++s) {
        int64_t f = chans ? chans[s] : s;
        decode_channel(v, bits, T, F, N, f, re, im);
        for (int64_t i = 0; i < N; ++i) {
            for (int64_t j = 0; j <= i; ++j) {
                int64_t acc_re = 0, acc_im = 0;
                for (int64_t t = 0; t < T; ++t) {
                    int64_t ri = re[i * T + t], ii = im[i * T + t];
                    int64_t rj = re[j * T + t], ij = im[j * T + t];
                    /* x_i * conj(x_j) */
                    acc_re += ri * rj + ii * ij;
                    acc_im += ii * rj - ri * ij;
                }
                int64_t p = i * (i + 1) / 2 + j;
                out[(s * P + p) * 2 + 0] = acc_re;
                out[(s * P + p) * 2 + 1] = acc_im;
            }
        }
    }
    free(re);
    free(im);
    return ORACLE_OK;
}

/*
 * Same loop with double accumulators (the FP64 oracle used to state the
 * error of the half-precision path).  out is [n_sel][P][2] double.
 */
int oracle_xcorr_f64(const uint8_t *v, int bits, int64_t T, int64_t F,
                     int64_t N, const int64_t *chans, int64_t n_sel,
                     double *out)
{
    int rc = check_args(v, bits, T, F, N, chans, n_sel, out);
    if (rc)
        return rc;
    const int64_t P = N * (N + 1) / 2;
    int *re = malloc(sizeof(int) * (size_t)(N * (T ? T : 1)));
    int *im = malloc(sizeof(int) * (size_t)(N * (T ? T : 1)));
    if (!re || !im) {
        free(re);
        free(im);
        return ORACLE_ENOMEM;
    }
    for (int64_t s = 0; s < n_sel; ++s) {
        int64_t f = chans ? chans[s] : s;
        decode_channel(v, bits, T, F, N, f, re, im);
        for (int64_t i = 0; i < N; ++i) {
            for (int64_t j = 0; j <= i; ++j) {
                double acc_re = 0.0, acc_im = 0.0;
                for (int64_t t = 0; t < T; ++t) {
                    double ri = re[i * T + t], ii = im[i * T + t];
                    double rj = re[j * T + t], ij = im[j * T + t];
                    acc_re += ri * rj + ii * ij;
                    acc_im += ii * rj - ri * ij;
                }
                int64_t p = i * (i + 1) / 2 + j;
                out[(s * P + p) * 2 + 0] = acc_re;
                out[(s * P + p) * 2 + 1] = acc_im;
            }
        }
    }
    free(re);
    free(im);
    return ORACLE_OK;
}

/*
 * Single visibility (i, j) of channel f, for spot checks at full size where
 * correlating whole channels would take too long.  Requires j <= i.
 */
int oracle_xcorr_pair_i64(const uint8_t *v, int bits, int64_t T, int64_t F,
                          int64_t N, int64_t f, int64_t i, int64_t j,
                          int64_t *out_re_im)
{
    if (!v || !out_re_im || (bits != 4 && bits != 8) || T < 0 || F < 1 ||
        N < 1 || f < 0 || f >= F || i < 0 || i >= N || j < 0 || j > i)
        return ORACLE_EINVAL;
    int64_t acc_re = 0, acc_im = 0;
    for (int64_t t = 0; t < T; ++t) {
        int64_t ri, ii, rj, ij;
        if (bits == 4) {
            uint8_t bi = v[(t * F + f) * N + i], bj = v[(t * F + f) * N + j];
            ri = sext4(bi >> 4);
            ii = sext4(bi);
            rj = sext4(bj >> 4);
            ij = sext4(bj);
        } else {
            const int8_t *si = (const int8_t *)v + ((t * F + f) * N + i) * 2;
            const int8_t *sj = (const int8_t *)v + ((t * F + f) * N + j) * 2;
            ri = si[0];
            ii = si[1];
            rj = sj[0];
            ij = sj[1];
        }
        acc_re += ri * rj + ii * ij;
        acc_im += ii * rj - ri * ij;
    }
    out_re_im[0] = acc_re;
    out_re_im[1] = acc_im;
    return ORACLE_OK;
}
