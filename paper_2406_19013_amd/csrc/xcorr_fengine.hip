// F-engine front end (paper Section 2.2): 8-bit ADC samples of each input ->
// polyphase filter bank of 2048 points with a 4-tap prototype -> real FFT ->
// 1024 channels -> per-(input, channel) EQ gain -> 4+4-bit requantisation ->
// corner turn into the X-engine's [T][F][N] order.
//
// One work-group = one spectrum m of 64 inputs; 8 waves, each filtering and
// transforming 8 of the inputs one after the other.  Per input and spectrum:
//   y[q] = sum_k h[k P + q] x[(m + k) P + q]            q < P = 2048
//   z[n] = y[2n] + i y[2n + 1]                          n < 1024
//   Z    = 1024-point complex DFT of z (radix 16 x 16 x 4, two LDS exchanges)
//   Y[c] = (Z[c] + Z*[N - c]) / 2 - i W^c (Z[c] - Z*[N - c]) / 2,  W = e^{-2 pi i / 2048}
//   code = pack(clip(rint(g Re Y)), clip(rint(g Im Y)))  for channels c < 1024
// The FIR coefficients a lane needs (4 taps x 16 sample pairs) stay in its
// registers for all 8 inputs; the codes of the 64 inputs are gathered in LDS
// and leave as one 64-byte row per (spectrum, channel).  Arithmetic in fp32;
// rounding is round-half-to-even.
#include "xcorr.h"
#include "xcorr_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

namespace xc {
namespace {

constexpr int kFeP = 2048;          // real points per spectrum
constexpr int kFeN = kFeP / 2;      // complex FFT size and channel count
constexpr int kFeTaps = 4;
constexpr int kFeGroup = 64;        // inputs per work-group
constexpr int kFeWaves = 8;
constexpr int kFeThreads = 64 * kFeWaves;
constexpr int kFeInputsPerWave = kFeGroup / kFeWaves;
constexpr int kFeBufStride = 17;                    // float2 per row of the pass-1 exchange (16 + 1 pad)
constexpr int kFeBufFloats = 2 * 64 * kFeBufStride;  // per wave: 64 rows
constexpr int kFeCodeStride = 80;                   // bytes per channel row of the code tile (64 + pad)

// ---- twiddle tables, computed at compile time in double ----------------------

// sin and cos of 2 pi num / den: quarter turns split off exactly in integer
// arithmetic, the remaining angle (below pi / 2) by Taylor series (16 terms
// reach double precision there)
struct SinCos {
    double s, c;
};
constexpr SinCos sincos_series(double t)
{
    double s = 0, c = 0, term_s = t, term_c = 1;
    for (int k = 0; k < 16; ++k) {
        s += term_s;
        c += term_c;
        term_s *= -t * t / ((2 * k + 2) * (2 * k + 3));
        term_c *= -t * t / ((2 * k + 1) * (2 * k + 2));
    }
    return {s, c};
}
constexpr SinCos sincos_turn(long num, long den)
{
    constexpr double kTwoPi = 6.283185307179586476925286766559;
    num %= den;
    if (num < 0)
        num += den;
    const long q = (4 * num) / den;           // quarter turns
    const long r = 4 * num - q * den;         // remainder, in units of 1 / (4 den) turn
    const SinCos b = sincos_series(kTwoPi * (double)r / (4.0 * den));
    switch (q) {
    case 0: return {b.s, b.c};
    case 1: return {b.c, -b.s};
    case 2: return {-b.s, -b.c};
    default: return {-b.c, b.s};
    }
}

template <int COUNT>
struct Table {
    float re[COUNT];
    float im[COUNT];
};
// W_N^e = exp(-2 pi i e / N)
constexpr Table<1024> make_tw_pass1()
{
    Table<1024> t{};
    for (int l = 0; l < 64; ++l)
        for (int k1 = 0; k1 < 16; ++k1) {
            const SinCos v = sincos_turn((long)l * k1, 1024);
            t.re[l * 16 + k1] = (float)v.c;
            t.im[l * 16 + k1] = (float)-v.s;
        }
    return t;
}
constexpr Table<64> make_tw_pass2()
{
    Table<64> t{};
    for (int m2 = 0; m2 < 4; ++m2)
        for (int j1 = 0; j1 < 16; ++j1) {
            const SinCos v = sincos_turn((long)m2 * j1, 64);
            t.re[m2 * 16 + j1] = (float)v.c;
            t.im[m2 * 16 + j1] = (float)-v.s;
        }
    return t;
}
constexpr Table<1024> make_tw_real()
{
    Table<1024> t{};
    for (int c = 0; c < 1024; ++c) {
        const SinCos v = sincos_turn(c, 2048);
        t.re[c] = (float)v.c;
        t.im[c] = (float)-v.s;
    }
    return t;
}
__device__ constexpr Table<1024> kTwPass1 = make_tw_pass1();
__device__ constexpr Table<64> kTwPass2 = make_tw_pass2();
__device__ constexpr Table<1024> kTwReal = make_tw_real();

// ---- complex helpers ----------------------------------------------------------

struct cf {
    float r, i;
};
__device__ __forceinline__ cf cadd(cf a, cf b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cf csub(cf a, cf b) { return {a.r - b.r, a.i - b.i}; }
__device__ __forceinline__ cf cmul(cf a, cf b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cf cmul_mi(cf a) { return {a.i, -a.r}; }   // a * (-i)

// forward 4-point DFT in place: x[k] = sum_n x[n] (-i)^{nk}
__device__ __forceinline__ void dft4(cf &x0, cf &x1, cf &x2, cf &x3)
{
    const cf a = cadd(x0, x2), b = csub(x0, x2), c = cadd(x1, x3), d = cmul_mi(csub(x1, x3));
    x0 = cadd(a, c);
    x2 = csub(a, c);
    x1 = cadd(b, d);
    x3 = csub(b, d);
}

// forward 16-point DFT of x[0..15] in place (4 x 4 with W16 twiddles); the
// output is in natural order
__device__ __forceinline__ void dft16(cf *x)
{
    // n = 4a + b: 4-point DFTs over a for each b -> U[b][c] (stored at x[4c + b]... )
    for (int b = 0; b < 4; ++b)
        dft4(x[b], x[4 + b], x[8 + b], x[12 + b]);   // x[4c + b] = U[b][c]
    // twiddles W16^{b c}
    constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508978f, r2 = 0.70710678118654752f;
    // (b, c) -> W16^{bc} = exp(-2 pi i b c / 16)
    x[4 * 1 + 1] = cmul(x[5], cf{c1, -s1});
    x[4 * 2 + 1] = cmul(x[9], cf{r2, -r2});
    x[4 * 3 + 1] = cmul(x[13], cf{s1, -c1});
    x[4 * 1 + 2] = cmul(x[6], cf{r2, -r2});
    x[4 * 2 + 2] = cmul_mi(x[10]);
    x[4 * 3 + 2] = cmul(x[14], cf{-r2, -r2});
    x[4 * 1 + 3] = cmul(x[7], cf{s1, -c1});
    x[4 * 2 + 3] = cmul(x[11], cf{-r2, -r2});
    x[4 * 3 + 3] = cmul(x[15], cf{-c1, s1});
    // 4-point DFTs over b for each c: X[c + 4 d] from x[4c + b]
    cf y[16];
    for (int c = 0; c < 4; ++c) {
        cf a0 = x[4 * c], a1 = x[4 * c + 1], a2 = x[4 * c + 2], a3 = x[4 * c + 3];
        dft4(a0, a1, a2, a3);
        y[c] = a0;
        y[c + 4] = a1;
        y[c + 8] = a2;
        y[c + 12] = a3;
    }
    for (int k = 0; k < 16; ++k)
        x[k] = y[k];
}

// this wave's LDS writes done before any lane reads them (and its reads done
// before the buffer is written again); the memory clobber keeps the compiler
// from moving LDS accesses across
__device__ __forceinline__ void lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

__device__ __forceinline__ int quant4(float v)
{
    const float r = __builtin_rintf(v);   // round half to even
    return (int)fminf(fmaxf(r, -8.0f), 7.0f);
}

struct FeArgs {
    const int8_t *adc;    // [N][S]
    int64_t S;            // samples per input
    int N;
    const float *h;       // [taps * P]
    const float *gains;   // [N][1024]
    int64_t n_spectra;
    void *out;            // CODES: uint8 [n_spectra][1024][N]; else float2 [N][n_spectra][1024]
};

// One wave's FFT of one (input, spectrum): returns the 16 channel values
// c = lane + 64 v (v < 16) of the real spectrum in y[v].
__device__ __forceinline__ void fe_transform(const FeArgs &a, int input, int64_t m, const float2 (&hc)[kFeTaps][16],
                                             float *buf, cf (&y)[16])
{
    const int lane = threadIdx.x & 63;
    // FIR: z[n] for n = 64 n1 + lane
    cf z[16];
    const int8_t *x = a.adc + (int64_t)input * a.S + m * kFeP + 2 * lane;
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) {
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int k = 0; k < kFeTaps; ++k) {
            const short pair = *(const short *)(x + k * kFeP + 128 * n1);
            re = fmaf(hc[k][n1].x, (float)(int8_t)(pair & 0xFF), re);
            im = fmaf(hc[k][n1].y, (float)(int8_t)(pair >> 8), im);
        }
        z[n1] = cf{re, im};
    }
    // pass 1: 16-point DFT over n1 (n = 64 n1 + l), twiddle W1024^{l k1}
    dft16(z);
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) {
        const cf w{kTwPass1.re[lane * 16 + k1], kTwPass1.im[lane * 16 + k1]};
        const cf v = cmul(z[k1], w);
        // A[n2 = lane][k1] at row n2, column k1
        *(float2 *)&buf[2 * (lane * kFeBufStride + k1)] = make_float2(v.r, v.i);
    }
    lds_sync();
    // pass 2: lane = (k1, m2); 16-point DFT over m1 of A[4 m1 + m2][k1], twiddle W64^{m2 j1}
    const int k1 = lane >> 2, m2 = lane & 3;
#pragma unroll
    for (int m1 = 0; m1 < 16; ++m1) {
        const float2 v = *(const float2 *)&buf[2 * ((4 * m1 + m2) * kFeBufStride + k1)];
        z[m1] = cf{v.x, v.y};
    }
    dft16(z);
#pragma unroll
    for (int j1 = 0; j1 < 16; ++j1)
        z[j1] = cmul(z[j1], cf{kTwPass2.re[m2 * 16 + j1], kTwPass2.im[m2 * 16 + j1]});
    lds_sync();
    // exchange: B[k1][m2][j1] at row 4 k1 + m2 (17-float2 rows), column j1
#pragma unroll
    for (int j1 = 0; j1 < 16; ++j1)
        *(float2 *)&buf[2 * ((4 * k1 + m2) * kFeBufStride + j1)] = make_float2(z[j1].r, z[j1].i);
    lds_sync();
    // pass 3: lane = (k1, r); for j1 = r + 4 u: 4-point DFT over m2 -> Z[k1 + 16 j1 + 256 j2]
    const int r = lane & 3;
    cf Z[16];   // Z[u][j2] at 4 u + j2
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int j1 = r + 4 * u;
        cf b[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float2 v = *(const float2 *)&buf[2 * ((4 * k1 + q) * kFeBufStride + j1)];
            b[q] = cf{v.x, v.y};
        }
        dft4(b[0], b[1], b[2], b[3]);
#pragma unroll
        for (int j2 = 0; j2 < 4; ++j2)
            Z[4 * u + j2] = b[j2];
    }
    lds_sync();
    // Z in natural order k = k1 + 16 (r + 4 u) + 256 j2, stored at k + k / 16 (pad)
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int j2 = 0; j2 < 4; ++j2) {
            const int k = k1 + 16 * (r + 4 * u) + 256 * j2;
            *(float2 *)&buf[2 * (k + (k >> 4))] = make_float2(Z[4 * u + j2].r, Z[4 * u + j2].i);
        }
    lds_sync();
    // real spectrum of channels c = lane + 64 v
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int c = lane + 64 * v;
        const int cn = (kFeN - c) & (kFeN - 1);
        const float2 p = *(const float2 *)&buf[2 * (c + (c >> 4))];
        const float2 q = *(const float2 *)&buf[2 * (cn + (cn >> 4))];
        const cf zc{p.x, p.y}, zn{q.x, -q.y};   // Z[c], conj Z[N - c]
        const cf e = cadd(zc, zn), d = csub(zc, zn);
        const cf w{kTwReal.re[c], kTwReal.im[c]};
        const cf od = cmul(w, d);                // W^c (Z[c] - Z*[N - c])
        // Y = e / 2 - i od / 2
        y[v] = cf{0.5f * (e.r + od.i), 0.5f * (e.i - od.r)};
    }
    lds_sync();
}

template <bool CODES>
__device__ __forceinline__ void fengine_body(uint8_t *smem, const FeArgs &a)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // work-group -> (spectrum, input group); spectra of one group are spread
    // over the 8 XCDs in contiguous runs, so that the tap overlap between
    // consecutive spectra hits the same L2
    const int64_t groups = (a.N + kFeGroup - 1) / kFeGroup;
    const int64_t per_xcd = (a.n_spectra * groups + 7) / 8;
    const int64_t item = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (item >= a.n_spectra * groups)
        return;
    const int64_t g = item / a.n_spectra, m = item % a.n_spectra;
    const int i0 = (int)g * kFeGroup;

    float *buf = (float *)smem + w * kFeBufFloats;
    uint8_t *codes = smem + kFeWaves * kFeBufFloats * sizeof(float);

    float2 hc[kFeTaps][16];
#pragma unroll
    for (int k = 0; k < kFeTaps; ++k)
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1)
            hc[k][n1] = *(const float2 *)(a.h + k * kFeP + 128 * n1 + 2 * lane);

    for (int ii = 0; ii < kFeInputsPerWave; ++ii) {
        const int input = i0 + w * kFeInputsPerWave + ii;
        if (input >= a.N)
            break;
        cf y[16];
        fe_transform(a, input, m, hc, buf, y);
        if constexpr (CODES) {
            const float *gi = a.gains + (int64_t)input * kFeN;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int c = lane + 64 * v;
                const float gv = gi[c];
                const int re = quant4(gv * y[v].r), im = quant4(gv * y[v].i);
                codes[c * kFeCodeStride + w * kFeInputsPerWave + ii] = (uint8_t)(((re & 15) << 4) | (im & 15));
            }
        } else {
            float2 *o = (float2 *)a.out + ((int64_t)input * a.n_spectra + m) * kFeN;
#pragma unroll
            for (int v = 0; v < 16; ++v)
                o[lane + 64 * v] = make_float2(y[v].r, y[v].i);
        }
    }
    if constexpr (CODES) {
        __syncthreads();
        // rows of 64 codes (16 bytes per thread) to out[m][c][i0 ..]
        uint8_t *o = (uint8_t *)a.out + (m * kFeN) * (int64_t)a.N + i0;
        for (int t = threadIdx.x; t < kFeN * 4; t += kFeThreads) {
            const int c = t >> 2, q = t & 3;
            if (i0 + 16 * q < a.N)
                *(uint4 *)(o + (int64_t)c * a.N + 16 * q) = *(const uint4 *)(codes + c * kFeCodeStride + 16 * q);
        }
    }
}

constexpr int kFeSmemCodes = kFeWaves * kFeBufFloats * 4 + kFeN * kFeCodeStride;
constexpr int kFeSmemSpectra = kFeWaves * kFeBufFloats * 4;

__global__ __launch_bounds__(kFeThreads) void xc_fengine_kernel(const FeArgs a)
{
    __shared__ __attribute__((aligned(16))) uint8_t smem[kFeSmemCodes];
    fengine_body<true>(smem, a);
}

__global__ __launch_bounds__(kFeThreads) void xc_pfb_spectra_kernel(const FeArgs a)
{
    __shared__ __attribute__((aligned(16))) uint8_t smem[kFeSmemSpectra];
    fengine_body<false>(smem, a);
}

int fe_check(const void *adc, int64_t S, int32_t N, const float *h, int64_t n_spectra, const void *out)
{
    if (!adc || !h || !out || N < 1 || N % 16 || S < (int64_t)kFeTaps * kFeP || S % 16 ||
        (uintptr_t)adc % 16 || (uintptr_t)h % 16 || (uintptr_t)out % 16 || n_spectra < 1 ||
        n_spectra > S / kFeP - kFeTaps + 1)
        return XCORR_E_INVAL;
    return XCORR_OK;
}

}  // namespace
}  // namespace xc

extern "C" int xcorr_pfb_prototype(int32_t n_points, int32_t taps, float *h_out)
{
    if (n_points < 2 || taps < 1 || !h_out)
        return XCORR_E_INVAL;
    const int64_t L = (int64_t)n_points * taps;
    const double pi = 3.14159265358979323846;
    for (int64_t n = 0; n < L; ++n) {
        const double w = 0.54 - 0.46 * std::cos(2.0 * pi * (double)n / (double)(L - 1));
        const double t = (double)n / n_points - taps / 2.0;
        const double s = t == 0.0 ? 1.0 : std::sin(pi * t) / (pi * t);
        h_out[n] = (float)(w * s);
    }
    return XCORR_OK;
}

extern "C" int xcorr_fengine(const void *d_adc, int64_t n_samples, int32_t n_inputs, const float *d_coeffs,
                             const float *d_gains, int64_t n_spectra, void *d_out, void *stream)
{
    using namespace xc;
    int rc = fe_check(d_adc, n_samples, n_inputs, d_coeffs, n_spectra, d_out);
    if (rc)
        return rc;
    if (!d_gains || (uintptr_t)d_gains % 16)
        return XCORR_E_INVAL;
    const int64_t items = n_spectra * ((n_inputs + kFeGroup - 1) / kFeGroup);
    if (items > (int64_t)1 << 30)
        return XCORR_E_INVAL;
    FeArgs a{(const int8_t *)d_adc, n_samples, n_inputs, d_coeffs, d_gains, n_spectra, d_out};
    const int grid = (int)(8 * ((items + 7) / 8));
    hipLaunchKernelGGL(xc_fengine_kernel, dim3(grid), dim3(kFeThreads), 0, reinterpret_cast<hipStream_t>(stream), a);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? XCORR_OK : api_error(XCORR_E_HIP, std::string("fengine launch: ") + hipGetErrorString(e));
}

extern "C" int xcorr_pfb_spectra(const void *d_adc, int64_t n_samples, int32_t n_inputs, const float *d_coeffs,
                                 int64_t n_spectra, void *d_out, void *stream)
{
    using namespace xc;
    int rc = fe_check(d_adc, n_samples, n_inputs, d_coeffs, n_spectra, d_out);
    if (rc)
        return rc;
    const int64_t items = n_spectra * ((n_inputs + kFeGroup - 1) / kFeGroup);
    if (items > (int64_t)1 << 30)
        return XCORR_E_INVAL;
    FeArgs a{(const int8_t *)d_adc, n_samples, n_inputs, d_coeffs, nullptr, n_spectra, d_out};
    const int grid = (int)(8 * ((items + 7) / 8));
    hipLaunchKernelGGL(xc_pfb_spectra_kernel, dim3(grid), dim3(kFeThreads), 0, reinterpret_cast<hipStream_t>(stream),
                       a);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? XCORR_OK : api_error(XCORR_E_HIP, std::string("pfb launch: ") + hipGetErrorString(e));
}
