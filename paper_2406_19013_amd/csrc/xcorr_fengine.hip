// F-engine front end (paper Section 2.2): 8-bit ADC samples of each input ->
// polyphase filter bank of 2048 points with a 4-tap prototype -> real FFT ->
// 1024 channels -> per-(input, channel) EQ gain -> 4+4-bit requantisation ->
// corner turn into the X-engine's [T][F][N] order.
//
// Persistent work-groups of 8 waves (two per SIMD); an item is one spectrum
// m of 16 inputs, 2 per wave, each filtered and transformed by one wave.  Per
// input and spectrum:
//   y[q] = sum_k h[k P + q] x[(m + k) P + q]            q < P = 2048
//   z[n] = y[2n] + i y[2n + 1]                          n < 1024
//   Z    = 1024-point complex DFT of z (radix 16 x 16 x 4)
//   Y[c] = (Z[c] + Z*[N - c]) / 2 - i W^c (Z[c] - Z*[N - c]) / 2,  W = e^{-2 pi i / 2048}
//   code = pack(clip(rint(g Re Y)), clip(rint(g Im Y)))  for channels c < 1024
// A lane reads 32 consecutive samples of each tap with 16-byte loads (one
// input ahead of the one it transforms); the prototype is copied into LDS
// once per work-group, ordered so that the 128 coefficients of a lane's sample
// positions come as 32 conflict-free 16-byte reads per transform (held in
// registers they took 512 per lane and left room for one wave per SIMD);
// four LDS exchanges per transform (into the stride-64 order, between
// the three radix passes, and for the Z[N - c] pairs).  Twiddles are built
// per lane from one base value by short power products (at most three
// roundings deep).  The 16 inputs' codes are gathered in LDS and leave as one
// 16-byte row per (spectrum, channel).  Arithmetic in fp32; rounding is
// round-half-to-even.
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
constexpr int kFeGroup = 16;        // inputs per item
constexpr int kFeWaves = 8;
constexpr int kFeThreads = 64 * kFeWaves;
constexpr int kFeInputsPerWave = kFeGroup / kFeWaves;
constexpr int kFeWgsPerCu = 1;   // 8 waves: two per SIMD, up to 256 registers each
constexpr int kFeBufStride = 17;                    // float2 per row of the pass exchanges (16 + 1 pad)
constexpr int kFeBufFloats = 2 * 64 * kFeBufStride;  // per wave: 64 rows
constexpr int kFeCodeStride = 20;                   // bytes per channel row of the code tile (16 + pad)
constexpr int kFeSmemProto = kFeTaps * kFeP * 4;    // the prototype, 32 KB

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
// W_den^e = exp(-2 pi i e / den) for e < COUNT
template <int COUNT>
constexpr Table<COUNT> make_powers(long den)
{
    Table<COUNT> t{};
    for (int e = 0; e < COUNT; ++e) {
        const SinCos v = sincos_turn(e, den);
        t.re[e] = (float)v.c;
        t.im[e] = (float)-v.s;
    }
    return t;
}
__device__ constexpr Table<64> kW1024 = make_powers<64>(1024);   // pass-1 bases W1024^l
__device__ constexpr Table<4> kW64 = make_powers<4>(64);         // pass-2 bases W64^m2
__device__ constexpr Table<64> kW2048 = make_powers<64>(2048);   // real-unpack bases W2048^l
constexpr Table<16> kW32 = make_powers<16>(32);                  // W2048^(64 v) = W32^v

// ---- complex helpers ----------------------------------------------------------

struct cf {
    float r, i;
};
__device__ __forceinline__ cf cadd(cf a, cf b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cf csub(cf a, cf b) { return {a.r - b.r, a.i - b.i}; }
__device__ __forceinline__ cf cmul(cf a, cf b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cf cmul_mi(cf a) { return {a.i, -a.r}; }   // a * (-i)

// p[k] = w^k for k < 16: w, w^2, w^3 and w^4, w^8, w^12, then products
// (each power at most three roundings from w)
__device__ __forceinline__ void powers16(cf w, cf (&p)[16])
{
    p[0] = cf{1.f, 0.f};
    p[1] = w;
    p[2] = cmul(w, w);
    p[3] = cmul(p[2], w);
    p[4] = cmul(p[2], p[2]);
    p[8] = cmul(p[4], p[4]);
    p[12] = cmul(p[8], p[4]);
#pragma unroll
    for (int a = 4; a < 16; a += 4)
#pragma unroll
        for (int b = 1; b < 4; ++b)
            p[a + b] = cmul(p[a], p[b]);
}

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

// Raw samples of one (input, spectrum) for this lane: 32 consecutive
// samples x[(m + k) P + 32 lane + t] of each tap k, as two 16-byte loads.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
struct FeRaw {
    u32x4 v[kFeTaps][2];
};
__device__ __forceinline__ void fe_load(const FeArgs &a, int input, int64_t m, FeRaw &r)
{
    const int lane = threadIdx.x & 63;
    const u32x4 *x = (const u32x4 *)(a.adc + (int64_t)input * a.S + m * kFeP + 32 * lane);
#pragma unroll
    for (int k = 0; k < kFeTaps; ++k) {
        r.v[k][0] = __builtin_nontemporal_load(x + k * (kFeP / 16));
        r.v[k][1] = __builtin_nontemporal_load(x + k * (kFeP / 16) + 1);
    }
}

__device__ __forceinline__ float byte_at(const u32x4 &v, int t)
{
    const uint32_t w = t < 4 ? v.x : t < 8 ? v.y : t < 12 ? v.z : v.w;
    return (float)(int8_t)(w >> (8 * (t & 3)));
}

// One wave's transform of one (input, spectrum), in two parts: the FIR of
// its raw samples (after which the raw registers take the next input's
// loads), then the FFT, which returns the 16 channel values c = lane + 64 v
// (v < 16) of the real spectrum in y[v].
// hl: the prototype in LDS, float4 (k, t4, lane) = h[k P + 32 lane + 4 t4 ..].
struct FeBases {
    cf w1024, w64, w2048;   // W1024^lane, W64^(lane % 4), W2048^lane
};
__device__ __forceinline__ void fe_fir(const FeRaw &raw, const float4 *hl, cf (&z)[16])
{
    const int lane = threadIdx.x & 63;
    // FIR on this lane's 32 samples -> z[n] for n = 16 lane + j; samples
    // 4 t4 .. 4 t4 + 3 make z[2 t4] and z[2 t4 + 1]
#pragma unroll
    for (int t4 = 0; t4 < 8; ++t4) {
        // The coefficient reads are the same for every transform: left alone
        // the compiler hoists or clusters all 32 (128 registers live at
        // once).  An opaque offset behind a memory clobber keeps each group
        // of four between its neighbours.
        int l = lane;
        asm volatile("" : "+v"(l) : : "memory");
        float r0 = 0.f, i0 = 0.f, r1 = 0.f, i1 = 0.f;
#pragma unroll
        for (int k = 0; k < kFeTaps; ++k) {
            const float4 h = hl[(k * 8 + t4) * 64 + l];
            const u32x4 &v = raw.v[k][t4 >> 2];
            const int t = (4 * t4) & 15;
            r0 = fmaf(h.x, byte_at(v, t), r0);
            i0 = fmaf(h.y, byte_at(v, t + 1), i0);
            r1 = fmaf(h.z, byte_at(v, t + 2), r1);
            i1 = fmaf(h.w, byte_at(v, t + 3), i1);
        }
        z[2 * t4] = cf{r0, i0};
        z[2 * t4 + 1] = cf{r1, i1};
    }
}

__device__ __forceinline__ void fe_fft(cf (&z)[16], const FeBases &bs, float *buf, cf (&y)[16])
{
    // the exchange addresses are the same for every transform; an opaque lane
    // makes the compiler form them here instead of keeping about a hundred
    // of them live across the loop (which spilled with two waves per SIMD)
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    // likewise the twiddles derived from the per-lane bases (about a hundred
    // registers if kept across the loop): formed anew for each transform
    FeBases b = bs;
    asm volatile("" : "+v"(b.w1024.r), "+v"(b.w1024.i), "+v"(b.w64.r), "+v"(b.w64.i), "+v"(b.w2048.r),
                 "+v"(b.w2048.i));
    // exchange 0: z at n + n / 16, read back with stride 64 (n = 64 n1 + lane)
#pragma unroll
    for (int j = 0; j < 16; ++j)
        *(float2 *)&buf[2 * (17 * lane + j)] = make_float2(z[j].r, z[j].i);
    lds_sync();
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) {
        const float2 v = *(const float2 *)&buf[2 * (68 * n1 + lane + (lane >> 4))];
        z[n1] = cf{v.x, v.y};
    }
    lds_sync();
    // pass 1: 16-point DFT over n1 (n = 64 n1 + l), twiddle W1024^{l k1}
    dft16(z);
    {
        cf tw[16];
        powers16(b.w1024, tw);
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) {
            const cf v = cmul(z[k1], tw[k1]);
            // A[n2 = lane][k1] at row n2, column k1
            *(float2 *)&buf[2 * (lane * kFeBufStride + k1)] = make_float2(v.r, v.i);
        }
    }
    lds_sync();
    // pass 2: lane = (k1, m2); 16-point DFT over m1 of A[4 m1 + m2][k1], twiddle W64^{m2 j1}
    const int k1 = lane >> 2, m2 = lane & 3;
#pragma unroll
    for (int m1 = 0; m1 < 16; ++m1) {
        const float2 v = *(const float2 *)&buf[2 * ((4 * m1 + m2) * kFeBufStride + k1)];
        z[m1] = cf{v.x, v.y};
    }
    lds_sync();
    dft16(z);
    {
        cf tw[16];
        powers16(b.w64, tw);
#pragma unroll
        for (int j1 = 0; j1 < 16; ++j1)
            z[j1] = cmul(z[j1], tw[j1]);
    }
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
    // Z in natural order k = k1 + 16 (r + 4 u) + 256 j2, stored at k + k / 16
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int j2 = 0; j2 < 4; ++j2) {
            const int k = k1 + 16 * (r + 4 * u) + 256 * j2;
            *(float2 *)&buf[2 * (k + (k >> 4))] = make_float2(Z[4 * u + j2].r, Z[4 * u + j2].i);
        }
    lds_sync();
    // real spectrum of channels c = lane + 64 v: W2048^c = W2048^lane W32^v
    const cf wl = b.w2048;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int c = lane + 64 * v;
        const int cn = (kFeN - c) & (kFeN - 1);
        const float2 p = *(const float2 *)&buf[2 * (c + (c >> 4))];
        const float2 q = *(const float2 *)&buf[2 * (cn + (cn >> 4))];
        const cf zc{p.x, p.y}, zn{q.x, -q.y};   // Z[c], conj Z[N - c]
        const cf e = cadd(zc, zn), d = csub(zc, zn);
        const cf w = v ? cmul(wl, cf{kW32.re[v], kW32.im[v]}) : wl;
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
    // items (spectrum m of input group g) in order m fastest; each XCD takes a
    // contiguous run, so the taps shared by consecutive spectra meet in its L2
    const int64_t groups = a.N / kFeGroup;
    const int64_t items = a.n_spectra * groups;
    const int64_t per_xcd = (items + 7) / 8;
    const int64_t first = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    const int64_t end = min(items, (int64_t)((blockIdx.x & 7) + 1) * per_xcd);
    const int64_t stride = gridDim.x >> 3;
    if (first >= end)
        return;

    float4 *hl = (float4 *)smem;
    float *buf = (float *)(smem + kFeSmemProto) + w * kFeBufFloats;
    uint8_t *codes = smem + kFeSmemProto + kFeWaves * kFeBufFloats * sizeof(float);

    // the prototype into LDS: float4 (k, t4, l) at (k * 8 + t4) * 64 + l
    for (int idx = threadIdx.x; idx < kFeTaps * 8 * 64; idx += kFeThreads) {
        const int k = idx >> 9, t4 = (idx >> 6) & 7, l = idx & 63;
        hl[idx] = *(const float4 *)(a.h + k * kFeP + 32 * l + 4 * t4);
    }
    __syncthreads();

    const FeBases bases{cf{kW1024.re[lane], kW1024.im[lane]}, cf{kW64.re[lane & 3], kW64.im[lane & 3]},
                        cf{kW2048.re[lane], kW2048.im[lane]}};
    // this wave's jobs: (item, ii) for items first, first + stride, ... and
    // ii < 4; the next job's samples are loaded while the current one runs
    auto input_of = [&](int64_t it, int ii) { return (int)(it / a.n_spectra) * kFeGroup + w * kFeInputsPerWave + ii; };
    FeRaw raw;
    fe_load(a, input_of(first, 0), first % a.n_spectra, raw);
    for (int64_t it = first; it < end; it += stride) {
        const int64_t m = it % a.n_spectra;
        const int g = (int)(it / a.n_spectra);
        for (int ii = 0; ii < kFeInputsPerWave; ++ii) {
            const int input = g * kFeGroup + w * kFeInputsPerWave + ii;
            cf z[16];
            fe_fir(raw, hl, z);
            if (ii + 1 < kFeInputsPerWave)
                fe_load(a, input + 1, m, raw);
            else if (it + stride < end)
                fe_load(a, input_of(it + stride, 0), (it + stride) % a.n_spectra, raw);
            // this input's EQ gains, loaded before the transform so that
            // their latency is hidden behind it
            float gv16[16];
            if constexpr (CODES) {
                const float *gi = a.gains + (int64_t)input * kFeN;
#pragma unroll
                for (int v = 0; v < 16; ++v)
                    gv16[v] = gi[lane + 64 * v];
            }
            cf y[16];
            fe_fft(z, bases, buf, y);
            if constexpr (CODES) {
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int c = lane + 64 * v;
                    const float gv = gv16[v];
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
            // one 16-byte row per channel: out[m][c][16 g ..]
            uint8_t *o = (uint8_t *)a.out + (m * kFeN) * (int64_t)a.N + g * kFeGroup;
#pragma unroll
            for (int c = threadIdx.x; c < kFeN; c += kFeThreads) {
                const uint32_t *row = (const uint32_t *)(codes + c * kFeCodeStride);
                *(uint4 *)(o + (int64_t)c * a.N) = make_uint4(row[0], row[1], row[2], row[3]);
            }
            __syncthreads();
        }
    }
}

constexpr int kFeSmemCodes = kFeSmemProto + kFeWaves * kFeBufFloats * 4 + kFeN * kFeCodeStride;
constexpr int kFeSmemSpectra = kFeSmemProto + kFeWaves * kFeBufFloats * 4;

__global__ __launch_bounds__(kFeThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void xc_fengine_kernel(const FeArgs a)
{
    __shared__ __attribute__((aligned(16))) uint8_t smem[kFeSmemCodes];
    fengine_body<true>(smem, a);
}

__global__ __launch_bounds__(kFeThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void xc_pfb_spectra_kernel(const FeArgs a)
{
    __shared__ __attribute__((aligned(16))) uint8_t smem[kFeSmemSpectra];
    fengine_body<false>(smem, a);
}

// persistent grid: kFeWgsPerCu work-groups per compute unit, a multiple of 8
// (one run of items per XCD), no more than there are items per XCD
int fe_grid(int64_t items)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 8)
        cus = 256;
    const int64_t per_xcd = (items + 7) / 8;
    return 8 * (int)std::max<int64_t>(1, std::min<int64_t>(cus / 8 * kFeWgsPerCu, per_xcd));
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
    const int64_t items = n_spectra * (n_inputs / kFeGroup);
    if (items > (int64_t)1 << 30)
        return XCORR_E_INVAL;
    FeArgs a{(const int8_t *)d_adc, n_samples, n_inputs, d_coeffs, d_gains, n_spectra, d_out};
    const int grid = fe_grid(items);
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
    const int64_t items = n_spectra * (n_inputs / kFeGroup);
    if (items > (int64_t)1 << 30)
        return XCORR_E_INVAL;
    FeArgs a{(const int8_t *)d_adc, n_samples, n_inputs, d_coeffs, nullptr, n_spectra, d_out};
    const int grid = fe_grid(items);
    hipLaunchKernelGGL(xc_pfb_spectra_kernel, dim3(grid), dim3(kFeThreads), 0, reinterpret_cast<hipStream_t>(stream),
                       a);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? XCORR_OK : api_error(XCORR_E_HIP, std::string("pfb launch: ") + hipGetErrorString(e));
}
