// gfx950 kernels of the X-engine cross-multiply-accumulate.
//
// For every channel f and pair j <= i:  V_ij = sum_t x_i[t] * conj(x_j[t])
// (paper Section 2.3 "X-engine"; Eq. 2 of Section 3.2), i.e. per channel the
// lower triangle of the Hermitian rank-T update X X^H, accumulated in int32.
//
//   xc_plain_kernel   VALU int32 multiply-adds (the comparison path)
//   (MFMA kernels: xcorr_mfma.hip, one object per diagonal block size)
//   xc_dump_kernel    accumulator -> caller buffer copy (or zero fill)
#include "xc_device.h"

namespace xc {
namespace {

// ---------------------------------------------------------------------------
// Plain path: one work-group per (channel, 64x64 pair tile of the lower
// triangle).  Thread (tx, ty) owns inputs i = 4ty..4ty+3 and j = 4tx..4tx+3 of
// the tile: 16 pairs, re and im in int32 registers.  Time is staged through
// LDS in chunks of 32 samples as raw packed bytes.
template <int BITS, int VEC>
__global__ __launch_bounds__(kThreads) void xc_plain_kernel(
    const uint8_t *__restrict__ volts, int64_t T, int F, int N, int ntiles, int nitems,
    int2 *__restrict__ acc, int accumulate)
{
    constexpr int BPS = BITS == 4 ? 1 : 2;
    constexpr int KC = 32;
    constexpr int SEG = 64 * BPS;               // bytes of 64 inputs in one time row
    constexpr int PIECES = 2 * KC * SEG / 16;   // 16-byte pieces per chunk (rows + cols)
    __shared__ __attribute__((aligned(16))) uint8_t sm[2][KC][SEG];

    const int item = xcd_item();
    if (item >= nitems)
        return;
    const int f = item / ntiles;
    const int tile = item - f * ntiles;
    int I = (int)((sqrtf(8.f * tile + 1.f) - 1.f) * 0.5f);
    while ((I + 1) * (I + 2) / 2 <= tile)
        ++I;
    while (I * (I + 1) / 2 > tile)
        --I;
    const int J = tile - I * (I + 1) / 2;

    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    int ar[4][4], ai[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
            ar[a][b] = ai[a][b] = 0;

    for (int64_t t0 = 0; t0 < T; t0 += KC) {
#pragma unroll
        for (int k = 0; k < PIECES / kThreads; ++k) {
            const int pc = tid + kThreads * k;
            const int seg = pc / (KC * SEG / 16);
            const int rem = pc - seg * (KC * SEG / 16);
            const int t = rem / (SEG / 16);
            const int p = rem - t * (SEG / 16);
            const int i0 = (seg ? J : I) * 64 + p * 16 / BPS;
            *reinterpret_cast<v4i *>(&sm[seg][t][p * 16]) =
                load_piece(volts, t0 + t, T, f, F, N, i0, BPS, VEC);
        }
        __syncthreads();
#pragma unroll 4
        for (int t = 0; t < KC; ++t) {
            int xr[4], xi[4], yr[4], yi[4];
            if constexpr (BITS == 4) {
                const uint32_t a = *reinterpret_cast<const uint32_t *>(&sm[0][t][ty * 4]);
                const uint32_t b = *reinterpret_cast<const uint32_t *>(&sm[1][t][tx * 4]);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    xr[k] = sext_nibble(a, 8 * k + 4);
                    xi[k] = sext_nibble(a, 8 * k);
                    yr[k] = sext_nibble(b, 8 * k + 4);
                    yi[k] = sext_nibble(b, 8 * k);
                }
            } else {
                const int8_t *a = reinterpret_cast<const int8_t *>(&sm[0][t][ty * 8]);
                const int8_t *b = reinterpret_cast<const int8_t *>(&sm[1][t][tx * 8]);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    xr[k] = a[2 * k];
                    xi[k] = a[2 * k + 1];
                    yr[k] = b[2 * k];
                    yi[k] = b[2 * k + 1];
                }
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    ar[a][b] += xr[a] * yr[b] + xi[a] * yi[b];
                    ai[a][b] += xi[a] * yr[b] - xr[a] * yi[b];
                }
        }
        __syncthreads();
    }

    const int64_t P = (int64_t)N * (N + 1) / 2;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int i = I * 64 + ty * 4 + a;
        if (i >= N)
            continue;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int j = J * 64 + tx * 4 + b;
            if (j > i)
                continue;
            int2 *dst = acc + (int64_t)f * P + (int64_t)i * (i + 1) / 2 + j;
            int re = ar[a][b], im = ai[a][b];
            if (accumulate) {
                const int2 o = *dst;
                re += o.x;
                im += o.y;
            }
            *dst = make_int2(re, im);
        }
    }
}

// ---------------------------------------------------------------------------
// Dump: copy the accumulators to the caller's buffer (16-byte vectors plus an
// 8-byte tail), or fill it with zeros for an empty integration.
__global__ __launch_bounds__(kThreads) void xc_dump_kernel(const int2 *__restrict__ src,
                                                           int2 *__restrict__ dst, int64_t n8,
                                                           int empty)
{
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    const int64_t n16 = n8 >> 1;
    const v4i *s16 = reinterpret_cast<const v4i *>(src);
    v4i *d16 = reinterpret_cast<v4i *>(dst);
    for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n16; k += stride)
        d16[k] = empty ? v4i{0, 0, 0, 0} : s16[k];
    if ((n8 & 1) && blockIdx.x == 0 && threadIdx.x == 0)
        dst[n8 - 1] = empty ? make_int2(0, 0) : src[n8 - 1];
}

}  // namespace

Plan make_plan(int N, int D)
{
    Plan p;
    p.D = D;
    p.NB = (N + 31) / 32;
    p.nseg = (p.NB + D - 1) / D;
    p.regions = p.nseg + p.nseg * (p.nseg - 1) / 2;
    return p;
}

bool plan_supported(int N, int D)
{
    const int nb = (N + 31) / 32;
    if (D < 1 || D > 6)
        return false;
    // D <= 4 kernels also have rectangular regions; D = 5, 6 are one triangle
    return D <= 4 ? (D > 1 || nb == 1) : nb <= D;
}

hipError_t launch_plain(int bits, const uint8_t *volts, int64_t T, int F, int N, int2 *acc,
                        int accumulate, hipStream_t s)
{
    const int nb = (N + 63) / 64;
    const int ntiles = nb * (nb + 1) / 2;
    const int64_t nitems64 = (int64_t)F * ntiles;
    if (nitems64 > (1LL << 30))
        return hipErrorInvalidValue;
    const int nitems = (int)nitems64;
    const int bps = bits == 4 ? 1 : 2;
    const int vec_ok = ((int64_t)N * bps % 16 == 0) && ((uintptr_t)volts % 16 == 0);
    dim3 grid(xcd_grid(nitems)), block(kThreads);
    auto kern = bits == 4 ? (vec_ok ? xc_plain_kernel<4, 1> : xc_plain_kernel<4, 0>)
                          : (vec_ok ? xc_plain_kernel<8, 1> : xc_plain_kernel<8, 0>);
    hipLaunchKernelGGL(kern, grid, block, 0, s, volts, T, F, N, ntiles, nitems, acc, accumulate);
    return hipGetLastError();
}

hipError_t launch_mfma8(const Plan &pl, bool f16, const uint8_t *volts, int64_t T, int F, int N, void *acc,
                        int accumulate, hipStream_t s)
{
    if (!plan_supported(N, pl.D))
        return hipErrorInvalidValue;
    switch (pl.D) {
    case 1: return launch_mfma8_d1(pl, f16, volts, T, F, N, acc, accumulate, s);
    case 2: return launch_mfma8_d2(pl, f16, volts, T, F, N, acc, accumulate, s);
    case 3: return launch_mfma8_d3(pl, f16, volts, T, F, N, acc, accumulate, s);
    case 4: return launch_mfma8_d4(pl, f16, volts, T, F, N, acc, accumulate, s);
    case 5: return launch_mfma8_d5(pl, f16, volts, T, F, N, acc, accumulate, s);
    case 6: return launch_mfma8_d6(pl, f16, volts, T, F, N, acc, accumulate, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dump(const void *acc, void *out, int64_t bytes, int empty, hipStream_t s)
{
    if (bytes % 8 || (uintptr_t)acc % 16 || (uintptr_t)out % 16)
        return hipErrorInvalidValue;
    const int64_t n8 = bytes / 8;
    const int64_t work = std::max<int64_t>(1, (n8 / 2 + kThreads - 1) / kThreads);
    const int blocks = (int)std::min<int64_t>(work, 8192);
    hipLaunchKernelGGL(xc_dump_kernel, dim3(blocks), dim3(kThreads), 0, s,
                       reinterpret_cast<const int2 *>(acc), reinterpret_cast<int2 *>(out), n8, empty);
    return hipGetLastError();
}

}  // namespace xc
