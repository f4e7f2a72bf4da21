// 4+4-bit int8-MFMA kernels of the X-engine, fused-product variant (one Re
// and one Im accumulator per tile; waves = product x K parity x tile half),
// every diagonal block size D in one translation unit.
#include "xc_mfma4.h"

namespace xc {
namespace {

// One work-group per (channel, region), regions as in the per-role kernel.
// Two work-groups per CU for D <= 2 (128 registers per wave), one above: at
// D = 3 the 128-register budget spills.
constexpr int fused_wgs_per_cu(int D) { return D <= 2 ? 2 : 1; }

template <int D, int VEC, int ACC>
__global__ __launch_bounds__(kMfmaThreads)
__attribute__((amdgpu_waves_per_eu(2 * fused_wgs_per_cu(D), 2 * fused_wgs_per_cu(D))))
void xc_mfma4f_kernel(const uint8_t *__restrict__ volts, int64_t T, int F, int N, int nseg, int R,
                      int nitems, int2 *acc_out, const int2 *acc_in, int accumulate)
{
    constexpr int KC = 64;
    constexpr int NBUF = fused_nbuf(D);
    __shared__ __attribute__((aligned(1024))) uint8_t smem[fused_smem_bytes(D)];

    const int item = xcd_item();
    if (item >= nitems)
        return;
    const int f = item / R;
    const int r = item - f * R;
    if (r < nseg) {
        mfma4f_dispatch<D, true, KC, NBUF, VEC, 0, ACC>(smem, volts, T, F, N, f, r * D, r * D, acc_out, acc_in,
                                                        accumulate);
    } else if constexpr (D <= 4) {
        const int k = r - nseg;
        int a = (int)((1.f + sqrtf(1.f + 8.f * k)) * 0.5f);
        while (a * (a - 1) / 2 > k)
            --a;
        while ((a + 1) * a / 2 <= k)
            ++a;
        const int b = k - a * (a - 1) / 2;
        mfma4f_dispatch<D, false, KC, NBUF, VEC, 0, ACC>(smem, volts, T, F, N, f, a * D, b * D, acc_out,
                                                         acc_in, accumulate);
    }
}

// Several blocks of one array in one launch (16-byte-aligned blocks, N a
// multiple of 16): as above, with the chunks taken from the block table.
template <int D, int ACC>
__global__ __launch_bounds__(kMfmaThreads)
__attribute__((amdgpu_waves_per_eu(2 * fused_wgs_per_cu(D), 2 * fused_wgs_per_cu(D))))
void xc_mfma4f_blocks_kernel(const BlockTable bt, int64_t T, int F, int N, int nseg, int R, int nitems,
                             int2 *acc_out, const int2 *acc_in, int accumulate)
{
    constexpr int KC = 64;
    constexpr int NBUF = fused_nbuf(D);
    __shared__ __attribute__((aligned(1024))) uint8_t smem[fused_smem_bytes(D)];

    const int item = xcd_item();
    if (item >= nitems)
        return;
    const int f = item / R;
    const int r = item - f * R;
    if (r < nseg) {
        mfma4f_dispatch<D, true, KC, NBUF, 1, 1, ACC>(smem, nullptr, T, F, N, f, r * D, r * D, acc_out, acc_in,
                                                      accumulate, &bt);
    } else if constexpr (D <= 4) {
        const int k = r - nseg;
        int a = (int)((1.f + sqrtf(1.f + 8.f * k)) * 0.5f);
        while (a * (a - 1) / 2 > k)
            --a;
        while ((a + 1) * a / 2 <= k)
            ++a;
        const int b = k - a * (a - 1) / 2;
        mfma4f_dispatch<D, false, KC, NBUF, 1, 1, ACC>(smem, nullptr, T, F, N, f, a * D, b * D, acc_out,
                                                       acc_in, accumulate, &bt);
    }
}

}  // namespace

template <int D>
static hipError_t launch_mfma4f_blocks_t(const Plan &pl, const BlockTable &bt, int n_blocks, int F, int N,
                                         int2 *acc, const int2 *acc_in, int accumulate, hipStream_t s)
{
    const int64_t nitems64 = (int64_t)F * pl.regions;
    if (nitems64 > (1LL << 30))
        return hipErrorInvalidValue;
    const int nitems = (int)nitems64;
    const int64_t T = (int64_t)n_blocks * bt.chunks_per_block * 64;
    auto kern = accumulate ? xc_mfma4f_blocks_kernel<D, 1> : xc_mfma4f_blocks_kernel<D, 0>;
    hipLaunchKernelGGL(kern, dim3(xcd_grid(nitems)), dim3(kMfmaThreads), 0, s, bt, T, F, N, pl.nseg, pl.regions,
                       nitems, acc, acc_in ? acc_in : acc, accumulate);
    return hipGetLastError();
}

hipError_t launch_mfma4f_blocks(const Plan &pl, const BlockTable &bt, int n_blocks, int F, int N, int2 *acc,
                                int accumulate, hipStream_t s, const int2 *acc_in)
{
    if (!plan_supported(N, pl.D) || n_blocks < 1 || n_blocks > kMaxFusedBlocks || bt.chunks_per_block < 1 ||
        (int64_t)n_blocks * bt.chunks_per_block * 64 > kMaxSamplesPerLaunch4 || N % 16 ||
        64LL * F * N >= (1LL << 31) - 16)
        return hipErrorInvalidValue;
    for (int b = 0; b < n_blocks; ++b)
        if (!bt.p[b] || (uintptr_t)bt.p[b] % 16)
            return hipErrorInvalidValue;
    switch (pl.D) {
    case 1: return launch_mfma4f_blocks_t<1>(pl, bt, n_blocks, F, N, acc, acc_in, accumulate, s);
    case 2: return launch_mfma4f_blocks_t<2>(pl, bt, n_blocks, F, N, acc, acc_in, accumulate, s);
    case 3: return launch_mfma4f_blocks_t<3>(pl, bt, n_blocks, F, N, acc, acc_in, accumulate, s);
    case 4: return launch_mfma4f_blocks_t<4>(pl, bt, n_blocks, F, N, acc, acc_in, accumulate, s);
    case 5: return launch_mfma4f_blocks_t<5>(pl, bt, n_blocks, F, N, acc, acc_in, accumulate, s);
    case 6: return launch_mfma4f_blocks_t<6>(pl, bt, n_blocks, F, N, acc, acc_in, accumulate, s);
    default: return hipErrorInvalidValue;
    }
}

template <int D>
static hipError_t launch_mfma4f_t(const Plan &pl, const uint8_t *volts, int64_t T, int F, int N,
                                  int2 *acc, const int2 *acc_in, int accumulate, hipStream_t s)
{
    const int64_t nitems64 = (int64_t)F * pl.regions;
    if (nitems64 > (1LL << 30))
        return hipErrorInvalidValue;
    const int nitems = (int)nitems64;
    const int vec_ok = (N % 16 == 0) && ((uintptr_t)volts % 16 == 0) &&
                       64LL * F * N < (1LL << 31) - 16;
    // overwrite and accumulate are separate kernels: the batched loads of the
    // accumulating epilogue cost the overwriting one registers and time
    auto kern = vec_ok ? (accumulate ? xc_mfma4f_kernel<D, 1, 1> : xc_mfma4f_kernel<D, 1, 0>)
                       : (accumulate ? xc_mfma4f_kernel<D, 0, 1> : xc_mfma4f_kernel<D, 0, 0>);
    hipLaunchKernelGGL(kern, dim3(xcd_grid(nitems)), dim3(kMfmaThreads), 0, s, volts, T, F, N,
                       pl.nseg, pl.regions, nitems, acc, acc_in ? acc_in : acc, accumulate);
    return hipGetLastError();
}

hipError_t launch_mfma4f(const Plan &pl, const uint8_t *volts, int64_t T, int F, int N, int2 *acc,
                         int accumulate, hipStream_t s, const int2 *acc_in)
{
    if (!plan_supported(N, pl.D) || T > kMaxSamplesPerLaunch4)
        return hipErrorInvalidValue;
    switch (pl.D) {
    case 1: return launch_mfma4f_t<1>(pl, volts, T, F, N, acc, acc_in, accumulate, s);
    case 2: return launch_mfma4f_t<2>(pl, volts, T, F, N, acc, acc_in, accumulate, s);
    case 3: return launch_mfma4f_t<3>(pl, volts, T, F, N, acc, acc_in, accumulate, s);
    case 4: return launch_mfma4f_t<4>(pl, volts, T, F, N, acc, acc_in, accumulate, s);
    case 5: return launch_mfma4f_t<5>(pl, volts, T, F, N, acc, acc_in, accumulate, s);
    case 6: return launch_mfma4f_t<6>(pl, volts, T, F, N, acc, acc_in, accumulate, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace xc
