// 4+4-bit int8-MFMA kernels of the X-engine, every diagonal block size D in
// one translation unit (the register allocation of the D = 6 kernel, which
// sits at the 256-register budget, has been seen to spill when its
// instantiation is compiled alone).
#include "xc_mfma4.h"

namespace xc {
namespace {

// One work-group per (channel, region).  Regions of one channel: nseg
// triangles on the diagonal segments, then the nseg(nseg-1)/2 rectangles
// (a, b), a > b, in row-major order.  Segments are D blocks each (the input
// count is zero-padded up to 32*D*nseg).
template <int D, int KC, int VEC>
__global__ __launch_bounds__(kMfmaThreads)
__attribute__((amdgpu_waves_per_eu(2 * mfma4_wgs_per_cu(D), 2 * mfma4_wgs_per_cu(D))))
void xc_mfma4_kernel(const uint8_t *__restrict__ volts, int64_t T, int F, int N, int nseg, int R,
                     int nitems, int2 *__restrict__ acc_out, int accumulate)
{
    constexpr int NBUF = mfma4_nbuf(D, KC);
    __shared__ __attribute__((aligned(1024))) uint8_t smem[mfma4_smem_bytes(D, KC)];

    const int item = xcd_item();
    if (item >= nitems)
        return;
    const int f = item / R;
    const int r = item - f * R;
    if (r < nseg) {
        mfma4_dispatch<D, true, KC, NBUF, VEC>(smem, volts, T, F, N, f, r * D, r * D, acc_out, accumulate);
    } else if constexpr (D <= 4) {
        const int k = r - nseg;
        int a = (int)((1.f + sqrtf(1.f + 8.f * k)) * 0.5f);
        while (a * (a - 1) / 2 > k)
            --a;
        while ((a + 1) * a / 2 <= k)
            ++a;
        const int b = k - a * (a - 1) / 2;
        mfma4_dispatch<D, false, KC, NBUF, VEC>(smem, volts, T, F, N, f, a * D, b * D, acc_out,
                                                accumulate);
    }
}

}  // namespace

template <int D, int KC>
static hipError_t launch_mfma4_t(const Plan &pl, const uint8_t *volts, int64_t T, int F, int N,
                                 int2 *acc, int accumulate, hipStream_t s)
{
    const int64_t nitems64 = (int64_t)F * pl.regions;
    if (nitems64 > (1LL << 30))
        return hipErrorInvalidValue;
    const int nitems = (int)nitems64;
    // the LDS-DMA path addresses one chunk of KC time rows with 32-bit offsets
    const int vec_ok = (N % 16 == 0) && ((uintptr_t)volts % 16 == 0) &&
                       (int64_t)KC * F * N < (1LL << 31) - 16;
    auto kern = vec_ok ? xc_mfma4_kernel<D, KC, 1> : xc_mfma4_kernel<D, KC, 0>;
    hipLaunchKernelGGL(kern, dim3(xcd_grid(nitems)), dim3(kMfmaThreads), 0, s, volts, T, F, N,
                       pl.nseg, pl.regions, nitems, acc, accumulate);
    return hipGetLastError();
}

hipError_t launch_mfma4(const Plan &pl, int kc, const uint8_t *volts, int64_t T, int F, int N,
                        int2 *acc, int accumulate, hipStream_t s)
{
    if ((kc != 64 && kc != 128) || !plan_supported(N, pl.D) || (kc == 128 && pl.D < 4))
        return hipErrorInvalidValue;
    if (kc == 128) {
        switch (pl.D) {
        case 4: return launch_mfma4_t<4, 128>(pl, volts, T, F, N, acc, accumulate, s);
        case 5: return launch_mfma4_t<5, 128>(pl, volts, T, F, N, acc, accumulate, s);
        case 6: return launch_mfma4_t<6, 128>(pl, volts, T, F, N, acc, accumulate, s);
        default: return hipErrorInvalidValue;
        }
    }
    switch (pl.D) {
    case 1: return launch_mfma4_t<1, 64>(pl, volts, T, F, N, acc, accumulate, s);
    case 2: return launch_mfma4_t<2, 64>(pl, volts, T, F, N, acc, accumulate, s);
    case 3: return launch_mfma4_t<3, 64>(pl, volts, T, F, N, acc, accumulate, s);
    case 4: return launch_mfma4_t<4, 64>(pl, volts, T, F, N, acc, accumulate, s);
    case 5: return launch_mfma4_t<5, 64>(pl, volts, T, F, N, acc, accumulate, s);
    case 6: return launch_mfma4_t<6, 64>(pl, volts, T, F, N, acc, accumulate, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace xc
