// 4+4-bit int8-MFMA kernels of the X-engine, three-product variant (see
// xc_gauss4.h): one persistent work-group per CU (two for D <= 3) walks its
// (channel, region) items as one continuous stream of LDS-DMA chunks.  A
// channel of up to 6 blocks is one triangle; more blocks (D <= 4) split into
// triangles of D blocks on the diagonal and D x D rectangles between them,
// run as two launches (all triangles, then all rectangles).  Triangles of 2
// to 4 blocks go two channels to an item (6, 12 or 20 tiles over 4, 6 or 8
// blocks), which spreads each chunk's fixed cost over twice the MFMAs.
//
// The kernels are compiled in one unit per diagonal size D (XC_G3_D = 1 .. 6,
// so that the units build in parallel), each defining gauss4_launch_d<D>; the
// unit without XC_G3_D holds the host entry points.
#include "xc_gauss4.h"

namespace xc {

// every launch for a plan with diagonal size D: the segment triangles, then
// (several segments) the rectangles between them
template <int D>
hipError_t gauss4_launch_d(const uint8_t *volts, int64_t T, int F, int N, int2 *out, const int2 *in, int nseg,
                           const BlockTable *bt, int accumulate, hipStream_t s);

#ifdef XC_G3_D
namespace {

template <int D, int SH, int ACC, int MB>
__global__ __launch_bounds__(kG3Threads)
__attribute__((amdgpu_waves_per_eu(g3_waves_per_eu<SH>(D), g3_waves_per_eu<SH>(D))))
void xc_gauss4_kernel(const G3Args a, const BlockTable bt)
{
    __shared__ __attribute__((aligned(1024))) uint8_t smem[g3_smem_bytes<SH>(D)];
    g3_dispatch<D, SH, ACC, MB>(smem, a, &bt);
}

// compute units of the current device (queried once per device)
int device_cu_count()
{
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 256;
    if (!cached[dev]) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 8)
            cus = 256;
        cached[dev] = cus;
    }
    return cached[dev];
}

template <int D, int SH>
hipError_t launch_shape(const G3Args &a, const BlockTable *bt, int accumulate, hipStream_t s)
{
    const int64_t items = g3_items<SH>(a.F, a.nreg);
    const int per = (int)((items + 7) / 8);
    const int m_max = device_cu_count() * g3_wgs_per_cu<SH>(D) / 8;
    const int grid = 8 * std::max(1, std::min(m_max, per));
    G3Args args = a;
    args.per = per;
    args.mrow0 = 0;
    args.mrows = grid / 8;
    BlockTable table{};
    if (bt)
        table = *bt;
    auto kern = bt ? (accumulate ? xc_gauss4_kernel<D, SH, 1, 1> : xc_gauss4_kernel<D, SH, 0, 1>)
                   : (accumulate ? xc_gauss4_kernel<D, SH, 1, 0> : xc_gauss4_kernel<D, SH, 0, 0>);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kG3Threads), 0, s, args, table);
    return hipGetLastError();
}

}  // namespace

template <>
hipError_t gauss4_launch_d<XC_G3_D>(const uint8_t *volts, int64_t T, int F, int N, int2 *out, const int2 *in,
                                    int nseg, const BlockTable *bt, int accumulate, hipStream_t s)
{
    constexpr int D = XC_G3_D;
    G3Args a{};
    a.volts = volts;
    a.T = T;
    a.F = F;
    a.N = N;
    a.out = out;
    a.in = in;
    G3Args t = a;
    t.nreg = nseg;
    hipError_t e;
    if constexpr (D >= 2 && D <= 4)
        e = a.F >= 2 ? launch_shape<D, kPair>(t, bt, accumulate, s) : launch_shape<D, kTri>(t, bt, accumulate, s);
    else
        e = launch_shape<D, kTri>(t, bt, accumulate, s);
    if constexpr (D <= 4) {
        if (e == hipSuccess && nseg > 1) {
            G3Args r = a;
            r.nreg = nseg * (nseg - 1) / 2;
            e = launch_shape<D, kRect>(r, bt, accumulate, s);
        }
    }
    return e;
}

#else

template <>
hipError_t gauss4_launch_d<1>(const uint8_t *, int64_t, int, int, int2 *, const int2 *, int, const BlockTable *, int,
                              hipStream_t);
template <>
hipError_t gauss4_launch_d<2>(const uint8_t *, int64_t, int, int, int2 *, const int2 *, int, const BlockTable *, int,
                              hipStream_t);
template <>
hipError_t gauss4_launch_d<3>(const uint8_t *, int64_t, int, int, int2 *, const int2 *, int, const BlockTable *, int,
                              hipStream_t);
template <>
hipError_t gauss4_launch_d<4>(const uint8_t *, int64_t, int, int, int2 *, const int2 *, int, const BlockTable *, int,
                              hipStream_t);
template <>
hipError_t gauss4_launch_d<5>(const uint8_t *, int64_t, int, int, int2 *, const int2 *, int, const BlockTable *, int,
                              hipStream_t);
template <>
hipError_t gauss4_launch_d<6>(const uint8_t *, int64_t, int, int, int2 *, const int2 *, int, const BlockTable *, int,
                              hipStream_t);

namespace {

hipError_t launch_any(int D, int nseg, const uint8_t *volts, int64_t T, int F, int N, int2 *out, const int2 *in,
                      const BlockTable *bt, int accumulate, hipStream_t s)
{
    switch (D) {
    case 1: return gauss4_launch_d<1>(volts, T, F, N, out, in, nseg, bt, accumulate, s);
    case 2: return gauss4_launch_d<2>(volts, T, F, N, out, in, nseg, bt, accumulate, s);
    case 3: return gauss4_launch_d<3>(volts, T, F, N, out, in, nseg, bt, accumulate, s);
    case 4: return gauss4_launch_d<4>(volts, T, F, N, out, in, nseg, bt, accumulate, s);
    case 5: return gauss4_launch_d<5>(volts, T, F, N, out, in, nseg, bt, accumulate, s);
    case 6: return gauss4_launch_d<6>(volts, T, F, N, out, in, nseg, bt, accumulate, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool gauss4_supported(const Plan &pl, int F, int N)
{
    const bool shape = pl.nseg == 1 ? (pl.D >= 1 && pl.D <= 6 && N <= 32 * pl.D)
                                    : (pl.D >= 1 && pl.D <= 4 && pl.nseg * pl.D * 32 >= N);
    return shape && N % 16 == 0 && F >= 1 && 64LL * F * N < (1LL << 31) - 16 &&
           (int64_t)F * pl.regions < (1LL << 30);
}

hipError_t launch_gauss4(const Plan &pl, const uint8_t *volts, int64_t T, int F, int N, int2 *acc, int accumulate,
                         hipStream_t s, const int2 *acc_in)
{
    if (!gauss4_supported(pl, F, N) || T < 1 || T > kMaxSamplesPerLaunch4 || !volts || (uintptr_t)volts % 16 ||
        !acc)
        return hipErrorInvalidValue;
    return launch_any(pl.D, pl.nseg, volts, T, F, N, acc, acc_in ? acc_in : acc, nullptr, accumulate, s);
}

hipError_t launch_gauss4_blocks(const Plan &pl, const BlockTable &bt, int n_blocks, int F, int N, int2 *acc,
                                int accumulate, hipStream_t s, const int2 *acc_in)
{
    if (!gauss4_supported(pl, F, N) || n_blocks < 1 || n_blocks > kMaxFusedBlocks || bt.chunks_per_block < 1 ||
        (int64_t)n_blocks * bt.chunks_per_block * 64 > kMaxSamplesPerLaunch4 || !acc)
        return hipErrorInvalidValue;
    for (int b = 0; b < n_blocks; ++b)
        if (!bt.p[b] || (uintptr_t)bt.p[b] % 16)
            return hipErrorInvalidValue;
    return launch_any(pl.D, pl.nseg, bt.p[0], (int64_t)n_blocks * bt.chunks_per_block * 64, F, N, acc,
                      acc_in ? acc_in : acc, &bt, accumulate, s);
}

#endif

}  // namespace xc
