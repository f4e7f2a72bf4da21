// Device-side helpers shared by the X-engine kernels (one translation unit
// each): vector types, XCD-aware work mapping, bounded loads, LDS transpose
// reads, barriers and wait counters.
#pragma once
#include "xcorr_internal.h"

#include <algorithm>
#include <type_traits>

namespace xc {
namespace {


typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) v2i lds_v2i;

constexpr int kThreads = 256;

// Work-group b is dispatched to XCD b % 8.  Give each XCD a contiguous range
// of work items so that the regions of one channel, and neighbouring channels
// (adjacent bytes of every time row), share that XCD's L2.  The grid is a
// multiple of 8; callers drop items >= the real count.
__device__ __forceinline__ int xcd_item()
{
    const int per = gridDim.x >> 3;
    return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

inline int xcd_grid(int nitems) { return ((nitems + 7) / 8) * 8; }

// 16 consecutive bytes of one (t, f) row starting at input i0; zero outside
// [0,T) x [0,N).  bps = bytes per sample.  vec_ok: rows are 16-byte aligned
// and N*bps is a multiple of 16, so a piece is either fully inside or fully
// outside the row.
__device__ __forceinline__ v4i load_piece(const uint8_t *__restrict__ volts, int64_t t, int64_t T,
                                          int f, int F, int N, int i0, int bps, int vec_ok)
{
    v4i r = {0, 0, 0, 0};
    if (t >= T || i0 >= N)
        return r;
    const int64_t row_bytes = (int64_t)N * bps;
    const uint8_t *src = volts + (t * F + f) * row_bytes + (int64_t)i0 * bps;
    if (vec_ok)
        return *reinterpret_cast<const v4i *>(src);
    const int avail = (int)std::min<int64_t>(16, row_bytes - (int64_t)i0 * bps);
    uint32_t w[4] = {0, 0, 0, 0};
    for (int b = 0; b < 16; ++b)
        if (b < avail)
            w[b >> 2] |= (uint32_t)src[b] << (8 * (b & 3));
    r.x = (int)w[0];
    r.y = (int)w[1];
    r.z = (int)w[2];
    r.w = (int)w[3];
    return r;
}

__device__ __forceinline__ int sext_nibble(uint32_t x, int lsb)
{
    return (int)(x << (28 - lsb)) >> 28;
}

}  // namespace
}  // namespace xc
