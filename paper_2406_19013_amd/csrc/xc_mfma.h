// Pieces shared by the int8 / FP16 MFMA kernels of the X-engine: the MFMA
// wrapper, the tile bookkeeping of a region, wait counters and the barrier.
#pragma once
#include "xc_device.h"

#include <utility>

namespace xc {
namespace {

typedef __attribute__((address_space(3))) uint8_t lds_u8;

// Calls f(std::integral_constant<int, I>) for I = B .. E-1, so that the body
// sees I as a constant expression (tile and block bookkeeping then folds at
// compile time instead of running as scalar loops).
template <int B, class F, int... Is>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Is...>)
{
    (f(std::integral_constant<int, B + Is>{}), ...);
}
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (E > B)
        static_for_impl<B>(f, std::make_integer_sequence<int, E - B>{});
}

__device__ __forceinline__ v16i mfma_i8(v4i a, v4i b, v16i c)
{
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

// Tiles of a region: TRI = the D(D+1)/2 tiles (I, J <= I) of D x D blocks;
// RECT = all D*D tiles of D row blocks by D column blocks.  Tile t is (I, J) in
// row-major order.  The 8 waves of a work-group are (role, half): half 0 owns
// tiles [0, NT/2), half 1 owns [NT/2, NT).
constexpr int tri_I(int t)
{
    int I = 0;
    while ((I + 1) * (I + 2) / 2 <= t)
        ++I;
    return I;
}
constexpr int tri_J(int t) { return t - tri_I(t) * (tri_I(t) + 1) / 2; }
// run-time versions (tile index not a compile-time constant)
__device__ __forceinline__ int tri_I_rt(int t)
{
    int I = (int)((sqrtf(8.f * t + 1.f) - 1.f) * 0.5f);
    I += (I + 1) * (I + 2) / 2 <= t;
    I -= I * (I + 1) / 2 > t;
    return I;
}
__device__ __forceinline__ int tri_J_rt(int t) { const int I = tri_I_rt(t); return t - I * (I + 1) / 2; }
constexpr int n_tiles(int D, bool tri) { return tri ? D * (D + 1) / 2 : D * D; }
constexpr int tile_I(int D, bool tri, int t) { return tri ? tri_I(t) : t / D; }
constexpr int tile_J(int D, bool tri, int t) { return tri ? tri_J(t) : t % D; }
constexpr int half_begin(int D, bool tri, int h) { return h ? n_tiles(D, tri) / 2 : 0; }
constexpr int half_end(int D, bool tri, int h) { return h ? n_tiles(D, tri) : n_tiles(D, tri) / 2; }
// LDS block index of a tile's row / column operand
constexpr int row_block(int D, bool tri, int t) { return tile_I(D, tri, t); }
constexpr int col_block(int D, bool tri, int t) { return tri ? tile_J(D, tri, t) : D + tile_J(D, tri, t); }
constexpr bool half_uses_row(int D, bool tri, int h, int b)
{
    for (int t = half_begin(D, tri, h); t < half_end(D, tri, h); ++t)
        if (row_block(D, tri, t) == b)
            return true;
    return false;
}
// Epilogue rounds of G staged tiles: slot u of round rc holds tile
// epilogue_slot_tile(...), or -1 if empty.  With an even G each round takes
// G/2 tiles from each half of the region, so that the waves of both halves
// free accumulator registers from the first round on; with an odd G tiles go
// in order.
constexpr int epilogue_slot_tile(int D, bool tri, int G, int rc, int u)
{
    const int NT = n_tiles(D, tri);
    if (G % 2) {
        const int t = rc * G + u;
        return t < NT ? t : -1;
    }
    const int H = G / 2, h = u < H ? 0 : 1;
    const int t = half_begin(D, tri, h) + rc * H + (u - h * H);
    return t < half_end(D, tri, h) ? t : -1;
}
constexpr int epilogue_rounds(int D, bool tri, int G)
{
    if (G % 2)
        return (n_tiles(D, tri) + G - 1) / G;
    const int H = G / 2;
    const int r0 = (half_end(D, tri, 0) - half_begin(D, tri, 0) + H - 1) / H;
    const int r1 = (half_end(D, tri, 1) - half_begin(D, tri, 1) + H - 1) / H;
    return r0 > r1 ? r0 : r1;
}
constexpr bool half_uses_col(int D, bool tri, int h, int b)
{
    for (int t = half_begin(D, tri, h); t < half_end(D, tri, h); ++t)
        if (col_block(D, tri, t) == b)
            return true;
    return false;
}

// s_waitcnt with only the vector-memory counter constrained (gfx9 encoding:
// vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
template <int N>
__device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N < 64, "vmcnt out of range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Wait until the chunk before the last r chunks a wave issued has arrived:
// at most r (wave-uniform, 0 <= r <= MAXR) chunks of LOADS loads each may
// still be outstanding.
template <int LOADS, int MAXR>
__device__ __forceinline__ void wait_vmcnt_chunks(int r)
{
    if constexpr (MAXR > 0) {
        if (r >= MAXR)
            wait_vmcnt<LOADS * MAXR>();
        else
            wait_vmcnt_chunks<LOADS, MAXR - 1>(r);
    } else {
        wait_vmcnt<0>();
    }
}

constexpr int kBufferOutOfRange = (int)0xFFFFFFF0;  // any offset >= num_records reads 0

// Cache policy of the LDS-DMA input loads (sc0 | nt | sc1): every input byte
// is read exactly once per launch, as a stream.  Measured 9 % faster on the
// 192-input kernel than the default policy, with identical results.
constexpr int kStreamLoadPolicy = 1 | 2 | 16;
// Loads whose bytes other work-groups of the XCD read at about the same time
// (a segment of inputs shared by the rectangles of one channel): the default
// policy, which keeps them in L2.
constexpr int kSharedLoadPolicy = 0;

// Work-group barrier without the release/acquire fence of __syncthreads (the
// fence would wait for every LDS-DMA load in flight, i.e. drain the ring).
// The "memory" clobber keeps the compiler from moving LDS accesses across it;
// loads whose data must be visible are waited for explicitly before it.
__device__ __forceinline__ void barrier_no_fence() { asm volatile("s_barrier" ::: "memory"); }

constexpr int kMfmaThreads = 512;   // 8 waves per work-group

// Running sums of one quad of an epilogue (rows i0 .. i0+3 of column j of a
// channel's lower triangle, the first at triangle index p), all four
// requested before any of the quad's stores: a thread loads and stores only
// its own elements, so the loads need not wait for earlier stores.  A row
// that does not exist (past N, or above the diagonal of a diagonal tile)
// reads element 0 and its value goes unused.
template <typename T2>
__device__ __forceinline__ void quad_running_sums(const T2 *sums, int p, int i0, int j, bool diag, int N,
                                                  T2 (&o)[4])
{
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int i = i0 + m;
        o[m] = sums[i < N && (!diag || j <= i) ? p : 0];
        p += i + 1;
    }
}

}  // namespace
}  // namespace xc
