// Device code of the three-product 4+4-bit int8-MFMA path.
//
// Per channel the packed voltages form a matrix X[i][t], one byte per sample
// (high nibble re, low nibble im, two's complement).  Three int8 forms of a
// byte x are exact and cost one bit operation each:
//     A = x ^ 0x08 = 16 re + im + 8,   B = x ^ 0x07 = 16 re - im + 7,
//     R = x & 0xF0 = 16 re                               (all in [-128, 127]).
// Over a set of samples (padding samples are zero bytes and count as zero
// voltages) the three real products
//     P_ab = A_i B_j^T,  P_ba = B_i A_j^T,  P_rr = R_i R_j^T
// give the visibility exactly (with SR_k = sum R_k, SA_k = sum A_k,
// g_k = 16 SR_k - 15 SA_k, h_k = 16 SR_k - SA_k, and Tp the padded count):
//     32 Im V_ij = P_ab - P_ba + g_i - g_j
//      2 Sum im_i im_j = 2 P_rr - P_ab - P_ba + h_i + h_j + 128 Tp
//     Re V_ij = P_rr / 256 + Sum im_i im_j
// so a tile costs three MFMAs per K step instead of the four real products of
// the direct form, and on a diagonal tile P_ba is the transpose of P_ab: two.
// Every product is an exact integer; |A B| and |R R| are at most 2^14 per
// sample, so each accumulator stays below 2^31 for up to 131,071 samples, and
// the combinations are evaluated in wrapping 32-bit arithmetic, whose result
// is exact because the true values (32 Im, 2 II) fit in int32.
//
// The per-input sums come from unsigned byte SADs, which issue beside the
// MFMAs (a dot-product instruction would share their pipe): with Z = x ^ 0x88
// (both nibbles offset by 8, so the unsigned byte is 16 (re + 8) + im + 8)
// and |A - R| = im + 8 per byte (A and R share the high nibble),
//     SA = sum Z - 128 Tp,   SR = sum Z - sum |A - R| - 128 Tp.
//
// Work split.  One work-group per channel region (here: the whole triangle of
// D 32-input blocks, D <= 6), persistent: each work-group walks its channels
// as one continuous stream of 64-sample chunks through an LDS ring, so the
// next channel's first chunks are in flight while the current channel's
// results are stored.  The triangle's tiles are split over 8 waves (two per
// SIMD) so that every SIMD carries near-equal MFMA work and the waves unpack
// as few blocks per K step as possible (a block's three forms are computed by
// every wave that reads it).  A wave owns every product of its tiles,
// combines them in registers and stores the visibilities directly (no
// staging), except the transposed P_ab of a diagonal tile, which goes through
// a small LDS tile.
#pragma once
#include "xc_mfma4.h"

namespace xc {
namespace {

// ---- compile-time work split of a triangle of D blocks over 8 waves --------

constexpr int g3_ntiles(int D) { return D * (D + 1) / 2; }
constexpr bool g3_diag(int t) { return tri_I(t) == tri_J(t); }
constexpr int g3_abs(int x) { return x < 0 ? -x : x; }

// Region geometry, by shape SH.  A triangle (SH = 0) of D blocks: local
// blocks 0 .. D-1, tiles (I, J <= I) in row-major order.  A D x D rectangle
// below the diagonal (SH = 1, D <= 4): local row blocks 0 .. D-1 and column
// blocks D .. 2D-1, tile t = (t / D, D + t % D), no diagonal tiles.  A
// channel pair (SH = 2): the triangles of one segment in two neighbouring
// channels, local blocks 0 .. D-1 of the first and D .. 2D-1 of the second,
// the second triangle's tiles after the first's.
constexpr int kTri = 0, kRect = 1, kPair = 2;
template <int SH>
constexpr int g3_tiles(int D) { return SH == kRect ? D * D : SH == kPair ? D * (D + 1) : D * (D + 1) / 2; }
template <int SH>
constexpr int g3_blocks(int D) { return SH == kTri ? D : 2 * D; }
template <int SH>
constexpr int g3_row(int D, int t)
{
    return SH == kRect ? t / D : SH == kPair && t >= D * (D + 1) / 2 ? D + tri_I(t - D * (D + 1) / 2) : tri_I(t);
}
template <int SH>
constexpr int g3_col(int D, int t)
{
    return SH == kRect ? D + t % D : SH == kPair && t >= D * (D + 1) / 2 ? D + tri_J(t - D * (D + 1) / 2) : tri_J(t);
}
template <int SH>
constexpr bool g3_isdiag(int D, int t) { return SH != kRect && g3_row<SH>(D, t) == g3_col<SH>(D, t); }

// Waves per work-group: two per SIMD, 256 registers each.
#ifndef XC_G3_WAVES
#define XC_G3_WAVES 8
#endif
constexpr int kG3Waves = XC_G3_WAVES;
constexpr int kG3Threads = 64 * kG3Waves;

// The split, evaluated once per D: wave slot s (on SIMD s % 4) takes the
// tiles whose bits are set in mask[s] (bit t: tile t in row-major order).
constexpr int kG3MaxWaves = 16;
struct G3Split {
    uint32_t mask[kG3MaxWaves];
    int sum_owner[8];   // wave slot that sums the forms of local block b
};
template <int SH>
constexpr int g3_units(int D, int t) { return g3_isdiag<SH>(D, t) ? 2 : 3; }
template <int SH>
constexpr bool g3_touches(int D, uint32_t mask, int b)
{
    for (int t = 0; t < g3_tiles<SH>(D); ++t)
        if ((mask >> t & 1) && (g3_row<SH>(D, t) == b || g3_col<SH>(D, t) == b))
            return true;
    return false;
}

// Generic split: tiles in row-major order are cut into W contiguous segments
// at the boundaries whose cumulative MFMA count (3 per off-diagonal tile, 2
// per diagonal tile) is closest to k/W of the total; segments go to SIMDs
// largest first, each to the SIMD with the least MFMA work so far; the sums
// of a block go to the least-loaded wave that reads it.
template <int SH>
constexpr G3Split g3_contiguous_split(int D, int W)
{
    G3Split sp{};
    const int NT = g3_tiles<SH>(D);
    int cum[6 * 7 / 2 + 1] = {};
    for (int t = 0; t < NT; ++t)
        cum[t + 1] = cum[t] + g3_units<SH>(D, t);
    const int U = cum[NT];
    int bound[kG3MaxWaves + 1] = {};
    for (int k = 1; k < W; ++k) {
        int best = 0;
        for (int b = 0; b <= NT; ++b)
            if (g3_abs(W * cum[b] - k * U) < g3_abs(W * cum[best] - k * U))
                best = b;
        bound[k] = best;
    }
    bound[W] = NT;
    int su[kG3MaxWaves] = {};
    for (int k = 0; k < W; ++k)
        su[k] = cum[bound[k + 1]] - cum[bound[k]];
    bool placed[kG3MaxWaves] = {};
    int simd_load[4] = {}, simd_used[4] = {}, units[kG3MaxWaves] = {};
    for (int n = 0; n < W; ++n) {
        int k = -1;
        for (int m = 0; m < W; ++m)
            if (!placed[m] && (k < 0 || su[m] > su[k]))
                k = m;
        int simd = 0;
        for (int q = 1; q < 4; ++q)
            if (simd_used[q] < W / 4 && (simd_used[simd] >= W / 4 || simd_load[q] < simd_load[simd]))
                simd = q;
        const int slot = simd + 4 * simd_used[simd];
        placed[k] = true;
        simd_load[simd] += su[k];
        ++simd_used[simd];
        for (int t = bound[k]; t < bound[k + 1]; ++t)
            sp.mask[slot] |= 1u << t;
        units[slot] = su[k];
    }
    for (int b = 0; b < g3_blocks<SH>(D); ++b) {
        int best = -1;
        for (int s = 0; s < W; ++s)
            if (g3_touches<SH>(D, sp.mask[s], b) && (best < 0 || units[s] < units[best]))
                best = s;
        sp.sum_owner[b] = best;
        if (best >= 0)
            units[best] += 3;
    }
    return sp;
}

// Searched splits for 8 waves and D = 5, 6: per SIMD the MFMA counts are as
// even as the tile sizes allow, each wave holds 5 to 9 MFMA accumulators, and
// the number of blocks that waves unpack per K step is the smallest found
// (D = 6: 20 instead of 25 for contiguous segments; D = 5: 18 instead of 20).
//   D = 6: slot 0 {(1,1) (4,1)}  1 {(2,2) (4,2)}  2 {(4,3) (5,3) (5,4)}
//          3 {(0,0) (4,0) (4,4)}  4 {(2,0) (5,0) (5,2)}  5 {(1,0) (3,0) (3,1)}
//          6 {(5,1) (5,5)}  7 {(2,1) (3,2) (3,3)}
//   D = 5: slot 0 {(4,2)}  1 {(4,3) (4,4)}  2 {(1,0) (1,1)}  3 {(0,0) (4,0)}
//          4 {(3,0) (3,3)}  5 {(2,2) (3,2)}  6 {(2,0) (2,1)}  7 {(3,1) (4,1)}
template <int SH>
constexpr G3Split g3_make_split(int D, int W)
{
    if (SH == kTri && W == 8 && D == 6)
        return G3Split{{0x804, 0x1020, 0xc2000, 0x4401, 0x28008, 0xc2, 0x110000, 0x310}, {3, 0, 1, 2, 0, 6, -1, -1}};
    if (SH == kTri && W == 8 && D == 5)
        return G3Split{{0x1000, 0x6000, 0x6, 0x401, 0x240, 0x120, 0x18, 0x880}, {4, 2, 5, 1, 0, -1, -1, -1}};
    return g3_contiguous_split<SH>(D, W);
}
template <int D, int SH>
constexpr G3Split kG3Split = g3_make_split<SH>(D, kG3Waves);

template <int D, int SH>
constexpr uint32_t g3_mask(int s) { return kG3Split<D, SH>.mask[s]; }
template <int D, int SH>
constexpr bool g3_has(int s, int t) { return t < 32 && (g3_mask<D, SH>(s) >> t & 1); }
// position of tile t among the tiles of slot s (its accumulator index)
template <int D, int SH>
constexpr int g3_rank(int s, int t)
{
    int r = 0;
    for (int u = 0; u < t; ++u)
        r += g3_has<D, SH>(s, u);
    return r;
}
template <int D, int SH>
constexpr int g3_ntiles_of(int s) { return g3_rank<D, SH>(s, g3_tiles<SH>(D)); }
template <int D, int SH>
constexpr bool g3_uses_block(int s, int b) { return g3_touches<SH>(D, g3_mask<D, SH>(s), b); }
template <int D, int SH>
constexpr bool g3_owns_sums(int s, int b)
{
    return kG3Split<D, SH>.sum_owner[b] == s;
}
// Order in which a wave unpacks its blocks within a K step: greedily the
// block that completes the most MFMA work with the blocks already unpacked
// (ties: the lower block), so that MFMAs start early and the later blocks'
// unpacking runs under them.  pos < 0 for a block the wave does not read.
template <int D, int SH>
constexpr int g3_block_pos(int s, int b)
{
    constexpr int NB = g3_blocks<SH>(D);
    if (!g3_uses_block<D, SH>(s, b))
        return -1;
    bool done[8] = {};
    for (int p = 0; p < NB; ++p) {
        int best = -1, best_gain = -1;
        for (int c = 0; c < NB; ++c) {
            if (done[c] || !g3_uses_block<D, SH>(s, c))
                continue;
            int gain = 0;
            for (int t = 0; t < g3_tiles<SH>(D); ++t) {
                const int r = g3_row<SH>(D, t), k = g3_col<SH>(D, t);
                if (g3_has<D, SH>(s, t) && (r == c || k == c)) {
                    const int o = r == c ? k : r;
                    if (o == c || done[o])
                        gain += g3_units<SH>(D, t);
                }
            }
            if (gain > best_gain) {
                best = c;
                best_gain = gain;
            }
        }
        if (best == b)
            return p;
        done[best] = true;
    }
    return -1;
}
// a tile's MFMAs go right after the later of its two blocks is unpacked
template <int D, int SH>
constexpr int g3_tile_pos(int s, int t)
{
    const int a = g3_block_pos<D, SH>(s, g3_row<SH>(D, t)), b = g3_block_pos<D, SH>(s, g3_col<SH>(D, t));
    return a > b ? a : b;
}
template <int D, int SH>
constexpr int g3_mfmas_of(int s)
{
    int n = 0;
    for (int t = 0; t < g3_tiles<SH>(D); ++t)
        if (g3_has<D, SH>(s, t))
            n += g3_units<SH>(D, t);
    return n;
}

// rows of a tile's running sums that an accumulating epilogue requests ahead
// of its stores: the whole tile where the registers allow, else half of it
template <int SH>
constexpr int g3_old_rows(int D) { return (SH == kTri && D <= 3) || (SH == kPair && D >= 4) ? 8 : 16; }

// LDS transpose slot of a diagonal tile: its block
template <int D, int SH>
constexpr int g3_diag_slot(int t) { return g3_row<SH>(D, t); }

// ---- resources ---------------------------------------------------------------

// two work-groups per CU for small triangles (128 registers per wave); a
// rectangle's or a channel pair's 2D blocks of operands need the full 256
template <int SH>
constexpr int g3_wgs_per_cu(int D) { return SH == kTri && D <= 3 ? 2 : 1; }
// waves of this kernel per SIMD
template <int SH>
constexpr int g3_waves_per_eu(int D) { return g3_wgs_per_cu<SH>(D) * kG3Waves / 4; }
// ring slots: 8 (4 with two work-groups per CU; 7 for a pair of 4-block
// triangles, whose 8 transpose tiles would not fit beside 8)
template <int SH>
constexpr int g3_nbuf(int D) { return g3_wgs_per_cu<SH>(D) == 2 ? 4 : SH == kPair && D >= 4 ? 7 : 8; }
constexpr int kG3Chunk = 64;                             // time rows per ring slot
#ifndef XC_G3_CPB
#define XC_G3_CPB 2
#endif
constexpr int kG3ChunksPerBarrier = XC_G3_CPB;             // chunks per work-group barrier
constexpr int kG3TileStride = 33;                        // ints per row of a transpose tile
template <int SH>
constexpr int g3_ring_bytes(int D) { return g3_nbuf<SH>(D) * kG3Chunk * kRowBytes; }
template <int SH>
constexpr int g3_tr_bytes(int D) { return SH == kRect ? 0 : g3_blocks<SH>(D) * 32 * kG3TileStride * 4; }
template <int SH>
constexpr int g3_gh_bytes(int D) { return g3_blocks<SH>(D) * 32 * 8; }
template <int SH>
constexpr int g3_smem_bytes(int D) { return g3_ring_bytes<SH>(D) + g3_tr_bytes<SH>(D) + g3_gh_bytes<SH>(D); }

// LDS-only wait: outstanding LDS operations of this wave done, memory
// operations in flight left alone (vmcnt and expcnt at their maxima).
__device__ __forceinline__ void wait_lgkm0() { __builtin_amdgcn_s_waitcnt(0xF | (3 << 14) | (7 << 4)); }

// Source of a launch: one contiguous input, or a table of caller blocks that
// hold whole 64-sample chunks (chunk c of an item is chunk c % cpb of block
// c / cpb; every channel item walks the same table).
struct G3Src {
    const uint8_t *volts;
    const BlockTable *bt;
};

struct G3Args {
    const uint8_t *volts;   // [T][F][N] packed (MB = 0)
    int64_t T;              // samples (MB = 1: n_blocks * cpb * 64)
    int F, N;
    int nreg;               // regions of this launch's shape per channel (or channel pair)
    int per;                // items (channel or channel pair, region) per XCD range
    int2 *out;              // [F][P] results
    const int2 *in;         // [F][P] running sums (ACC = 1)
    int mrow0, mrows;       // work-group rows (blockIdx / 8) that serve these items
};

// Items of a launch of shape SH: (channel, region), or (channel pair, region)
// for SH = kPair, the last pair of an odd F holding one channel.
template <int SH>
__host__ __device__ __forceinline__ int g3_items(int F, int nreg) { return (SH == kPair ? (F + 1) / 2 : F) * nreg; }

// First global block of a region's rows and of its columns: triangle r of a
// channel (or of a channel pair) starts at block D r; rectangle k (k-th pair
// a > b in row-major order) has rows from segment a and columns from segment
// b.
template <int D, int SH>
__device__ __forceinline__ void g3_region_origin(int r, int &rb, int &cb)
{
    if constexpr (SH != kRect) {
        rb = cb = D * r;
    } else {
        int a = (int)((1.f + sqrtf(1.f + 8.f * r)) * 0.5f);
        while (a * (a - 1) / 2 > r)
            --a;
        while ((a + 1) * a / 2 <= r)
            ++a;
        rb = D * a;
        cb = D * (r - a * (a - 1) / 2);
    }
}

// One wave's share of a launch: its tiles of every channel item of its
// work-group, K loop over the continuous chunk stream, and the epilogue of
// each item.  ACC: 0 stores the sums of this launch, 1 adds the running sums
// of `in`.
template <int D, int SH, int SLOT, int ACC, int MB>
__device__ __forceinline__ void g3_wave(uint8_t *smem, const G3Args &a, const BlockTable *bt,
                                        const uint8_t *__restrict__ volts)
{
    constexpr int NBUF = g3_nbuf<SH>(D);
    constexpr int KC = kG3Chunk;
    constexpr int BUF = KC * kRowBytes;
    constexpr int LOADS = KC * 16 / kG3Threads;         // 16-byte DMA units per lane per chunk
    constexpr int NTT = g3_tiles<SH>(D);
    constexpr int NB = g3_blocks<SH>(D);
    constexpr int NT = g3_ntiles_of<D, SH>(SLOT) > 0 ? g3_ntiles_of<D, SH>(SLOT) : 1;

    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    if constexpr (g3_waves_per_eu<SH>(D) == 1) {
        // an AGPR operand in the function makes the compiler take the MFMA
        // forms that accumulate in AGPRs (with one wave per SIMD it then
        // has 256 of each)
        int hint = 0;
        asm volatile("" : "+a"(hint));
    }
    const int lane = tid & 63;
    const int g = lane >> 4, q = lane & 15;
    lds_u8 *const ring = (lds_u8 *)smem;
    int *const trs = (int *)(smem + g3_ring_bytes<SH>(D));                             // transpose tiles
    int *const gh = (int *)(smem + g3_ring_bytes<SH>(D) + g3_tr_bytes<SH>(D));      // g, h per local input

    // this work-group's items (channel, region): the local items m, m + M, ...
    // of its XCD's range of consecutive items
    const int xcd = blockIdx.x & 7, m = (int)(blockIdx.x >> 3) - a.mrow0, M = a.mrows;
    const int r0 = xcd * a.per;
    const int rlen = min(a.per, g3_items<SH>(a.F, a.nreg) - r0);
    const int n_my = rlen > m ? (rlen - m + M - 1) / M : 0;
    const int nch = (int)((a.T + KC - 1) / KC);
    const int total = n_my * nch;
    if (total == 0)
        return;
    const int64_t row_bytes = (int64_t)a.F * a.N;
    const int64_t chunk_bytes = KC * row_bytes;
    const int Tp = nch * KC;

    // DMA share of this wave: unit U = (SLOT * LOADS + k) * 64 + lane of a
    // chunk -> time row U / 16, position U % 16 (swizzled unit p); units
    // 0 .. 2D-1 hold the region's row blocks, 2D .. 4D-1 its column blocks
    // (rectangles) or the same blocks of the next channel (channel pairs);
    // the lane offsets of an item are recomputed when the issue pointer
    // reaches it, so nothing is held across the K loop for them
    auto dma_offset = [&](int k, int f, int rb, int cb) {
        const int U = (SLOT * LOADS + k) * 64 + lane;
        const int r = U >> 4;
        const int p = (U & 15) ^ ((r & 7) << 1);
        const bool hi = p >= 2 * D;
        const int fo = SH == kPair && hi ? f + 1 : f;
        const int byte = !hi ? 32 * rb + 16 * p : 32 * (SH == kPair ? rb : cb) + 16 * (p - 2 * D);
        return p < 2 * NB && byte < a.N && fo < a.F ? (int)(r * row_bytes) + fo * a.N + byte : kBufferOutOfRange;
    };
    // operand read offsets (see frag_tr8): row (g >> 1) * 16 + (q >> 1) of the
    // K step, unit 2b + (g & 1) swizzled
    const int row_off = ((g >> 1) * 16 + (q >> 1)) * kRowBytes + (q & 1) * 8;
    int colo[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
        colo[b] = ((2 * b + (g & 1)) ^ (q & 14)) << 4;

    // issue state (wave-uniform): item and chunk of the next chunk to issue
    int is_k = 0, is_c = 0;
    int voff[LOADS];
    auto set_issue_item = [&](int k) {
        const int it = r0 + m + k * M;
        const int fq = it / a.nreg;
        int rb, cb;
        g3_region_origin<D, SH>(it - fq * a.nreg, rb, cb);
#pragma unroll
        for (int u = 0; u < LOADS; ++u)
            voff[u] = dma_offset(u, SH == kPair ? 2 * fq : fq, rb, cb);
    };
    set_issue_item(0);
    auto issue_next = [&](int bufi) {
        const uint8_t *src;
        int records;
        if constexpr (MB) {
            // addressed from the first block (the restrict-qualified base)
            src = volts + (bt->p[is_c / bt->chunks_per_block] - bt->p[0]) +
                  (int64_t)(is_c % bt->chunks_per_block) * chunk_bytes;
            records = (int)chunk_bytes;
        } else {
            src = volts + (int64_t)is_c * chunk_bytes;
            const int64_t rows = min((int64_t)KC, a.T - (int64_t)is_c * KC);
            records = (int)(rows * row_bytes);
        }
        __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc((void *)src, (short)0, records, 0x00020000);
        lds_u8 *dst = ring + bufi * BUF + SLOT * LOADS * 1024;
#pragma unroll
        for (int k = 0; k < LOADS; ++k)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (__attribute__((address_space(3))) void *)(dst + k * 1024),
                                                     16, voff[k], 0, 0, SH == kRect ? kSharedLoadPolicy : kStreamLoadPolicy);
        if (++is_c == nch) {
            is_c = 0;
            if (++is_k < n_my)
                set_issue_item(is_k);
        }
    };

    v16i acc_ab[NT], acc_ba[NT], acc_rr[NT];
    // per-input sums of the owned blocks, as unsigned byte SADs (two chains
    // each): sz = sum of X ^ 0x88 (16 (re + 8) + im + 8 per sample), sl =
    // sum of |A - R| (im + 8 per sample: A and R share the high nibble)
    int sz[NB], sl[NB], sz2[NB], sl2[NB];
    auto clear = [&]() {
        static_for<0, NT>([&](auto tc) {
            acc_ab[tc] = v16i{};
            acc_ba[tc] = v16i{};
            acc_rr[tc] = v16i{};
        });
        static_for<0, NB>([&](auto bc) {
            sz[bc] = 0;
            sl[bc] = 0;
            sz2[bc] = 0;
            sl2[bc] = 0;
        });
    };
    clear();

    // The K loop is a two-stage pipeline over 32-sample K steps: while the
    // MFMAs of one step run, the next step's operands are read from LDS and
    // unpacked into the other register set.  raw: the packed bytes of a step;
    // A, B, R: its three forms; the owner of a block also sums its forms.
    auto read_step = [&](lds_u8 *cb, int koff, v4i *X) {
        static_for<0, NB>([&](auto bc) {
            constexpr int b = bc;
            if constexpr (g3_uses_block<D, SH>(SLOT, b))
                X[b] = frag_tr8<8 * kRowBytes>(cb + colo[b] + koff);
        });
    };
    // epilogue of one item (channel, region): combine, descale and store this
    // wave's tiles
    auto epilogue = [&](int it) {
        const int fq = it / a.nreg;
        const int f = SH == kPair ? 2 * fq : fq;   // first channel of the item
        int rb, cb;
        g3_region_origin<D, SH>(it - fq * a.nreg, rb, cb);
        // every wave has read the previous item's g and h before they are
        // overwritten: the group barriers of the K loop need not fall between
        // two epilogues (an item of at most CPB chunks that ends the
        // work-group's stream has none)
        wait_lgkm0();
        barrier_no_fence();
        // per-input sums: lanes l and l + 32 hold the two K halves of input l % 32
        static_for<0, NB>([&](auto bc) {
            constexpr int b = bc;
            if constexpr (g3_owns_sums<D, SH>(SLOT, b)) {
                const int szl = sz[b] + sz2[b], sll = sl[b] + sl2[b];
                const uint32_t szt = (uint32_t)(szl + __shfl_xor(szl, 32));
                const uint32_t slt = (uint32_t)(sll + __shfl_xor(sll, 32));
                // g = 16 SR - 15 SA and h = 16 SR - SA, with SR = sum R =
                // szt - slt - 128 Tp and SA = sum A = szt - 128 Tp
                if (lane < 32)
                    *(int2 *)&gh[(b * 32 + lane) * 2] =
                        make_int2((int)(szt - 16u * slt - 128u * (uint32_t)Tp),
                                  (int)(15u * szt - 16u * slt - 1920u * (uint32_t)Tp));
            }
        });
        wait_lgkm0();
        barrier_no_fence();
        const int64_t P = (int64_t)a.N * (a.N + 1) / 2;
        const int jl = lane & 31;
        const int il0 = 4 * (lane >> 5);
        static_for<0, NTT>([&](auto tc) {
            constexpr int t = tc;
            if constexpr (g3_has<D, SH>(SLOT, t)) {
            constexpr int q = g3_rank<D, SH>(SLOT, t);
            constexpr int I = g3_row<SH>(D, t), J = g3_col<SH>(D, t);   // local blocks
            constexpr bool diag = g3_isdiag<SH>(D, t);
            // a channel pair's second triangle: the next channel, blocks
            // I - D and J - D of its segment (none for the last of an odd F)
            constexpr bool second = SH == kPair && I >= D;
            constexpr int Ib = second ? I - D : I, Jb = second ? J - D : J;
            const int fch = second ? f + 1 : f;
            if (fch < a.F) {
            int2 *const out_f = a.out + (int64_t)fch * P;
            const int2 *const in_f = a.in + (int64_t)fch * P;
            // column input: local index for the sums, global for the output
            const int jloc = J * 32 + jl;
            const int j = (SH == kRect ? cb + (J - D) : rb + Jb) * 32 + jl;
            const int2 ghj = *(const int2 *)&gh[jloc * 2];
            // running sums of the tile's rows (ACC = 1), OR of them at a time
            // (the first group before the transpose), each group requested
            // before the stores it feeds: the elements a thread loads and
            // stores are its own, so the loads need not wait for earlier
            // stores (a valid address where the pair does not exist)
            constexpr int OR = g3_old_rows<SH>(D);
            int2 old[ACC ? OR : 1];
            auto load_old = [&](int r0) {
#pragma unroll
                for (int r = 0; r < OR; ++r) {
                    const int i = (rb + Ib) * 32 + 8 * ((r0 + r) >> 2) + il0 + ((r0 + r) & 3);
                    const bool ok = i < a.N && (!diag || j <= i);
                    old[r] = in_f[ok ? (int64_t)i * (i + 1) / 2 + j : 0];
                }
            };
            if constexpr (ACC)
                load_old(0);
            v16i ba;
            if constexpr (diag) {
                // P_ba of a diagonal tile is the transpose of its P_ab
                int *const tr = trs + g3_diag_slot<D, SH>(t) * 32 * kG3TileStride;
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    tr[(8 * (r >> 2) + il0 + (r & 3)) * kG3TileStride + jl] = acc_ab[q][r];
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    ba[r] = tr[jl * kG3TileStride + 8 * (r >> 2) + il0 + (r & 3)];
            } else {
                ba = acc_ba[q];
            }
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                const int ibl = I * 32 + 8 * r4 + il0;                // rows ibl .. ibl + 3 (local)
                const int ib = (rb + Ib) * 32 + 8 * r4 + il0;         // and their global inputs
                if constexpr (ACC && OR < 16)
                    if (r4 > 0 && 4 * r4 % OR == 0)
                        load_old(4 * r4);
                const int4 ghi01 = *(const int4 *)&gh[ibl * 2];
                const int4 ghi23 = *(const int4 *)&gh[ibl * 2 + 4];
                const int gi[4] = {ghi01.x, ghi01.z, ghi23.x, ghi23.z};
                const int hi[4] = {ghi01.y, ghi01.w, ghi23.y, ghi23.w};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int r = 4 * r4 + u;
                    const int i = ib + u;
                    const uint32_t ab = (uint32_t)acc_ab[q][r], bav = (uint32_t)ba[r];
                    const uint32_t rr = (uint32_t)acc_rr[q][r];
                    const int im = (int)(ab - bav + (uint32_t)gi[u] - (uint32_t)ghj.x) >> 5;
                    const int ii = (int)(2u * rr - ab - bav + (uint32_t)hi[u] + (uint32_t)ghj.y + 128u * (uint32_t)Tp) >> 1;
                    int re = (acc_rr[q][r] >> 8) + ii;
                    int imv = im;
                    if constexpr (ACC) {
                        re += old[r % OR].x;
                        imv += old[r % OR].y;
                    }
                    if (i < a.N && (!diag || j <= i))
                        out_f[(int64_t)i * (i + 1) / 2 + j] = make_int2(re, imv);
                }
            }
            }
            }
        });
    };

    // Chunks are waited for and their slots recycled in groups of CPB: one
    // work-group barrier per group.  The prologue fills every slot, waits for
    // the first group and reads the packed operands of its first K step.
    constexpr int CPB = kG3ChunksPerBarrier;
    static_assert(CPB >= 1 && CPB < NBUF, "groups must leave chunks in flight");
    int n_issued = 0;
#pragma unroll
    for (int c = 0; c < NBUF; ++c)
        if (c < total) {
            issue_next(c);
            ++n_issued;
        }
    wait_vmcnt_chunks<LOADS, NBUF - 1>(n_issued - 1 - min(CPB - 1, total - 1));
    barrier_no_fence();
    v4i X0[NB], X1[NB];    // packed operands of the current and the next K step
    read_step(ring + row_off, 0, X0);

    // one K step: unpack its operands and issue its MFMAs
    // Dataflow order: unpack one block, then issue the MFMAs of the tiles
    // that block completes, then the next block, whose unpack runs under
    // those MFMAs; the scheduling groups at the end keep MFMAs and VALU work
    // interleaved (one MFMA, then up to 6 VALU instructions).
    auto step = [&](const v4i *X) {
        v4i A[NB], B[NB], R[NB];
        static_for<0, NB>([&](auto kc) {
            constexpr int k = kc;
            static_for<0, NB>([&](auto bc) {
                constexpr int b = bc;
                if constexpr (g3_block_pos<D, SH>(SLOT, b) == k) {
                    A[b] = X[b] ^ 0x08080808;
                    B[b] = X[b] ^ 0x07070707;
                    R[b] = X[b] & (int)0xF0F0F0F0;
                    if constexpr (g3_owns_sums<D, SH>(SLOT, b)) {
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            int &z = k & 1 ? sz2[b] : sz[b];
                            int &l = k & 1 ? sl2[b] : sl[b];
                            z = (int)__builtin_amdgcn_sad_u8((uint32_t)(A[b][k] ^ (int)0x80808080), 0u, (uint32_t)z);
                            l = (int)__builtin_amdgcn_sad_u8((uint32_t)A[b][k], (uint32_t)R[b][k], (uint32_t)l);
                        }
                    }
                }
            });
            static_for<0, NTT>([&](auto tc) {
                constexpr int t = tc;
                if constexpr (g3_has<D, SH>(SLOT, t) && g3_tile_pos<D, SH>(SLOT, t) == k) {
                    constexpr int q = g3_rank<D, SH>(SLOT, t);
                    constexpr int I = g3_row<SH>(D, t), J = g3_col<SH>(D, t);
                    acc_ab[q] = mfma_i8(A[I], B[J], acc_ab[q]);
                    if constexpr (!g3_isdiag<SH>(D, t))
                        acc_ba[q] = mfma_i8(B[I], A[J], acc_ba[q]);
                    acc_rr[q] = mfma_i8(R[I], R[J], acc_rr[q]);
                }
            });
        });
        static_for<0, g3_mfmas_of<D, SH>(SLOT)>([&](auto) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 6, 0);   // up to six VALU
        });
    };

    int bufc = 0;          // ring slot of chunk gi
    int ck = 0, cc = 0;    // item, and chunk within the item, being computed
    for (int gi = 0; gi < total; ++gi) {
        lds_u8 *const cb = ring + bufc * BUF + row_off;
        const int nbufc = bufc + 1 == NBUF ? 0 : bufc + 1;
        // first K step of chunk gi; the second step's operands are read
        // meanwhile
        read_step(cb, 32 * kRowBytes, X1);
        step(X0);
        const bool more = gi + 1 < total;
        const bool item_end = cc + 1 == nch;
        if (more && (gi + 1) % CPB == 0) {
            // Next group gi + 1 .. gi + CPB: complete when this wave has at
            // most the chunks issued after it outstanding (loads complete in
            // order; the stores of an earlier epilogue only make the wait
            // longer).  After the barrier every wave has read both steps of
            // this group's chunks (each waits for its LDS reads first), so
            // their slots take the next chunks of the stream.
            const int last = min(gi + CPB, total - 1);
            wait_vmcnt_chunks<LOADS, NBUF - 1>(n_issued - 1 - last);
            wait_lgkm0();
            barrier_no_fence();
            int slot = bufc - (CPB - 1);
            slot = slot < 0 ? slot + NBUF : slot;
#pragma unroll
            for (int k = 0; k < CPB; ++k) {
                if (n_issued < total) {
                    issue_next(slot);
                    ++n_issued;
                }
                slot = slot + 1 == NBUF ? 0 : slot + 1;
            }
        }
        // second K step of chunk gi, with the next chunk's first step read
        // meanwhile unless an item ends here
        lds_u8 *const nb = ring + nbufc * BUF + row_off;
        if (more && !item_end)
            read_step(nb, 0, X0);
        step(X1);
        if (item_end) {
            epilogue(r0 + m + ck * M);
            clear();
            if (more)
                read_step(nb, 0, X0);
        }
        bufc = nbufc;
        if (item_end) {
            cc = 0;
            ++ck;
        } else {
            ++cc;
        }
    }
}

template <int D, int SH, int ACC, int MB>
__device__ __forceinline__ void g3_dispatch(uint8_t *smem, const G3Args &a, const BlockTable *bt)
{
    switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
#define XC_CASE(W)                                              \
    case W:                                                     \
        if constexpr (W < kG3Waves)                             \
            g3_wave<D, SH, W, ACC, MB>(smem, a, bt, a.volts); \
        break;
        XC_CASE(0) XC_CASE(1) XC_CASE(2) XC_CASE(3) XC_CASE(4) XC_CASE(5) XC_CASE(6) XC_CASE(7)
        XC_CASE(8) XC_CASE(9) XC_CASE(10) XC_CASE(11) XC_CASE(12) XC_CASE(13) XC_CASE(14) XC_CASE(15)
#undef XC_CASE
    default: break;
    }
}

}  // namespace
}  // namespace xc
