// Device code of the 4+4-bit int8-MFMA path: one work-group body per region
// shape and wave.  Included by the single-array kernels (xcorr_mfma4.hip) and
// the batched persistent kernel (xcorr_batch.hip).
#pragma once
#include "xc_mfma.h"

namespace xc {
namespace {

// ---------------------------------------------------------------------------
// 4+4-bit int8-MFMA path.
//
// Per channel the packed voltages form a matrix X[i][t] (one byte per sample).
// With R = 16*re and Im16 = 16*im as int8 (a nibble moved to the high half of
// a byte is 16x its value, exact), the four real products
//     RR = R R^T, II = Im16 Im16^T, IR = Im16 R^T, RI = R Im16^T
// give 256*Re V = RR + II and 256*Im V = IR - RI on every 32x32 tile.  Each
// of the four waves of a work-group computes one of the four products for
// every tile of its region, so the waves carry identical MFMA counts for any
// region shape.  Raw packed bytes are staged in LDS in their HBM order
// [t][inputs]; ds_read_b64_tr_b8 turns 8 time rows x 16 inputs into the
// per-lane [input][8 samples] MFMA operand layout, and two masks unpack it.
//
// v_mfma_i32_32x32x32_i8 operand layout (gfx950): lane l supplies row l%32,
// k-half l/32, 16 int8; result register r of lane l is row 8(r/4) + 4(l/32) +
// r%4, column l%32.

// Two transposing 8-byte reads, 8 time rows apart: the lane's 16 samples of
// one input.  `p` is an LDS address; the row offsets fold into the
// instructions' immediate offsets.
template <int EIGHT_ROWS>
__device__ __forceinline__ v4i frag_tr8(lds_u8 *p)
{
    const v2i lo = __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_v2i *)p);
    const v2i hi = __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_v2i *)(p + EIGHT_ROWS));
    return v4i{lo.x, lo.y, hi.x, hi.y};
}

// Wave roles: which real product a wave accumulates.  A role fixes the nibble
// of its row (A) and column (B) operands: 0 = real part, 4 = imaginary part.
enum Role { kRR = 0, kII = 1, kIR = 2, kRI = 3 };
constexpr int role_shift_a(int role) { return (role == kII || role == kIR) ? 4 : 0; }
constexpr int role_shift_b(int role) { return (role == kII || role == kRI) ? 4 : 0; }

// A nibble moved into the high half of a byte reads as 16x its value: the
// real part is x & 0xF0, the imaginary part (x << 4) & 0xF0, both exact int8.
__device__ __forceinline__ v4i re16(v4i x) { return x & (int)0xF0F0F0F0; }
__device__ __forceinline__ v4i im16(v4i x) { return (x << 4) & (int)0xF0F0F0F0; }

// LDS layout of one staged chunk: KC time rows of 256 bytes, i.e. 16 units of
// 16 bytes.  Unit p of a row holds inputs 16p..16p+15 of the region (units
// 0..2D-1: row blocks, 2D..4D-1: column blocks of a rectangle).  Unit p of row
// r is stored at position p ^ ((r & 7) << 1), so that the 8 rows x 2 units a
// transpose-read of two 16-lane groups touches fall on 16 distinct positions
// (64 distinct banks).
constexpr int kRowBytes = 256;

// One 32-sample K step of one wave: read each LDS block the wave's tiles
// touch once (two transpose reads), unpack the nibble(s) its role needs, and
// issue its tiles' MFMAs.  addr[b] = this lane's LDS address of block b in the
// current chunk; KOFF = the K step's row offset.
template <int D, bool TRI, int ROLE, int HALF, int KOFF>
__device__ __forceinline__ void k_step(lds_u8 *const *addr, v16i *acc)
{
    constexpr int NB = TRI ? D : 2 * D;
    constexpr int T0 = half_begin(D, TRI, HALF), T1 = half_end(D, TRI, HALF);
    constexpr int SA = role_shift_a(ROLE), SB = role_shift_b(ROLE);
    v4i A[NB], B[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const bool ua = half_uses_row(D, TRI, HALF, b), ub = half_uses_col(D, TRI, HALF, b);
        if (ua || ub) {
            const v4i x = frag_tr8<8 * kRowBytes>(addr[b] + KOFF);
            if (ua)
                A[b] = SA ? im16(x) : re16(x);
            if (ub)
                B[b] = (ua && SA == SB) ? A[b] : (SB ? im16(x) : re16(x));
        }
    }
#pragma unroll
    for (int t = T0; t < T1; ++t)
        acc[t - T0] = mfma_i8(A[row_block(D, TRI, t)], B[col_block(D, TRI, t)], acc[t - T0]);
}



// Occupancy plan: regions of D <= 3 blocks fit 128 registers per wave, so two
// work-groups share a CU (their barriers are independent, which hides LDS
// latency); larger regions take the CU alone.  LDS per work-group holds the
// ring of NBUF packed chunks; after the main loop it is reused as the
// epilogue stage of G tiles x 4 products x 4 KB.
constexpr int mfma4_wgs_per_cu(int D) { return D <= 3 ? 2 : 1; }
constexpr int mfma4_nbuf(int D, int KC) { return D <= 3 ? 4 : (KC == 64 ? 6 : 3); }
constexpr int mfma4_epilogue_tiles(int D) { return D <= 3 ? 4 : 7; }
constexpr int mfma4_smem_bytes(int D, int KC)
{
    return mfma4_nbuf(D, KC) * KC * kRowBytes > mfma4_epilogue_tiles(D) * 16384
               ? mfma4_nbuf(D, KC) * KC * kRowBytes
               : mfma4_epilogue_tiles(D) * 16384;
}

// Whole work-group body for one region shape and one wave (role, half).
// row_blk / col_blk: first 32-input block of the region's rows / columns.
//
// VEC = 1 (N a multiple of 16, 16-byte aligned input): chunks of KC time rows
// go HBM -> LDS by buffer_load_dwordx4 ... lds into a ring of NBUF buffers,
// NBUF-1 chunks ahead of the MFMAs; the buffer descriptor of each chunk ends at
// the last valid time row, and inputs >= N use an out-of-range offset, so the
// hardware supplies the zero padding.  VEC = 0: each chunk is staged through
// registers, with byte loads for the ragged row end.
template <int D, bool TRI, int KC, int NBUF, int VEC, int ROLE, int HALF>
__device__ __forceinline__ void mfma4_region(uint8_t *smem, const uint8_t *__restrict__ volts,
                                             int64_t T, int F, int N, int f, int row_blk, int col_blk,
                                             int2 *__restrict__ acc_out, int accumulate)
{
    constexpr int NT = n_tiles(D, TRI);
    constexpr int T0 = half_begin(D, TRI, HALF), T1 = half_end(D, TRI, HALF);
    constexpr int NB = TRI ? D : 2 * D;                 // 32-input blocks staged per row
    constexpr int BUF = KC * kRowBytes;
    constexpr int LOADS = KC * 16 / kMfmaThreads;       // 16-byte units per thread per chunk
    constexpr int G = mfma4_epilogue_tiles(D);          // tiles per epilogue round
    static_assert(LOADS * kMfmaThreads == KC * 16, "chunk must be a whole number of wave loads");

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int g = lane >> 4, q = lane & 15;
    lds_u8 *const ring = (lds_u8 *)smem;

    // operand read offsets: row (g>>1)*16 + q>>1 of the K step, unit 2b + (g&1)
    const int row_off = ((g >> 1) * 16 + (q >> 1)) * kRowBytes + (q & 1) * 8;
    int colo[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
        colo[b] = ((2 * b + (g & 1)) ^ (q & 14)) << 4;

    // fill slots: unit U = (wave*LOADS + k)*64 + lane -> row U/16, position U%16
    const int64_t row_bytes = (int64_t)F * N;
    int voff[LOADS];
#pragma unroll
    for (int k = 0; k < LOADS; ++k) {
        const int U = (wave * LOADS + k) * 64 + lane;
        const int r = U >> 4;
        const int p = (U & 15) ^ ((r & 7) << 1);
        const int i0 = p < 2 * D ? row_blk * 32 + 16 * p : col_blk * 32 + 16 * (p - 2 * D);
        const bool valid = p < 2 * NB && i0 < N;
        voff[k] = valid ? (int)(r * row_bytes + (int64_t)f * N + i0) : kBufferOutOfRange;
    }

    v16i acc[T1 > T0 ? T1 - T0 : 1];   // a half may own no tile (D = 1)
#pragma unroll
    for (int t = 0; t < (T1 > T0 ? T1 - T0 : 1); ++t)
        acc[t] = v16i{};

    const int nchunks = (int)((T + KC - 1) / KC);
    auto issue = [&](int c, int bufi) {
        const int64_t rows = min((int64_t)KC, T - (int64_t)c * KC);
        __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(volts + (int64_t)c * KC * row_bytes), (short)0, (int)(rows * row_bytes), 0x00020000);
        lds_u8 *dst = ring + bufi * BUF + wave * LOADS * 1024;
#pragma unroll
        for (int k = 0; k < LOADS; ++k)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (__attribute__((address_space(3))) void *)(dst + k * 1024),
                                                     16, voff[k], 0, 0, kStreamLoadPolicy);
    };
    auto fill_sync = [&](int c, int bufi) {
        lds_u8 *dst = ring + bufi * BUF;
#pragma unroll
        for (int k = 0; k < LOADS; ++k) {
            const int U = (wave * LOADS + k) * 64 + lane;
            const int r = U >> 4;
            const int p = (U & 15) ^ ((r & 7) << 1);
            const int i0 = p < 2 * D ? row_blk * 32 + 16 * p : col_blk * 32 + 16 * (p - 2 * D);
            const v4i val = p < 2 * NB ? load_piece(volts, (int64_t)c * KC + r, T, f, F, N, i0, 1, 0)
                                       : v4i{0, 0, 0, 0};
            *(__attribute__((address_space(3))) v4i *)(dst + U * 16) = val;
        }
    };

    if constexpr (VEC) {
#pragma unroll
        for (int c = 0; c < NBUF - 1; ++c)
            if (c < nchunks)
                issue(c, c);
    }
    int bufc = 0;                 // ring slot of chunk c
    for (int c = 0; c < nchunks; ++c) {
        if constexpr (VEC) {
            if (c + NBUF - 2 < nchunks)
                wait_vmcnt<LOADS * (NBUF - 2)>();
            else
                wait_vmcnt<0>();
            barrier_no_fence();   // chunk c is in LDS; every wave is done with chunk c-1
            if (c + NBUF - 1 < nchunks)
                issue(c + NBUF - 1, bufc == 0 ? NBUF - 1 : bufc - 1);   // the slot chunk c-1 used
        } else {
            __syncthreads();      // every wave is done with the slot being refilled
            fill_sync(c, bufc);
            __syncthreads();
        }
        lds_u8 *addr[NB];
        lds_u8 *const cb = ring + bufc * BUF + row_off;
#pragma unroll
        for (int b = 0; b < NB; ++b)
            addr[b] = cb + colo[b];
#pragma unroll
        for (int ks = 0; ks < KC / 32; ++ks) {
            if (ks == 0)
                k_step<D, TRI, ROLE, HALF, 0>(addr, acc);
            else if (ks == 1)
                k_step<D, TRI, ROLE, HALF, 32 * kRowBytes>(addr, acc);
            else if (ks == 2)
                k_step<D, TRI, ROLE, HALF, 64 * kRowBytes>(addr, acc);
            else
                k_step<D, TRI, ROLE, HALF, 96 * kRowBytes>(addr, acc);
        }
        bufc = bufc + 1 == NBUF ? 0 : bufc + 1;
    }
    __syncthreads();              // every wave is done with the ring

    // Epilogue: the four roles' products of each tile meet in LDS, G tiles per
    // round; 256*Re = RR + II and 256*Im = IR - RI (each a multiple of 256).
    // Stage layout per (role, tile): [quad rq][lane][4] int32, so that a lane
    // writes its registers 4..4rq+3 as one 16-byte store; result register r of
    // lane l is row 8(r/4) + 4(l/32) + r%4, column l%32 of the tile.
    typedef __attribute__((address_space(3))) v4i lds_v4i;
    lds_v4i *const stage = (lds_v4i *)smem;
    const int64_t P = (int64_t)N * (N + 1) / 2;
    int2 *const out_f = acc_out + (int64_t)f * P;
#pragma unroll
    for (int t0 = 0; t0 < NT; t0 += G) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int t = t0 + u;
            if (t >= T0 && t < T1) {
#pragma unroll
                for (int rq = 0; rq < 4; ++rq)
                    stage[((ROLE * G + u) * 4 + rq) * 64 + lane] =
                        v4i{acc[t - T0][4 * rq], acc[t - T0][4 * rq + 1], acc[t - T0][4 * rq + 2],
                            acc[t - T0][4 * rq + 3]};
            }
        }
        __syncthreads();
        const int NQ = (NT - t0 < G ? NT - t0 : G) * 256;   // (tile, rq, lane) quads this round
#pragma unroll
        for (int qq = tid; qq < NQ; qq += kMfmaThreads) {
            const int u = qq >> 8, rq = (qq >> 6) & 3, ln = qq & 63;
            const int t = t0 + u;
            const int I = TRI ? tri_I_rt(t) : t / D;
            const int J = TRI ? tri_J_rt(t) : t % D;
            const int i0 = (row_blk + I) * 32 + 8 * rq + 4 * (ln >> 5);
            const int j = (col_blk + J) * 32 + (ln & 31);
            const int e = (u * 4 + rq) * 64 + ln;
            const v4i rr = stage[(kRR * G * 4) * 64 + e];
            const v4i ii = stage[(kII * G * 4) * 64 + e];
            const v4i ir = stage[(kIR * G * 4) * 64 + e];
            const v4i ri = stage[(kRI * G * 4) * 64 + e];
            int64_t p = (int64_t)i0 * (i0 + 1) / 2 + j;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int i = i0 + m;
                if (i < N && j <= i) {
                    int re = (rr[m] >> 8) + (ii[m] >> 8);
                    int im = (ir[m] >> 8) - (ri[m] >> 8);
                    if (accumulate) {
                        const int2 o = out_f[p];
                        re += o.x;
                        im += o.y;
                    }
                    out_f[p] = make_int2(re, im);
                }
                p += i + 1;
            }
        }
        __syncthreads();
    }
}

template <int D, bool TRI, int KC, int NBUF, int VEC>
__device__ __forceinline__ void mfma4_dispatch(uint8_t *smem, const uint8_t *__restrict__ volts,
                                               int64_t T, int F, int N, int f, int row_blk, int col_blk,
                                               int2 *__restrict__ acc_out, int accumulate)
{
    // each wave runs one complete specialised body; all bodies execute the
    // same sequence of work-group barriers
    switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
#define XC_CASE(W)                                                                                  \
    case W:                                                                                         \
        mfma4_region<D, TRI, KC, NBUF, VEC, ((W) & 3), ((W) >> 2)>(smem, volts, T, F, N, f, row_blk,   \
                                                                 col_blk, acc_out, accumulate);    \
        break;
        XC_CASE(0) XC_CASE(1) XC_CASE(2) XC_CASE(3) XC_CASE(4) XC_CASE(5) XC_CASE(6) XC_CASE(7)
#undef XC_CASE
    default: break;
    }
}


// ---------------------------------------------------------------------------
// Fused-product variant.  Re and Im each take one accumulator per tile:
//     C_re += R_i R_j^T  then  C_re += I_i I_j^T          (= 256 Re)
//     C_im += I_i R_j^T  then  C_im += R_i (~I_j)^T       (= 256 Im - 16 S_i)
// with ~I = -I - 1 (a bitwise NOT of 16*im, exact in int8) and S_i the sum of
// re_i over the samples, taken with v_dot4 on the R operand and added back in
// the epilogue.  Eight waves = product (Re, Im) x K parity x tile half, so a
// wave reads each operand block once per 32-sample K step and feeds it to
// twice as many MFMAs as in the per-role layout above: half the LDS transpose
// reads per MFMA.  The two parities' partial sums are descaled separately
// (each partial is a multiple of 256 once its row-sum term is added), so no
// int32 sum exceeds the bound: per parity |partial| <= 32896 per sample.

constexpr int fused_role(int prod, int par) { return prod + 2 * par; }
// tiles per epilogue round: the stage (4 roles x G x 4 KB plus the row sums)
// fits the ring for D <= 3 (two work-groups per CU); for D >= 4 it takes
// 131 KB, more than the ring, so that D = 6's 21 tiles need three rounds
constexpr int fused_epilogue_tiles(int D) { return D <= 3 ? 3 : 8; }
// ring depth (64-row chunks of 16 KB): as deep as LDS allows, one work-group
// per CU for D >= 4, two for D <= 3
constexpr int fused_nbuf(int D) { return D <= 3 ? 4 : 8; }
constexpr int fused_smem_bytes(int D)
{
    return fused_nbuf(D) * 64 * kRowBytes > fused_epilogue_tiles(D) * 16384 + 2 * D * 256
               ? fused_nbuf(D) * 64 * kRowBytes
               : fused_epilogue_tiles(D) * 16384 + 2 * D * 256;
}

// Does half HALF compute the row sums of row block I (the half owning the
// first tile of row I)?
constexpr bool owns_rowsum(int D, bool tri, int half, int I)
{
    const int t = tri ? I * (I + 1) / 2 : I * D;
    return (t >= half_begin(D, tri, half)) && (t < half_end(D, tri, half));
}

template <int D, bool TRI, int PROD, int HALF, int KOFF>
__device__ __forceinline__ void k_step_fused(lds_u8 *const *addr, v16i *acc, int *rsum)
{
    constexpr int NB = TRI ? D : 2 * D;
    constexpr int T0 = half_begin(D, TRI, HALF), T1 = half_end(D, TRI, HALF);
    v4i A0[NB], B0[NB], A1[NB], B1[NB];   // operands of the first and second product
    static_for<0, NB>([&](auto bc) {
        constexpr int b = bc;
        constexpr bool ua = half_uses_row(D, TRI, HALF, b), ub = half_uses_col(D, TRI, HALF, b);
        if constexpr (ua || ub) {
            const v4i x = frag_tr8<8 * kRowBytes>(addr[b] + KOFF);
            const v4i r = re16(x), i = im16(x);
            if constexpr (PROD == 0) {
                A0[b] = r;   // R_i R_j^T
                B0[b] = r;
                A1[b] = i;   // I_i I_j^T
                B1[b] = i;
            } else {
                if constexpr (ua) {
                    A0[b] = i;   // I_i R_j^T
                    A1[b] = r;   // R_i (~I_j)^T
                    if constexpr (b < D && owns_rowsum(D, TRI, HALF, b))
                        for (int k = 0; k < 4; ++k)
                            rsum[b] = __builtin_amdgcn_sdot4(r[k], 0x01010101, rsum[b], false);
                }
                if constexpr (ub) {
                    B0[b] = r;
                    B1[b] = ~i;
                }
            }
        }
    });
    // all first products, then all second ones: consecutive MFMAs never
    // depend on each other's accumulator
    static_for<T0, T1>([&](auto tc) {
        constexpr int t = tc;
        acc[t - T0] = mfma_i8(A0[row_block(D, TRI, t)], B0[col_block(D, TRI, t)], acc[t - T0]);
    });
    static_for<T0, T1>([&](auto tc) {
        constexpr int t = tc;
        acc[t - T0] = mfma_i8(A1[row_block(D, TRI, t)], B1[col_block(D, TRI, t)], acc[t - T0]);
    });
}

// MB = 1: the chunks come from a table of caller blocks (bt), T = all blocks'
// samples; MB = 0: from one contiguous input (volts).
// accumulate = 1 adds the sums found at acc_in (acc_out for an integration in
// progress, or the accumulators when the result goes to a separate buffer).
// ACC: 0 = the launch overwrites, 1 = it accumulates (the running sums are
// loaded in batches), 2 = the `accumulate` argument decides (per element).
// COMPACT: one copy of the K loop and a runtime loop over the epilogue's
// tiles, for the persistent kernel that holds every tile shape (its code
// would otherwise outgrow the instruction cache); the other kernels unroll.
template <int D, bool TRI, int KC, int NBUF, int VEC, int PROD, int PAR, int HALF, int MB = 0, int ACC = 2,
          bool COMPACT = false>
__device__ __forceinline__ void mfma4f_region(uint8_t *smem, const uint8_t *__restrict__ volts,
                                              int64_t T, int F, int N, int f, int row_blk, int col_blk,
                                              int2 *acc_out, const int2 *acc_in, int accumulate,
                                              const BlockTable *bt = nullptr)
{
    static_assert(!MB || (VEC && KC == 64), "block tables feed the LDS-DMA path with 64-row chunks");
    constexpr int T0 = half_begin(D, TRI, HALF), T1 = half_end(D, TRI, HALF);
    constexpr int NB = TRI ? D : 2 * D;
    constexpr int BUF = KC * kRowBytes;
    constexpr int LOADS = KC * 16 / kMfmaThreads;
    constexpr int G = fused_epilogue_tiles(D);
    constexpr int ROLE = fused_role(PROD, PAR);
    static_assert(LOADS * kMfmaThreads == KC * 16, "chunk must be a whole number of wave loads");
    static_assert(KC % 64 == 0, "a chunk holds whole pairs of 32-sample K steps");
    static_assert(4 * G * 4096 + 2 * D * 64 * 4 <= fused_smem_bytes(D), "epilogue stage fits");

    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));   // keep per-lane offsets inside an enclosing item loop
    const int lane = tid & 63;
    constexpr int WAVE = 4 * PROD + 2 * PAR + (HALF ^ PROD);   // the wave that runs this role
    const int g = lane >> 4, q = lane & 15;
    lds_u8 *const ring = (lds_u8 *)smem;

    const int row_off = ((g >> 1) * 16 + (q >> 1)) * kRowBytes + (q & 1) * 8;
    int colo[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
        colo[b] = ((2 * b + (g & 1)) ^ (q & 14)) << 4;

    const int64_t row_bytes = (int64_t)F * N;
    int voff[LOADS];
#pragma unroll
    for (int k = 0; k < LOADS; ++k) {
        const int U = (WAVE * LOADS + k) * 64 + lane;
        const int r = U >> 4;
        const int p = (U & 15) ^ ((r & 7) << 1);
        const int i0 = p < 2 * D ? row_blk * 32 + 16 * p : col_blk * 32 + 16 * (p - 2 * D);
        const bool valid = p < 2 * NB && i0 < N;
        voff[k] = valid ? (int)(r * row_bytes + (int64_t)f * N + i0) : kBufferOutOfRange;
    }

    v16i acc[T1 > T0 ? T1 - T0 : 1];
#pragma unroll
    for (int t = 0; t < (T1 > T0 ? T1 - T0 : 1); ++t)
        acc[t] = v16i{};
    int rsum[D];
#pragma unroll
    for (int b = 0; b < D; ++b)
        rsum[b] = 0;

    const int nchunks = (int)((T + KC - 1) / KC);
    // DMA state of the next chunk to issue, wave-uniform: its source, the
    // input bytes left from there (MB = 0), its block and position in that
    // block (MB = 1).  Chunks are issued strictly in order.
    const int64_t chunk_bytes = KC * row_bytes;
    const uint8_t *nsrc;
    int64_t nleft = 0;
    int nblk = 0, nin = 0;
    if constexpr (MB)
        nsrc = bt->p[0];
    else {
        nsrc = volts;
        nleft = T * row_bytes;
    }
    auto issue_next = [&](int bufi) {
        // block-table chunks are always whole; the input's last may be short
        const int records = MB ? (int)chunk_bytes : (int)(nleft < chunk_bytes ? nleft : chunk_bytes);
        __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc((void *)nsrc, (short)0, records, 0x00020000);
        lds_u8 *dst = ring + bufi * BUF + WAVE * LOADS * 1024;
#pragma unroll
        for (int k = 0; k < LOADS; ++k)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (__attribute__((address_space(3))) void *)(dst + k * 1024),
                                                     16, voff[k], 0, 0, kStreamLoadPolicy);
        nsrc += chunk_bytes;
        if constexpr (MB) {
            if (++nin == bt->chunks_per_block) {
                nin = 0;
                if (++nblk < kMaxFusedBlocks)
                    nsrc = bt->p[nblk];
            }
        } else {
            nleft -= chunk_bytes;
        }
    };
    auto fill_sync = [&](int c, int bufi) {
        lds_u8 *dst = ring + bufi * BUF;
#pragma unroll
        for (int k = 0; k < LOADS; ++k) {
            const int U = (WAVE * LOADS + k) * 64 + lane;
            const int r = U >> 4;
            const int p = (U & 15) ^ ((r & 7) << 1);
            const int i0 = p < 2 * D ? row_blk * 32 + 16 * p : col_blk * 32 + 16 * (p - 2 * D);
            const v4i val = p < 2 * NB ? load_piece(volts, (int64_t)c * KC + r, T, f, F, N, i0, 1, 0)
                                       : v4i{0, 0, 0, 0};
            *(__attribute__((address_space(3))) v4i *)(dst + U * 16) = val;
        }
    };
    auto compute = [&](int bufi) {
        lds_u8 *addr[NB];
        lds_u8 *const cb = ring + bufi * BUF + row_off;
#pragma unroll
        for (int b = 0; b < NB; ++b)
            addr[b] = cb + colo[b];
        // 32-sample K steps of this chunk: this wave takes those of its parity
        static_for<0, KC / 64>([&](auto kc) {
            k_step_fused<D, TRI, PROD, HALF, (2 * kc + PAR) * 32 * kRowBytes>(addr, acc, rsum);
        });
    };

    int bufc = 0;
    if constexpr (VEC) {
#pragma unroll
        for (int c = 0; c < NBUF - 1; ++c)
            if (c < nchunks)
                issue_next(c);
        if constexpr (COMPACT) {
            for (int c = 0; c < nchunks; ++c) {
                const int after = nchunks - 1 - c;   // chunks issued after chunk c, at most
                if (after >= NBUF - 2)
                    wait_vmcnt<LOADS * (NBUF - 2)>();
                else
                    wait_vmcnt_chunks<LOADS, NBUF - 3>(after);
                barrier_no_fence();
                if (after >= NBUF - 1)
                    issue_next(bufc == 0 ? NBUF - 1 : bufc - 1);
                compute(bufc);
                bufc = bufc + 1 == NBUF ? 0 : bufc + 1;
            }
        } else {
            int c = 0;
            // steady state: chunk c is complete when this wave has at most the
            // NBUF - 2 chunks issued after it outstanding; then chunk c + NBUF - 1
            // goes into the slot the previous iteration read
            for (; c + NBUF - 1 < nchunks; ++c) {
                wait_vmcnt<LOADS * (NBUF - 2)>();
                barrier_no_fence();
                issue_next(bufc == 0 ? NBUF - 1 : bufc - 1);
                compute(bufc);
                bufc = bufc + 1 == NBUF ? 0 : bufc + 1;
            }
            // tail: everything is issued; nchunks - 1 - c chunks follow chunk c
            for (; c < nchunks; ++c) {
                wait_vmcnt_chunks<LOADS, NBUF - 2>(nchunks - 1 - c);
                barrier_no_fence();
                compute(bufc);
                bufc = bufc + 1 == NBUF ? 0 : bufc + 1;
            }
        }
    } else {
        for (int c = 0; c < nchunks; ++c) {
            __syncthreads();
            fill_sync(c, bufc);
            __syncthreads();
            compute(bufc);
            bufc = bufc + 1 == NBUF ? 0 : bufc + 1;
        }
    }
    __syncthreads();

    // Epilogue, in rounds of G tiles: stage [role = (product, parity)][slot]
    // [rq][lane] v4i and the row sums [parity][row block][64 lanes]; then each
    // thread adds the four roles of its quads (rows i0..i0+3 of one column),
    // descales each parity separately and stores.  A wave's quads are known at
    // compile time: slots u = PROD, PROD + 2, ... of the round, row quad
    // rq = 2 PAR + (HALF ^ PROD), which is the wave's index mod 4.
    typedef __attribute__((address_space(3))) v4i lds_v4i;
    lds_v4i *const stage = (lds_v4i *)smem;
    int *const sstage = (int *)(smem + 4 * G * 4096);
    // lane offsets of the epilogue, from an opaque copy of the thread index so
    // that none of them is computed before the K loop and held across it
    int etid = threadIdx.x;
    asm volatile("" : "+v"(etid));
    const int elane = etid & 63;
    if constexpr (PROD == 1) {
        static_for<0, D>([&](auto bc) {
            if constexpr (owns_rowsum(D, TRI, HALF, bc))
                sstage[(PAR * D + bc) * 64 + elane] = rsum[bc];
        });
    }
    constexpr int RQ = 2 * PAR + (HALF ^ PROD);
    constexpr int KQ = (G + 1) / 2;
    const int64_t P = (int64_t)N * (N + 1) / 2;
    int2 *const out_f = acc_out + (int64_t)f * P;
    const int2 *const in_f = acc_in + (int64_t)f * P;
    const int il0 = 8 * RQ + 4 * (elane >> 5);   // first row of the quad within its 32-row block
    const int jl = elane & 31;
    if constexpr (COMPACT) {
        // G tiles per round, in order
        constexpr int NT = n_tiles(D, TRI);
#pragma unroll 1
        for (int t0 = 0; t0 < NT; t0 += G) {
            static_for<T0, T1>([&](auto tc) {
                constexpr int t = tc;
                const int u = t - t0;
                if (u >= 0 && u < G) {
                    static_for<0, 4>([&](auto rqc) {
                        constexpr int rq = rqc;
                        stage[((ROLE * G + u) * 4 + rq) * 64 + elane] =
                            v4i{acc[t - T0][4 * rq], acc[t - T0][4 * rq + 1], acc[t - T0][4 * rq + 2],
                                acc[t - T0][4 * rq + 3]};
                    });
                }
            });
            __syncthreads();
            const int NQ = (NT - t0 < G ? NT - t0 : G) * 256;   // (tile, rq, lane) quads this round
#pragma unroll 1
            for (int qq = etid; qq < NQ; qq += kMfmaThreads) {
                const int u = qq >> 8, rq = (qq >> 6) & 3, ln = qq & 63;
                const int t = t0 + u;
                const int I = TRI ? tri_I_rt(t) : t / D;
                const int J = TRI ? tri_J_rt(t) : t % D;
                const int ql0 = 8 * rq + 4 * (ln >> 5);
                const int i0 = (row_blk + I) * 32 + ql0;
                const int j = (col_blk + J) * 32 + (ln & 31);
                const int e = (u * 4 + rq) * 64 + ln;
                const v4i re0 = stage[(fused_role(0, 0) * G * 4) * 64 + e];
                const v4i re1 = stage[(fused_role(0, 1) * G * 4) * 64 + e];
                const v4i im0 = stage[(fused_role(1, 0) * G * 4) * 64 + e];
                const v4i im1 = stage[(fused_role(1, 1) * G * 4) * 64 + e];
                const lds_v4i *const rs = (const lds_v4i *)(sstage + I * 64 + ql0);
                const v4i s0 = rs[0] + rs[8];
                const v4i s1 = rs[D * 16] + rs[D * 16 + 8];
                int p = i0 * (i0 + 1) / 2 + j;
                // the quad's running sums, all requested before its stores
                int2 oq[4] = {};
                if constexpr (ACC != 0)
                    if (ACC == 1 || accumulate)
                        quad_running_sums(in_f, p, i0, j, true, N, oq);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int i = i0 + m;
                    if (i < N && j <= i) {
                        const int re = (re0[m] >> 8) + (re1[m] >> 8);
                        const int im = ((im0[m] + s0[m]) >> 8) + ((im1[m] + s1[m]) >> 8);
                        out_f[p] = make_int2(re + oq[m].x, im + oq[m].y);
                    }
                    p += i + 1;
                }
            }
            if (t0 + G < NT)
                __syncthreads();
        }
        return;
    }
    static_for<0, epilogue_rounds(D, TRI, G)>([&](auto rc) {
        static_for<0, G>([&](auto uc) {
            constexpr int u = uc;
            constexpr int t = epilogue_slot_tile(D, TRI, G, rc, u);
            if constexpr (t >= T0 && t < T1) {
                static_for<0, 4>([&](auto rqc) {
                    constexpr int rq = rqc;
                    stage[((ROLE * G + u) * 4 + rq) * 64 + elane] =
                        v4i{acc[t - T0][4 * rq], acc[t - T0][4 * rq + 1], acc[t - T0][4 * rq + 2],
                            acc[t - T0][4 * rq + 3]};
                });
            }
        });
        __syncthreads();
        // running sums of every quad of this thread, loaded before any store
        // (from a valid address where the pair does not exist)
        int2 old[ACC == 1 && D > 3 ? KQ : 1][4];
        if constexpr (ACC == 1 && D > 3) {
            static_for<0, KQ>([&](auto kc) {
                constexpr int u = PROD + 2 * kc;
                constexpr int t = u < G ? epilogue_slot_tile(D, TRI, G, rc, u) : -1;
                if constexpr (t >= 0) {
                    constexpr int I = tile_I(D, TRI, t), J = tile_J(D, TRI, t);
                    const int i0 = (row_blk + I) * 32 + il0;
                    const int j = (col_blk + J) * 32 + jl;
                    int p = i0 * (i0 + 1) / 2 + j;
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int i = i0 + m;
                        const bool ok = i < N && (!(TRI && I == J) || j <= i);
                        old[kc][m] = in_f[ok ? p : 0];
                        p += i + 1;
                    }
                }
            });
        }
        static_for<0, KQ>([&](auto kc) {
            constexpr int u = PROD + 2 * kc;
            constexpr int t = u < G ? epilogue_slot_tile(D, TRI, G, rc, u) : -1;
            if constexpr (t >= 0) {
                constexpr int I = tile_I(D, TRI, t), J = tile_J(D, TRI, t);
                constexpr bool diag = TRI && I == J;
                const int i0 = (row_blk + I) * 32 + il0;
                const int j = (col_blk + J) * 32 + jl;
                const int e = (u * 4 + RQ) * 64 + elane;
                const v4i re0 = stage[(fused_role(0, 0) * G * 4) * 64 + e];
                const v4i re1 = stage[(fused_role(0, 1) * G * 4) * 64 + e];
                const v4i im0 = stage[(fused_role(1, 0) * G * 4) * 64 + e];
                const v4i im1 = stage[(fused_role(1, 1) * G * 4) * 64 + e];
                // row sums of rows i0..i0+3, both K halves, per parity
                const lds_v4i *const rs = (const lds_v4i *)(sstage + I * 64 + il0);
                const v4i s0 = rs[0] + rs[8];
                const v4i s1 = rs[D * 16] + rs[D * 16 + 8];
                int p = i0 * (i0 + 1) / 2 + j;
                // otherwise the quad's running sums, requested before its stores
                int2 oq[4] = {};
                if constexpr (ACC != 0 && !(ACC == 1 && D > 3))
                    if (ACC == 1 || accumulate)
                        quad_running_sums(in_f, p, i0, j, diag, N, oq);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int i = i0 + m;
                    if (i < N && (!diag || j <= i)) {
                        const int re = (re0[m] >> 8) + (re1[m] >> 8);
                        const int im = ((im0[m] + s0[m]) >> 8) + ((im1[m] + s1[m]) >> 8);
                        int2 o = oq[m];
                        if constexpr (ACC == 1 && D > 3)
                            o = old[kc][m];
                        out_f[p] = make_int2(re + o.x, im + o.y);
                    }
                    p += i + 1;
                }
                // one quad at a time: hoisting the next quad's LDS reads
                // above these stores would need registers the accumulators
                // of later rounds still hold
                __builtin_amdgcn_sched_barrier(0);
            }
        });
        // the next round overwrites the stage; after the last one the caller
        // synchronises before it reuses LDS
        if constexpr (rc + 1 < epilogue_rounds(D, TRI, G))
            __syncthreads();
    });
}

template <int D, bool TRI, int KC, int NBUF, int VEC, int MB = 0, int ACC = 2, bool COMPACT = false>
__device__ __forceinline__ void mfma4f_dispatch(uint8_t *smem, const uint8_t *__restrict__ volts,
                                                int64_t T, int F, int N, int f, int row_blk, int col_blk,
                                                int2 *acc_out, const int2 *acc_in, int accumulate,
                                                const BlockTable *bt = nullptr)
{
    switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
#define XC_CASE(W)                                                                                     \
    case W:                                                                                            \
        mfma4f_region<D, TRI, KC, NBUF, VEC, ((W) >> 2), (((W) >> 1) & 1), (((W) & 1) ^ ((W) >> 2)), MB, ACC, \
                      COMPACT>(                                                                         \
            smem, volts, T, F, N, f, row_blk, col_blk, acc_out, acc_in, accumulate, bt);               \
        break;
        XC_CASE(0) XC_CASE(1) XC_CASE(2) XC_CASE(3) XC_CASE(4) XC_CASE(5) XC_CASE(6) XC_CASE(7)
#undef XC_CASE
    default: break;
    }
}


}  // namespace
}  // namespace xc
