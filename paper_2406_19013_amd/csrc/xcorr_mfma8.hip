// 8+8-bit int8 / FP16 MFMA kernels of the X-engine for one diagonal block
// size D (compiled once per D with -DXC_D=1..6; each object exports
// launch_mfma8_d<D>).
#include "xc_mfma.h"

#include <type_traits>

#ifndef XC_D
#error "compile with -DXC_D=<diagonal block size>"
#endif

namespace xc {
namespace {

// 8+8-bit paths: int8 MFMA with exact int32 accumulation, or FP16 MFMA with
// FP32 accumulation.
//
// Samples are (re, im) int8 pairs.  With X = [re, im] interleaved along K, one
// product X_i X_j^T gives Re V directly.  For Im the column operand is
// X'_j = [~im_j, re_j] (swap the bytes of each pair, invert the first):
// X_i X'_j^T = sum re_i (-im_j - 1) + im_i re_j = Im V - S_i with
// S_i = sum_t re_i[t], added back in the epilogue (int8 path).  The FP16 path
// negates exactly and needs no correction.  Every value is an integer below
// 2^11, so the FP16 operands are exact; FP32 accumulation rounds only once a
// partial sum passes 2^24.
//
// Eight waves per work-group: product (Re, Im) x K parity x tile half.  Wave w
// sits on SIMD w mod 4 = (product, parity), so each SIMD carries one product
// over every other 16-sample K step for all tiles of the region.
//
// LDS: time rows of 512 bytes = 32 units of 16 bytes (unit p = inputs
// 8p..8p+7 of the region's staged blocks, 4 units per 32-input block); unit p
// of row r is stored at position p ^ ((r & 3) << 2).  ds_read_b64_tr_b16
// (lanes 4j..4j+3 supply the quarters of row j of a 4 x 16-element tile, lane
// q receives column q) delivers one input's 4 consecutive (re, im) samples.

constexpr int kRow8 = 512;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v4s lds_v4s;
typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef _Float16 v2h __attribute__((ext_vector_type(2)));

__device__ __forceinline__ v2i tr16(lds_u8 *p)
{
    const v4s x = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s *)p);
    return __builtin_bit_cast(v2i, x);
}

// [re, im] pair bytes -> [~im, re] (column operand of the Im product)
__device__ __forceinline__ int swap_not(int x)
{
    return (int)__builtin_amdgcn_perm((unsigned)x, (unsigned)x, 0x02030001u) ^ 0x00FF00FF;
}

// two int8 (re, im) pairs (one dword) -> two half2 (re, im), exact
__device__ __forceinline__ void pairs_to_f16(int x, int &h0, int &h1)
{
    const unsigned t = (unsigned)x ^ 0x80808080u;               // b + 128
    const unsigned a = __builtin_amdgcn_perm(0x64646464u, t, 0x04010400u);
    const unsigned b = __builtin_amdgcn_perm(0x64646464u, t, 0x04030402u);
    const v2h off = {(_Float16)-1152.0f, (_Float16)-1152.0f};  // 1024 + 128
    h0 = __builtin_bit_cast(int, __builtin_bit_cast(v2h, a) + off);
    h1 = __builtin_bit_cast(int, __builtin_bit_cast(v2h, b) + off);
}

// half2 (re, im) -> (-im, re)
__device__ __forceinline__ int neg_swap_f16(int h)
{
    return (int)__builtin_amdgcn_alignbit((unsigned)h, (unsigned)h, 16) ^ 0x00008000;
}

constexpr int role8(int prod, int par) { return prod + 2 * par; }

// Does half HALF compute the row sums of row block I (the half owning the
// first tile of row I)?
constexpr bool half_owns_rowsum(int D, bool tri, int half, int I)
{
    const int t = tri ? I * (I + 1) / 2 : I * D;
    return (t >= half_begin(D, tri, half)) && (t < half_end(D, tri, half));
}

template <int D, bool TRI, bool F16, int PROD, int HALF, int KOFF>
__device__ __forceinline__ void k_step8(lds_u8 *const *addr, typename std::conditional<F16, v16f, v16i>::type *acc,
                                        int *rsum)
{
    constexpr int NB = TRI ? D : 2 * D;
    constexpr int T0 = half_begin(D, TRI, HALF), T1 = half_end(D, TRI, HALF);
    if constexpr (!F16) {
        v4i A[NB], B[NB];
        static_for<0, NB>([&](auto bc) {
            constexpr int b = bc;
            constexpr bool ua = half_uses_row(D, TRI, HALF, b), ub = half_uses_col(D, TRI, HALF, b);
            if constexpr (ua || ub) {
                const v2i lo = tr16(addr[b] + KOFF);
                const v2i hi = tr16(addr[b] + KOFF + 4 * kRow8);
                const v4i x = v4i{lo.x, lo.y, hi.x, hi.y};
                if constexpr (ua) {
                    A[b] = x;
                    if constexpr (PROD == 1 && b < D && half_owns_rowsum(D, TRI, HALF, b))
                        for (int k = 0; k < 4; ++k)
                            rsum[b] = __builtin_amdgcn_sdot4(x[k], 0x00010001, rsum[b], false);
                }
                if constexpr (ub) {
                    if constexpr (PROD == 0)
                        B[b] = x;
                    else
                        B[b] = v4i{swap_not(x.x), swap_not(x.y), swap_not(x.z), swap_not(x.w)};
                }
            }
        });
        static_for<T0, T1>([&](auto tc) {
            constexpr int t = tc;
            acc[t - T0] = mfma_i8(A[row_block(D, TRI, t)], B[col_block(D, TRI, t)], acc[t - T0]);
        });
    } else {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            v8h A[NB], B[NB];
            static_for<0, NB>([&](auto bc) {
                constexpr int b = bc;
                constexpr bool ua = half_uses_row(D, TRI, HALF, b), ub = half_uses_col(D, TRI, HALF, b);
                if constexpr (ua || ub) {
                    const v2i x = tr16(addr[b] + KOFF + m * 8 * kRow8);
                    int h[4];
                    pairs_to_f16(x.x, h[0], h[1]);
                    pairs_to_f16(x.y, h[2], h[3]);
                    if constexpr (ua)
                        A[b] = __builtin_bit_cast(v8h, v4i{h[0], h[1], h[2], h[3]});
                    if constexpr (ub) {
                        if constexpr (PROD == 0)
                            B[b] = __builtin_bit_cast(v8h, v4i{h[0], h[1], h[2], h[3]});
                        else
                            B[b] = __builtin_bit_cast(v8h, v4i{neg_swap_f16(h[0]), neg_swap_f16(h[1]),
                                                               neg_swap_f16(h[2]), neg_swap_f16(h[3])});
                    }
                }
            });
            static_for<T0, T1>([&](auto tc) {
                constexpr int t = tc;
                acc[t - T0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A[row_block(D, TRI, t)],
                                                                    B[col_block(D, TRI, t)], acc[t - T0], 0, 0, 0);
            });
        }
    }
}

constexpr int mfma8_nbuf() { return 4; }
// tiles per epilogue round; for D >= 4 the stage (4 roles x 8 tiles x 4 KB
// plus the row sums, 131 KB) is larger than the 128 KB ring
constexpr int mfma8_epilogue_tiles(int D) { return D <= 3 ? 4 : 8; }
constexpr int mfma8_smem_bytes(int KC, int D)
{
    return mfma8_nbuf() * KC * kRow8 > 4 * mfma8_epilogue_tiles(D) * 4096 + 2 * D * 256
               ? mfma8_nbuf() * KC * kRow8
               : 4 * mfma8_epilogue_tiles(D) * 4096 + 2 * D * 256;
}

template <int D, bool TRI, bool F16, int KC, int NBUF, int VEC, int PROD, int PAR, int HALF>
__device__ __forceinline__ void mfma8_region(uint8_t *smem, const uint8_t *__restrict__ volts, int64_t T,
                                             int F, int N, int f, int row_blk, int col_blk,
                                             void *__restrict__ acc_out, int accumulate)
{
    using AccT = typename std::conditional<F16, v16f, v16i>::type;
    constexpr int T0 = half_begin(D, TRI, HALF), T1 = half_end(D, TRI, HALF);
    constexpr int NB = TRI ? D : 2 * D;
    constexpr int BUF = KC * kRow8;
    constexpr int LOADS = KC * 32 / kMfmaThreads;
    constexpr int G = mfma8_epilogue_tiles(D);
    constexpr int ROLE = role8(PROD, PAR);
    static_assert(LOADS * kMfmaThreads == KC * 32, "chunk must be a whole number of wave loads");
    static_assert(KC % 32 == 0, "a chunk holds whole pairs of 16-sample K steps");

    const int lane = threadIdx.x & 63;
    constexpr int WAVE = PROD + 2 * PAR + 4 * HALF;   // the wave that runs this role
    const int g = lane >> 4, q = lane & 15;
    lds_u8 *const ring = (lds_u8 *)smem;

    // operand read offsets (int8: samples 8*(g>>1) + 4c + q>>2 of the K step;
    // FP16: samples 8m + 4*(g>>1) + q>>2), unit 4b + 2(g&1) + ((q>>1)&1)
    const int row_off = (F16 ? ((g >> 1) * 4 + (q >> 2)) : ((g >> 1) * 8 + (q >> 2))) * kRow8 + (q & 1) * 8;
    int colo[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
        colo[b] = ((4 * b + 2 * (g & 1) + ((q >> 1) & 1)) ^ ((q >> 2) << 2)) << 4;

    // fill slots: unit U = (wave*LOADS + k)*64 + lane -> row U/32, position U%32
    const int64_t row_bytes = (int64_t)F * N * 2;
    int voff[LOADS];
#pragma unroll
    for (int k = 0; k < LOADS; ++k) {
        const int U = (WAVE * LOADS + k) * 64 + lane;
        const int r = U >> 5;
        const int p = (U & 31) ^ ((r & 3) << 2);
        const int i0 = p < 4 * D ? row_blk * 32 + 8 * p : col_blk * 32 + 8 * (p - 4 * D);
        const bool valid = p < 4 * NB && i0 < N;
        voff[k] = valid ? (int)(r * row_bytes + ((int64_t)f * N + i0) * 2) : kBufferOutOfRange;
    }

    AccT acc[T1 > T0 ? T1 - T0 : 1];
#pragma unroll
    for (int t = 0; t < (T1 > T0 ? T1 - T0 : 1); ++t)
        acc[t] = AccT{};
    int rsum[D];
#pragma unroll
    for (int b = 0; b < D; ++b)
        rsum[b] = 0;

    const int nchunks = (int)((T + KC - 1) / KC);
    // DMA state of the next chunk to issue (wave-uniform): its source and the
    // input bytes left from there; chunks are issued strictly in order
    const int64_t chunk_bytes = KC * row_bytes;
    const uint8_t *nsrc = volts;
    int64_t nleft = T * row_bytes;
    auto issue_next = [&](int bufi) {
        const int records = (int)(nleft < chunk_bytes ? nleft : chunk_bytes);
        __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc((void *)nsrc, (short)0, records, 0x00020000);
        lds_u8 *dst = ring + bufi * BUF + WAVE * LOADS * 1024;
#pragma unroll
        for (int k = 0; k < LOADS; ++k)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (__attribute__((address_space(3))) void *)(dst + k * 1024),
                                                     16, voff[k], 0, 0, kStreamLoadPolicy);
        nsrc += chunk_bytes;
        nleft -= chunk_bytes;
    };
    auto fill_sync = [&](int c, int bufi) {
        lds_u8 *dst = ring + bufi * BUF;
#pragma unroll
        for (int k = 0; k < LOADS; ++k) {
            const int U = (WAVE * LOADS + k) * 64 + lane;
            const int r = U >> 5;
            const int p = (U & 31) ^ ((r & 3) << 2);
            const int i0 = p < 4 * D ? row_blk * 32 + 8 * p : col_blk * 32 + 8 * (p - 4 * D);
            const v4i val = p < 4 * NB ? load_piece(volts, (int64_t)c * KC + r, T, f, F, N, i0, 2, 0)
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
        // 16-sample K steps of this chunk: this wave takes those of its parity
        k_step8<D, TRI, F16, PROD, HALF, PAR * 16 * kRow8>(addr, acc, rsum);
        if constexpr (KC == 64)
            k_step8<D, TRI, F16, PROD, HALF, (PAR + 2) * 16 * kRow8>(addr, acc, rsum);
    };

    int bufc = 0;
    if constexpr (VEC) {
#pragma unroll
        for (int c = 0; c < NBUF - 1; ++c)
            if (c < nchunks)
                issue_next(c);
        // one loop body (two copies of it cost registers): chunk c is
        // complete when at most the chunks this wave issued after it are
        // outstanding; while chunks remain, chunk c + NBUF - 1 goes into the
        // slot the previous iteration read
        for (int c = 0; c < nchunks; ++c) {
            const int after = nchunks - 1 - c;
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
        for (int c = 0; c < nchunks; ++c) {
            __syncthreads();
            fill_sync(c, bufc);
            __syncthreads();
            compute(bufc);
            bufc = bufc + 1 == NBUF ? 0 : bufc + 1;
        }
    }
    __syncthreads();

    // Epilogue: Re = sum of the two parities' Re products, Im = the two Im
    // products (+ S_i on the int8 path), G tiles per round.  Stage layout as
    // in the 4-bit path; the row sums follow the tile stage.  A wave's quads
    // are known at compile time: slots u = HALF, HALF + 2, ... of the round,
    // row quad rq = PROD + 2 PAR, which is the wave's index mod 4.
    typedef __attribute__((address_space(3))) v4i lds_v4i;
    lds_v4i *const stage = (lds_v4i *)smem;
    int *const sstage = (int *)(smem + 4 * G * 4096);          // [parity][row block][64 lanes]
    // lane offsets of the epilogue, from an opaque copy of the thread index so
    // that none of them is computed before the K loop and held across it
    int etid = threadIdx.x;
    asm volatile("" : "+v"(etid));
    const int elane = etid & 63;
    if constexpr (!F16 && PROD == 1) {
        static_for<0, D>([&](auto bc) {
            if constexpr (half_owns_rowsum(D, TRI, HALF, bc))
                sstage[(PAR * D + bc) * 64 + elane] = rsum[bc];
        });
    }
    constexpr int RQ = PROD + 2 * PAR;
    constexpr int KQ = (G + 1) / 2;
    const int64_t P = (int64_t)N * (N + 1) / 2;
    const int il0 = 8 * RQ + 4 * (elane >> 5);   // first row of the quad within its 32-row block
    const int jl = elane & 31;
    static_for<0, epilogue_rounds(D, TRI, G)>([&](auto rc) {
        static_for<0, G>([&](auto uc) {
            constexpr int u = uc;
            constexpr int t = epilogue_slot_tile(D, TRI, G, rc, u);
            if constexpr (t >= T0 && t < T1) {
                static_for<0, 4>([&](auto rqc) {
                    constexpr int rq = rqc;
                    if constexpr (F16)
                        stage[((ROLE * G + u) * 4 + rq) * 64 + elane] = __builtin_bit_cast(
                            v4i, v4f{acc[t - T0][4 * rq], acc[t - T0][4 * rq + 1], acc[t - T0][4 * rq + 2],
                                     acc[t - T0][4 * rq + 3]});
                    else
                        stage[((ROLE * G + u) * 4 + rq) * 64 + elane] =
                            v4i{acc[t - T0][4 * rq], acc[t - T0][4 * rq + 1], acc[t - T0][4 * rq + 2],
                                acc[t - T0][4 * rq + 3]};
                });
            }
        });
        __syncthreads();
        static_for<0, KQ>([&](auto kc) {
            constexpr int u = HALF + 2 * kc;
            constexpr int t = u < G ? epilogue_slot_tile(D, TRI, G, rc, u) : -1;
            if constexpr (t >= 0) {
                constexpr int I = tile_I(D, TRI, t), J = tile_J(D, TRI, t);
                constexpr bool diag = TRI && I == J;
                const int i0 = (row_blk + I) * 32 + il0;
                const int j = (col_blk + J) * 32 + jl;
                const int e = (u * 4 + RQ) * 64 + elane;
                const v4i re0 = stage[(role8(0, 0) * G * 4) * 64 + e];
                const v4i re1 = stage[(role8(0, 1) * G * 4) * 64 + e];
                const v4i im0 = stage[(role8(1, 0) * G * 4) * 64 + e];
                const v4i im1 = stage[(role8(1, 1) * G * 4) * 64 + e];
                int p = i0 * (i0 + 1) / 2 + j;
                if constexpr (F16) {
                    // whole-vector casts: a bit cast of one subscripted element
                    // is not reliable in this compiler
                    const v4f fr0 = __builtin_bit_cast(v4f, re0), fr1 = __builtin_bit_cast(v4f, re1);
                    const v4f fi0 = __builtin_bit_cast(v4f, im0), fi1 = __builtin_bit_cast(v4f, im1);
                    float2 *const dst = static_cast<float2 *>(acc_out) + (int64_t)f * P;
                    float2 o[4];
                    if (accumulate)
                        quad_running_sums(dst, p, i0, j, diag, N, o);
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int i = i0 + m;
                        if (i < N && (!diag || j <= i)) {
                            float re = fr0[m] + fr1[m];
                            float im = fi0[m] + fi1[m];
                            if (accumulate) {
                                re += o[m].x;
                                im += o[m].y;
                            }
                            dst[p] = make_float2(re, im);
                        }
                        p += i + 1;
                    }
                } else {
                    // rows i0..i0+3: sums of real parts over both parities and K halves
                    const lds_v4i *const rs = (const lds_v4i *)(sstage + I * 64 + il0);
                    const v4i S = rs[0] + rs[8] + rs[D * 16] + rs[D * 16 + 8];
                    int2 *const dst = static_cast<int2 *>(acc_out) + (int64_t)f * P;
                    int2 o[4];
                    if (accumulate)
                        quad_running_sums(dst, p, i0, j, diag, N, o);
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int i = i0 + m;
                        if (i < N && (!diag || j <= i)) {
                            int re = re0[m] + re1[m];
                            int im = im0[m] + im1[m] + S[m];
                            if (accumulate) {
                                re += o[m].x;
                                im += o[m].y;
                            }
                            dst[p] = make_int2(re, im);
                        }
                        p += i + 1;
                    }
                }
                // one quad at a time (registers: later rounds' accumulators)
                __builtin_amdgcn_sched_barrier(0);
            }
        });
        // the next round overwrites the stage; the launch ends after the last
        if constexpr (rc + 1 < epilogue_rounds(D, TRI, G))
            __syncthreads();
    });
}

template <int D, bool TRI, bool F16, int KC, int NBUF, int VEC>
__device__ __forceinline__ void mfma8_dispatch(uint8_t *smem, const uint8_t *__restrict__ volts, int64_t T,
                                               int F, int N, int f, int row_blk, int col_blk,
                                               void *__restrict__ acc_out, int accumulate)
{
    switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
#define XC_CASE8(W)                                                                                     \
    case W:                                                                                             \
        mfma8_region<D, TRI, F16, KC, NBUF, VEC, ((W) & 1), (((W) >> 1) & 1), ((W) >> 2)>(            \
            smem, volts, T, F, N, f, row_blk, col_blk, acc_out, accumulate);                            \
        break;
        XC_CASE8(0) XC_CASE8(1) XC_CASE8(2) XC_CASE8(3) XC_CASE8(4) XC_CASE8(5) XC_CASE8(6) XC_CASE8(7)
#undef XC_CASE8
    default: break;
    }
}

template <int D, bool F16, int KC, int VEC>
__global__ __launch_bounds__(kMfmaThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void xc_mfma8_kernel(const uint8_t *__restrict__ volts, int64_t T, int F, int N, int nseg, int R,
                     int nitems, void *__restrict__ acc_out, int accumulate)
{
    constexpr int NBUF = mfma8_nbuf();
    __shared__ __attribute__((aligned(1024))) uint8_t smem[mfma8_smem_bytes(KC, D)];
    static_assert(4 * mfma8_epilogue_tiles(D) * 4096 + 2 * D * 64 * 4 <= mfma8_smem_bytes(KC, D), "stage fits");

    const int item = xcd_item();
    if (item >= nitems)
        return;
    const int f = item / R;
    const int r = item - f * R;
    if (r < nseg) {
        mfma8_dispatch<D, true, F16, KC, NBUF, VEC>(smem, volts, T, F, N, f, r * D, r * D, acc_out, accumulate);
    } else if constexpr (D <= 4) {
        const int k = r - nseg;
        int a = (int)((1.f + sqrtf(1.f + 8.f * k)) * 0.5f);
        while (a * (a - 1) / 2 > k)
            --a;
        while ((a + 1) * a / 2 <= k)
            ++a;
        const int b = k - a * (a - 1) / 2;
        mfma8_dispatch<D, false, F16, KC, NBUF, VEC>(smem, volts, T, F, N, f, a * D, b * D, acc_out, accumulate);
    }
}

}  // namespace

template <int D, bool F16>
static hipError_t launch_mfma8_t(const Plan &pl, const uint8_t *volts, int64_t T, int F, int N, void *acc,
                                 int accumulate, hipStream_t s)
{
    constexpr int KC = 64;
    const int64_t nitems64 = (int64_t)F * pl.regions;
    if (nitems64 > (1LL << 30))
        return hipErrorInvalidValue;
    const int nitems = (int)nitems64;
    const int vec_ok = (N % 8 == 0) && ((uintptr_t)volts % 16 == 0) &&
                       (int64_t)KC * F * N * 2 < (1LL << 31) - 16;
    auto kern = vec_ok ? xc_mfma8_kernel<D, F16, KC, 1> : xc_mfma8_kernel<D, F16, KC, 0>;
    hipLaunchKernelGGL(kern, dim3(xcd_grid(nitems)), dim3(kMfmaThreads), 0, s, volts, T, F, N, pl.nseg,
                       pl.regions, nitems, acc, accumulate);
    return hipGetLastError();
}

#define XC_CAT2(a, b) a##b
#define XC_CAT(a, b) XC_CAT2(a, b)

hipError_t XC_CAT(launch_mfma8_d, XC_D)(const Plan &pl, bool f16, const uint8_t *volts, int64_t T, int F, int N,
                                        void *acc, int accumulate, hipStream_t s)
{
    return f16 ? launch_mfma8_t<XC_D, true>(pl, volts, T, F, N, acc, accumulate, s)
               : launch_mfma8_t<XC_D, false>(pl, volts, T, F, N, acc, accumulate, s);
}

}  // namespace xc
