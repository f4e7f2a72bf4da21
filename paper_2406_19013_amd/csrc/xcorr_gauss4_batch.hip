// Batched launch of the three-product 4+4-bit kernel: one launch correlates
// several arrays of uneven N, F and sample count.
//
// Each array contributes one job per region shape of its plan (its diagonal
// triangles, and its rectangles when it has several segments).  A job names
// the rows of work-groups that serve it (a row is 8 work-groups, one per
// XCD); those work-groups walk its (channel, region) items exactly as a
// launch of that shape alone does, and a work-group runs the jobs that name
// its row one after another.  The item ranges are fixed before the launch, so
// there are no queue counters to reset and a captured graph replays as is.
#include "xc_gauss4.h"

#include <algorithm>
#include <cstddef>

namespace xc {
namespace {

// region shapes the batched launch carries: triangles of 6 blocks, pairs of
// 2-, 3- and 4-block triangles (two channels to an item; single triangles
// where F = 1), rectangles of 2, 3 and 4; a job's kind is 2 * shape +
// accumulate
enum G3Shape { kTri2, kTri3, kTri4, kTri6, kRect2, kRect3, kRect4, kPair2, kPair3, kPair4 };

constexpr int kMaxG3Jobs = 2 * kMaxBatchArrays;

struct G3Job {
    G3Args a;
    int kind;
};

struct G3BatchArgs {
    int n;                      // jobs, run in this order
    G3Job job[kMaxG3Jobs];
};

constexpr int g3_batch_smem_bytes()
{
    int m = 0;
    for (int d : {2, 3, 4, 6})
        m = std::max(m, g3_smem_bytes<kTri>(d));
    for (int d : {2, 3, 4})
        m = std::max(m, g3_smem_bytes<kRect>(d));
    for (int d : {2, 3, 4})
        m = std::max(m, g3_smem_bytes<kPair>(d));
    return m;
}

// The job of a work-group is picked by a run-time index, so it is read from
// the kernel-argument segment (the argument starts it) as scalar loads into a
// local copy; indexing the argument itself would copy the whole table to
// private memory.  (Copying the table into LDS first measured 20 % slower.)
using kernarg_int = const __attribute__((address_space(4))) int;

template <typename T>
__device__ __forceinline__ T kernarg_read(int byte_offset)
{
    static_assert(sizeof(T) % 4 == 0, "whole dwords");
    kernarg_int *p = (kernarg_int *)((const __attribute__((address_space(4))) uint8_t *)
                                         __builtin_amdgcn_kernarg_segment_ptr() + byte_offset);
    int w[sizeof(T) / 4];
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k)
        w[k] = p[k];
    T v;
    __builtin_memcpy(&v, w, sizeof v);
    return v;
}

__global__ __launch_bounds__(kG3Threads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void xc_gauss4_batch_kernel(const G3BatchArgs b)
{
    __shared__ __attribute__((aligned(1024))) uint8_t smem[g3_batch_smem_bytes()];
    const int row = (int)(blockIdx.x >> 3);
    constexpr int jobs = offsetof(G3BatchArgs, job);
    for (int j = 0; j < b.n; ++j) {
        const G3Job job = kernarg_read<G3Job>(jobs + j * (int)sizeof(G3Job));
        const G3Args &a = job.a;
        if (row < a.mrow0 || row >= a.mrow0 + a.mrows)
            continue;
        // the previous job's stores drained (the DMA ring's waits count
        // outstanding vector-memory operations) and its LDS use over
        wait_vmcnt<0>();
        __syncthreads();
        switch (job.kind) {
#define XC_SHAPE(S, D, RECT)                                                  \
    case 2 * S: g3_dispatch<D, RECT, 0, 0>(smem, a, nullptr); break;          \
    case 2 * S + 1: g3_dispatch<D, RECT, 1, 0>(smem, a, nullptr); break;
        XC_SHAPE(kTri2, 2, kTri) XC_SHAPE(kTri3, 3, kTri) XC_SHAPE(kTri4, 4, kTri) XC_SHAPE(kTri6, 6, kTri)
        XC_SHAPE(kRect2, 2, kRect) XC_SHAPE(kRect3, 3, kRect) XC_SHAPE(kRect4, 4, kRect)
        XC_SHAPE(kPair2, 2, kPair) XC_SHAPE(kPair3, 3, kPair) XC_SHAPE(kPair4, 4, kPair)
#undef XC_SHAPE
        default: break;
        }
    }
}

// Relative time of one 64-sample chunk of one item of a shape: its MFMAs per
// 32-sample step (three per off-diagonal tile, two per diagonal tile) plus a
// fixed 31 for the chunk's loads, barrier and operand reads (fitted to the
// measured chunk times of the 4- and 6-block triangles, 0.81 and 1.25 us at
// 2048 samples; the 4-block rectangle, 1.2 us, lands within 10 %).
int64_t chunk_cost(int D, bool rect) { return 31 + (rect ? 3LL * D * D : 3LL * D * (D - 1) / 2 + 2LL * D); }
// a pair item: both channels' MFMAs, one chunk's fixed cost
int64_t pair_chunk_cost(int D) { return chunk_cost(D, false) + (chunk_cost(D, false) - 31); }

}  // namespace

bool gauss4_batch_shape(const Plan &pl, int F, int N)
{
    const bool carried = pl.nseg == 1 ? (pl.D == 2 || pl.D == 3 || pl.D == 4 || pl.D == 6) : (pl.D >= 2 && pl.D <= 4);
    return carried && gauss4_supported(pl, F, N);
}

bool gauss4_batch_supported(const BatchArray &A)
{
    Plan pl{};
    pl.D = A.D;
    pl.nseg = A.nseg;
    pl.regions = A.regions;
    pl.NB = (A.N + 31) / 32;
    return gauss4_batch_shape(pl, A.F, A.N) && A.volts && (uintptr_t)A.volts % 16 == 0 && A.acc && A.T >= 1 &&
           A.T <= kMaxSamplesPerLaunch4;
}

hipError_t launch_gauss4_batch(const BatchArgs &args, int cus, hipStream_t s)
{
    if (args.n < 1 || args.n > kMaxBatchArrays || cus < 8)
        return hipErrorInvalidValue;
    G3BatchArgs b{};
    int64_t work[kMaxG3Jobs], per[kMaxG3Jobs];
    for (int i = 0; i < args.n; ++i) {
        const BatchArray &A = args.a[i];
        if (!gauss4_batch_supported(A))
            return hipErrorInvalidValue;
        for (int rect = 0; rect <= (A.nseg > 1 ? 1 : 0); ++rect) {
            G3Job &J = b.job[b.n];
            const bool pair = !rect && A.D >= 2 && A.D <= 4 && A.F >= 2;
            const int shape = rect ? kRect2 + (A.D - 2)
                              : pair ? kPair2 + (A.D - 2)
                                     : (A.D == 6 ? kTri6 : kTri2 + (A.D - 2));
            J.kind = 2 * shape + (A.accumulate ? 1 : 0);
            J.a.volts = A.volts;
            J.a.T = A.T;
            J.a.F = A.F;
            J.a.N = A.N;
            J.a.nreg = rect ? A.nseg * (A.nseg - 1) / 2 : A.nseg;
            J.a.out = A.acc;
            J.a.in = A.acc;
            const int64_t items = pair ? g3_items<kPair>(A.F, J.a.nreg) : (int64_t)A.F * J.a.nreg;
            per[b.n] = (items + 7) / 8;
            J.a.per = (int)per[b.n];
            // an item: its chunks plus about four chunks' worth of epilogue
            // (the combination and the stores of its tiles)
            work[b.n] = (pair ? pair_chunk_cost(A.D) : chunk_cost(A.D, rect)) * ((A.T + 63) / 64 + 4);
            ++b.n;
        }
    }
    // Every job is spread over all rows of work-groups (one work-group per
    // CU), as a launch of its own would be, and the work-groups walk the jobs
    // in turn, largest first: a work-group that finishes its share of one job
    // starts the next at once, so the jobs' tails overlap and no launch gaps
    // remain.  (Giving each job its own rows instead, so that the arrays run
    // side by side, measured 12 % slower for two equal arrays.)  A job with
    // fewer items per XCD than rows takes the rows after the previous such
    // job's, so small jobs spread over the work-groups.
    const int rows = cus / 8;
    int order[kMaxG3Jobs];
    for (int j = 0; j < b.n; ++j)
        order[j] = j;
    std::stable_sort(order, order + b.n, [&](int x, int y) { return per[x] * work[x] > per[y] * work[y]; });
    G3BatchArgs sorted = b;
    int next_small = 0;
    for (int k = 0; k < b.n; ++k) {
        G3Job &J = sorted.job[k];
        J = b.job[order[k]];
        J.a.mrows = (int)std::min<int64_t>(rows, per[order[k]]);
        if (J.a.mrows == rows) {
            J.a.mrow0 = 0;
        } else {
            if (next_small + J.a.mrows > rows)
                next_small = 0;
            J.a.mrow0 = next_small;
            next_small += J.a.mrows;
        }
    }
    b = sorted;
    hipLaunchKernelGGL(xc_gauss4_batch_kernel, dim3(8 * rows), dim3(kG3Threads), 0, s, b);
    return hipGetLastError();
}

}  // namespace xc
