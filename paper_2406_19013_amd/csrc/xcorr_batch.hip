// Batched persistent kernel of the 4+4-bit int8-MFMA path: one launch
// correlates several arrays of uneven N, F and sample count.
//
// Work items are (array, channel, region) in array order.  The item list is
// cut into 8 contiguous ranges, one per XCD (work-group b runs on XCD b % 8),
// so that the regions of a channel tend to share an L2; a work-group drains
// its own XCD's range first and then takes items from the other ranges.  A
// range's head is a global counter advanced by atomic add.  The work-group
// that finishes last (a done counter) sets the counters back to zero, so
// consecutive launches and graph replays need no clearing step.
#include "xc_mfma4.h"

namespace xc {
namespace {

constexpr int kBatchKC = 64;
// region sizes the batched kernel carries: 2, 3, 4 (any N) and 6 (N <= 192)
constexpr int batch_smem_bytes()
{
    int m = 0;
    for (int d : {2, 3, 4, 6})
        m = fused_smem_bytes(d) > m ? fused_smem_bytes(d) : m;
    return m;
}

// rectangle k (row-major over a > b) of nseg segments -> segments (a, b)
__device__ __forceinline__ void rect_ab(int k, int &a, int &b)
{
    a = (int)((1.f + sqrtf(1.f + 8.f * k)) * 0.5f);
    while (a * (a - 1) / 2 > k)
        --a;
    while ((a + 1) * a / 2 <= k)
        ++a;
    b = k - a * (a - 1) / 2;
}

template <int D, int VEC>
__device__ __forceinline__ void batch_item(uint8_t *smem, const BatchArray &A, int local)
{
    // the work-group runs alone on its CU: the ring may be as deep as D = 4's
    constexpr int NBUF = fused_nbuf(4);
    const int f = local / A.regions;
    const int r = local - f * A.regions;
    if (r < A.nseg) {
        mfma4f_dispatch<D, true, kBatchKC, NBUF, VEC, 0, 2, true>(smem, A.volts, A.T, A.F, A.N, f, r * D, r * D, A.acc,
                                                      A.acc, A.accumulate);
    } else if constexpr (D <= 4) {
        int a, b;
        rect_ab(r - A.nseg, a, b);
        mfma4f_dispatch<D, false, kBatchKC, NBUF, VEC, 0, 2, true>(smem, A.volts, A.T, A.F, A.N, f, a * D, b * D, A.acc,
                                                       A.acc, A.accumulate);
    }
}

template <int VEC>
__global__ __launch_bounds__(kMfmaThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void xc_batch4_kernel(const BatchArgs args, int *__restrict__ queue)
{
    __shared__ __attribute__((aligned(1024))) uint8_t smem[batch_smem_bytes()];
    __shared__ int s_item;
    const int xcd = blockIdx.x & 7;
    const int per = (args.total + 7) >> 3;
    int q = 0;   // ranges this work-group has found empty (thread 0 only)
    for (;;) {
        __syncthreads();   // every wave is done with s_item and with LDS
        if (threadIdx.x == 0) {
            int item = -1;
            while (q < 8) {
                const int x = (xcd + q) & 7;
                const int n = min(per, args.total - x * per);
                if (n > 0) {
                    const int k = atomicAdd(&queue[x], 1);
                    if (k < n) {
                        item = x * per + k;
                        break;
                    }
                }
                ++q;
            }
            s_item = item;
        }
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        if (item < 0)
            break;
        // the previous item's accumulator stores must be complete before the
        // LDS-DMA ring counts outstanding vector-memory operations again
        wait_vmcnt<0>();
        int a = 0;
        while (a + 1 < args.n && args.a[a + 1].item_begin <= item)
            ++a;
        const BatchArray &A = args.a[a];
        const int local = item - A.item_begin;
        switch (A.D) {
        case 2: batch_item<2, VEC>(smem, A, local); break;
        case 3: batch_item<3, VEC>(smem, A, local); break;
        case 6: batch_item<6, VEC>(smem, A, local); break;
        default: batch_item<4, VEC>(smem, A, local); break;
        }
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&queue[8], 1) == (int)gridDim.x - 1) {
            for (int x = 0; x <= 8; ++x)
                atomicExch(&queue[x], 0);
        }
    }
}

__global__ void xc_fill_zero_kernel(int *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0;
}

// Deterministic filler for the autotuner's input block: a hash of the byte
// index; 8+8-bit values are kept in [-127, 127].
__global__ void xc_fill_pattern_kernel(uint8_t *p, int64_t n, int eight_bit)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t h = (uint32_t)i * 2654435761u;
        h ^= h >> 15;
        h *= 2246822519u;
        h ^= h >> 13;
        p[i] = eight_bit ? (uint8_t)(int8_t)((int)(h % 255u) - 127) : (uint8_t)(h >> 24);
    }
}

}  // namespace

hipError_t launch_batch4(const BatchArgs &args, int *queue, int vec, int grid, hipStream_t s)
{
    if (args.n < 1 || args.n > kMaxBatchArrays || args.total < 1 || grid < 1 || !queue)
        return hipErrorInvalidValue;
    for (int a = 0; a < args.n; ++a) {
        const BatchArray &A = args.a[a];
        if (A.D < 2 || A.D == 5 || A.D > 6 || (A.D == 6 && A.N > 192) || A.T < 1 || A.T > kMaxSamplesPerLaunch4 || !A.volts || !A.acc ||
            (uintptr_t)A.acc % 16)
            return hipErrorInvalidValue;
    }
    grid = ((grid + 7) / 8) * 8;
    auto kern = vec ? xc_batch4_kernel<1> : xc_batch4_kernel<0>;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kMfmaThreads), 0, s, args, queue);
    return hipGetLastError();
}

hipError_t launch_fill_pattern(uint8_t *p, int64_t n, int eight_bit, hipStream_t s)
{
    if (!p || n < 1)
        return hipErrorInvalidValue;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(xc_fill_pattern_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, eight_bit);
    return hipGetLastError();
}

hipError_t launch_fill_zero(int *p, int n, hipStream_t s)
{
    if (!p || n < 1)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(xc_fill_zero_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace xc
