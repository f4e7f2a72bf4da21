// Hardware ceilings of the 4+4-bit correlation launch on this GPU (the
// denominators of a measured roofline; no correlation is computed here).
//
//   MFMA: one work-group of 8 waves per compute unit (two per SIMD, as the
//   correlation kernel) issuing independent 32x32x32 int8 MFMAs whose
//   operands are voltage bytes read from the caller's buffer, so the
//   multipliers toggle as they do on real data.
//
//   STREAM: the [T][F][N] input streamed into an LDS ring with the grid,
//   channel-to-work-group mapping, 64-sample chunks, 16-byte LDS-DMA loads and
//   cache policy of the correlation kernel, and nothing else done with it.
#include "xc_mfma.h"
#include "xcorr.h"
#include "xcorr_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace xc {
namespace {

constexpr int kCeilThreads = 512;
constexpr int kCeilNbuf = 8;
constexpr int kCeilChunk = 64;
constexpr int kCeilLoads = kCeilChunk * 16 / kCeilThreads;   // 16-byte loads per lane per chunk
constexpr int kCeilRowBytes = 256;                         // LDS bytes per time row (16 units of 16 B)

__device__ __forceinline__ void ceiling_mfma(const uint8_t *__restrict__ src, int64_t span, int64_t iters,
                                             int *out)
{
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * (kCeilThreads / 64) + (threadIdx.x >> 6);
    const int64_t base = (wid * 4096) % span;    // a multiple of 16; base + 4096 <= bytes
    v4i op[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        op[k] = *(const v4i *)(src + base + k * 1024 + lane * 16);
    v16i acc[8];
#pragma unroll
    for (int m = 0; m < 8; ++m)
        acc[m] = v16i{};
    for (int64_t it = 0; it < iters; ++it) {
        static_for<0, 8>([&](auto mc) {
            constexpr int m = mc;
            acc[m] = mfma_i8(op[m & 3], op[(m + 1) & 3], acc[m]);
        });
        static_for<0, 8>([&](auto mc) {
            constexpr int m = mc;
            acc[m] = mfma_i8(op[(m + 2) & 3], op[(m + 3) & 3], acc[m]);
        });
    }
    uint32_t s = 0;
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int r = 0; r < 16; ++r)
            s += (uint32_t)acc[m][r];
    out[(int64_t)blockIdx.x * kCeilThreads + threadIdx.x] = (int)s;
}

__global__ __launch_bounds__(kCeilThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void xc_ceiling_mfma_kernel(const uint8_t *src, int64_t span, int64_t iters, int *out)
{
    ceiling_mfma(src, span, iters, out);
}

__device__ __forceinline__ void ceiling_stream(uint8_t *smem, const uint8_t *__restrict__ volts, int64_t T, int F,
                                               int N, int per, int *out)
{
    constexpr int BUF = kCeilChunk * kCeilRowBytes;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    lds_u8 *const ring = (lds_u8 *)smem;
    const int xcd = blockIdx.x & 7, m = blockIdx.x >> 3, M = gridDim.x >> 3;
    const int r0 = xcd * per;
    const int rlen = min(per, F - r0);
    const int n_my = rlen > m ? (rlen - m + M - 1) / M : 0;
    const int nch = (int)((T + kCeilChunk - 1) / kCeilChunk);
    const int64_t row_bytes = (int64_t)F * N;
    const int64_t chunk_bytes = kCeilChunk * row_bytes;
    int issued = 0;
    for (int k = 0; k < n_my; ++k) {
        const int f = r0 + m + k * M;
        int voff[kCeilLoads];
#pragma unroll
        for (int u = 0; u < kCeilLoads; ++u) {
            const int U = (w * kCeilLoads + u) * 64 + lane;
            const int r = U >> 4, p = U & 15;
            voff[u] = 16 * p < N ? (int)(r * row_bytes) + f * N + 16 * p : kBufferOutOfRange;
        }
        for (int c = 0; c < nch; ++c) {
            const uint8_t *src = volts + (int64_t)c * chunk_bytes;
            const int64_t rows = min((int64_t)kCeilChunk, T - (int64_t)c * kCeilChunk);
            __amdgpu_buffer_rsrc_t rsrc =
                __builtin_amdgcn_make_buffer_rsrc((void *)src, (short)0, (int)(rows * row_bytes), 0x00020000);
            lds_u8 *dst = ring + (issued % kCeilNbuf) * BUF + w * kCeilLoads * 1024;
#pragma unroll
            for (int u = 0; u < kCeilLoads; ++u)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rsrc, (__attribute__((address_space(3))) void *)(dst + u * 1024), 16, voff[u], 0, 0,
                    kStreamLoadPolicy);
            ++issued;
            // at most kCeilNbuf - 1 chunks of this wave in flight, so the
            // slot the next chunk takes has landed
            wait_vmcnt<(kCeilNbuf - 1) * kCeilLoads>();
        }
    }
    wait_vmcnt<0>();
    __syncthreads();
    out[(int64_t)blockIdx.x * kCeilThreads + threadIdx.x] = ((const int *)smem)[threadIdx.x];
}

__global__ __launch_bounds__(kCeilThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void xc_ceiling_stream_kernel(const uint8_t *volts, int64_t T, int F, int N, int per, int *out)
{
    __shared__ __attribute__((aligned(1024))) uint8_t smem[kCeilNbuf * kCeilChunk * kCeilRowBytes];
    ceiling_stream(smem, volts, T, F, N, per, out);
}

int cu_count()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 8)
        return 0;
    return cus;
}

}  // namespace
}  // namespace xc

extern "C" int xcorr_ceiling(int32_t kind, const void *d_volts, int64_t n_samples, int32_t n_chans,
                             int32_t n_inputs, int64_t iters, void *d_out, int64_t out_ints, double *ops,
                             void *stream)
{
    using namespace xc;
    if (!d_volts || (uintptr_t)d_volts % 16 || !d_out || !ops || n_samples < 1 || n_chans < 1 || n_inputs < 16 ||
        n_inputs > 256 || n_inputs % 16 || 64LL * n_chans * n_inputs >= (1LL << 31) - 16)
        return XCORR_E_INVAL;
    const int cus = cu_count();
    if (!cus)
        return api_error(XCORR_E_HIP, "cannot read the compute-unit count");
    const int64_t bytes = n_samples * n_chans * (int64_t)n_inputs;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (kind == XCORR_CEILING_MFMA_I8) {
        const int grid = cus;
        if (iters < 1 || bytes < 4096 || out_ints < (int64_t)grid * kCeilThreads)
            return XCORR_E_INVAL;
        const int64_t span = (bytes - 4096) / 16 * 16 + 16;
        hipLaunchKernelGGL(xc_ceiling_mfma_kernel, dim3(grid), dim3(kCeilThreads), 0, s,
                           (const uint8_t *)d_volts, span, iters, (int *)d_out);
        *ops = (double)grid * (kCeilThreads / 64) * iters * 16 * 65536.0;
    } else if (kind == XCORR_CEILING_STREAM) {
        const int per = (n_chans + 7) / 8;
        const int grid = 8 * std::max(1, std::min(cus / 8, per));
        if (out_ints < (int64_t)grid * kCeilThreads)
            return XCORR_E_INVAL;
        hipLaunchKernelGGL(xc_ceiling_stream_kernel, dim3(grid), dim3(kCeilThreads), 0, s,
                           (const uint8_t *)d_volts, n_samples, (int)n_chans, (int)n_inputs, per, (int *)d_out);
        *ops = (double)bytes;
    } else {
        return XCORR_E_INVAL;
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? XCORR_OK : api_error(XCORR_E_HIP, std::string("ceiling launch: ") + hipGetErrorString(e));
}
