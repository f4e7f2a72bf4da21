// Full-Stokes visibilities of dual-polarisation feeds from the input
// visibilities (paper Section 1: full-Stokes output of 96 dual-polarisation
// feeds; Section 3.3: X north-south, Y east-west).  Input 2 f + pol is feed
// f's polarisation pol (0 = X, 1 = Y); for feeds a >= b
//   XX = V(2a, 2b), YY = V(2a+1, 2b+1), XY = V(2a, 2b+1), YX = V(2a+1, 2b)
// (for a = b, XY = conj V(2a+1, 2a), the stored entry), and
//   I = XX + YY, Q = XX - YY, U = XY + YX, V = -i (XY - YX)
// in exact int64 arithmetic.  One thread per (channel, feed pair): it reads
// four int32 (re, im) pairs and writes 64 contiguous bytes; a streaming,
// HBM-bound pass.
#include "xcorr.h"
#include "xcorr_internal.h"

#include <hip/hip_runtime.h>

#include <string>

namespace xc {
namespace {

struct c64 {
    long long r, i;
};

__device__ __forceinline__ c64 vis_at(const int2 *v, int64_t p)
{
    const int2 x = v[p];
    return {x.x, x.y};
}

__global__ __launch_bounds__(256) void xc_stokes_kernel(const int2 *__restrict__ vis, int nf, int64_t P, int64_t Pf,
                                                        longlong2 *__restrict__ out)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t f = blockIdx.y;
    if (q >= Pf)
        return;
    // feed pair q = a (a + 1) / 2 + b, b <= a
    int64_t a = (int64_t)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
    while (a * (a + 1) / 2 > q)
        --a;
    while ((a + 1) * (a + 2) / 2 <= q)
        ++a;
    const int64_t b = q - a * (a + 1) / 2;
    const int2 *v = vis + f * P;
    const int64_t r0 = (2 * a) * (2 * a + 1) / 2, r1 = (2 * a + 1) * (2 * a + 2) / 2;   // rows 2a, 2a + 1
    const c64 xx = vis_at(v, r0 + 2 * b);
    const c64 yy = vis_at(v, r1 + 2 * b + 1);
    const c64 yx = vis_at(v, r1 + 2 * b);
    c64 xy;
    if (a > b) {
        xy = vis_at(v, r0 + 2 * b + 1);
    } else {
        const c64 t = vis_at(v, r1 + 2 * a);   // V(2a+1, 2a) = conj XY
        xy = {t.r, -t.i};
    }
    longlong2 *o = out + (f * Pf + q) * 4;
    o[0] = make_longlong2(xx.r + yy.r, xx.i + yy.i);
    o[1] = make_longlong2(xx.r - yy.r, xx.i - yy.i);
    o[2] = make_longlong2(xy.r + yx.r, xy.i + yx.i);
    o[3] = make_longlong2(xy.i - yx.i, -(xy.r - yx.r));
}

}  // namespace
}  // namespace xc

extern "C" int xcorr_stokes(const void *d_vis, int32_t n_inputs, int32_t n_chans, void *d_out, void *stream)
{
    using namespace xc;
    if (!d_vis || !d_out || n_inputs < 2 || n_inputs % 2 || n_chans < 1 || n_chans > 65535 ||
        (uintptr_t)d_vis % 8 || (uintptr_t)d_out % 16)
        return XCORR_E_INVAL;
    const int nf = n_inputs / 2;
    const int64_t P = (int64_t)n_inputs * (n_inputs + 1) / 2, Pf = (int64_t)nf * (nf + 1) / 2;
    if ((Pf + 255) / 256 > 0x7fffffff)
        return XCORR_E_INVAL;
    hipLaunchKernelGGL(xc_stokes_kernel, dim3((unsigned)((Pf + 255) / 256), (unsigned)n_chans), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), (const int2 *)d_vis, nf, P, Pf, (longlong2 *)d_out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? XCORR_OK : api_error(XCORR_E_HIP, std::string("stokes launch: ") + hipGetErrorString(e));
}
