// Internal declarations shared by the host API and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include "xcorr.h"
#include <cstdint>
#include <string>

struct xcorr_ctx;

namespace xc {

// Work split of one channel's lower triangle for the MFMA paths.  Inputs are
// grouped into 32-input blocks (NB = ceil(N/32)); the block triangle is cut
// into diagonal segments of D blocks (triangular regions) and the rectangles
// between segments (rectangular regions, only when D <= 4).  One work-group
// handles one (channel, region).
struct Plan {
    int D = 0;              // diagonal segment size in blocks
    int NB = 0;             // 32-input blocks
    int nseg = 0;           // diagonal segments
    int regions = 0;        // regions per channel
};

// Host-side helpers of the C ABI shared between its source files.
int api_error(int code, const std::string &msg);   // records the detail, returns code
struct CtxShape {
    int n_inputs, n_chans, sample_bits, path;
    int64_t max_samples_per_dump;
};
CtxShape ctx_shape(const xcorr_ctx *ctx);

Plan make_plan(int N, int D);
bool plan_supported(int N, int D);

// One integration through a stack-held context whose running sums (when the
// integration needs any) are `ws`; allocates nothing (the static-scratch
// entry point).
int correlate_once(const xcorr_config *cfg, void *ws, size_t ws_bytes, const void *d_volts, int64_t n_samples,
                   void *d_out, int64_t *n_integrated, hipStream_t s);

// Launchers: enqueue on `stream`, return hipSuccess or the launch error.
// `accumulate` = 0 overwrites the accumulators, 1 adds to them.
// T <= kMaxSamplesPerLaunch for the MFMA paths (the host splits longer ingests).
// 4+4-bit: the fused-product kernel keeps two K-parity partial sums of at
// most 32896 per sample each (|256 Im| + |16 re|), over 32-sample steps, so a
// launch takes at most 2 * 32 * floor((2^31 - 1) / 32896 / 32) samples.
constexpr int64_t kMaxSamplesPerLaunch4 = 130560;

constexpr int64_t kMaxSamplesPerLaunch8 = 133143;  // |re*re| <= 127^2 per sample

hipError_t launch_plain(int bits, const uint8_t *volts, int64_t T, int F, int N, int2 *acc,
                        int accumulate, hipStream_t s);
hipError_t launch_mfma4(const Plan &pl, int kc, const uint8_t *volts, int64_t T, int F, int N,
                        int2 *acc, int accumulate, hipStream_t s);
// fused-product variant (one Re and one Im accumulator per tile), the default
// acc_in (default: acc) is where accumulate = 1 reads the running sums; with
// acc_in != acc the result goes to acc (e.g. a caller's dump buffer).
hipError_t launch_mfma4f(const Plan &pl, const uint8_t *volts, int64_t T, int F, int N, int2 *acc,
                         int accumulate, hipStream_t s, const int2 *acc_in = nullptr);
// 8+8-bit input, int8 MFMA (f16 = false, int2 accumulators) or FP16 MFMA with
// FP32 accumulation (f16 = true, float2 accumulators).
hipError_t launch_mfma8(const Plan &pl, bool f16, const uint8_t *volts, int64_t T, int F, int N, void *acc,
                        int accumulate, hipStream_t s);
// per-D launchers of the 8+8-bit kernels (xcorr_mfma8.hip compiled with -DXC_D=d)
hipError_t launch_mfma8_d1(const Plan &pl, bool f16, const uint8_t *volts, int64_t T, int F, int N,
                          void *acc, int accumulate, hipStream_t s);
hipError_t launch_mfma8_d2(const Plan &pl, bool f16, const uint8_t *volts, int64_t T, int F, int N,
                          void *acc, int accumulate, hipStream_t s);
hipError_t launch_mfma8_d3(const Plan &pl, bool f16, const uint8_t *volts, int64_t T, int F, int N,
                          void *acc, int accumulate, hipStream_t s);
hipError_t launch_mfma8_d4(const Plan &pl, bool f16, const uint8_t *volts, int64_t T, int F, int N,
                          void *acc, int accumulate, hipStream_t s);
hipError_t launch_mfma8_d5(const Plan &pl, bool f16, const uint8_t *volts, int64_t T, int F, int N,
                          void *acc, int accumulate, hipStream_t s);
hipError_t launch_mfma8_d6(const Plan &pl, bool f16, const uint8_t *volts, int64_t T, int F, int N,
                          void *acc, int accumulate, hipStream_t s);

hipError_t launch_dump(const void *acc, void *out, int64_t bytes, int empty, hipStream_t s);

// Several caller blocks of one array in one 4+4-bit launch: chunk c of the
// launch is chunk c % chunks_per_block of block c / chunks_per_block (every
// block holds chunks_per_block whole 64-row chunks).
constexpr int kMaxFusedBlocks = 8;
struct BlockTable {
    const uint8_t *p[kMaxFusedBlocks];
    int chunks_per_block;
};
hipError_t launch_mfma4f_blocks(const Plan &pl, const BlockTable &bt, int n_blocks, int F, int N, int2 *acc,
                                int accumulate, hipStream_t s, const int2 *acc_in = nullptr);

// Three-product kernel (4+4-bit, int8 MFMA): persistent; a whole triangle per
// channel (N <= 32 D, D <= 6) or segments of D <= 4 blocks with the rectangles
// between them (two launches); N a multiple of 16, 16-byte-aligned input.
// acc_in as for launch_mfma4f.
bool gauss4_supported(const Plan &pl, int F, int N);
hipError_t launch_gauss4(const Plan &pl, const uint8_t *volts, int64_t T, int F, int N, int2 *acc, int accumulate,
                         hipStream_t s, const int2 *acc_in = nullptr);
hipError_t launch_gauss4_blocks(const Plan &pl, const BlockTable &bt, int n_blocks, int F, int N, int2 *acc,
                                int accumulate, hipStream_t s, const int2 *acc_in = nullptr);

// Batched launch (4+4-bit, int8 MFMA) over up to kMaxBatchArrays arrays of
// uneven N, F and sample counts; the descriptors travel by value in the kernel
// arguments, so a captured graph holds everything it needs.  The queue-driven
// kernel (launch_batch4) drains a work queue of (array, channel, region)
// items; the three-product one (launch_gauss4_batch, below) walks per-shape
// jobs.
constexpr int kMaxBatchArrays = 16;
constexpr int kBatchQueueInts = 16;   // 8 per-XCD queue heads, a done counter, padding

struct BatchArray {
    const uint8_t *volts;   // [T][F][N] packed 4+4-bit
    int2 *acc;              // [F][P] accumulators
    int64_t T;              // samples in this launch (>= 1)
    int F, N;
    int D, nseg, regions;   // region plan, D in {2, 3, 4}
    int accumulate;
    int item_begin;         // first work item of this array
};

struct BatchArgs {
    int n;                  // arrays
    int total;              // work items
    BatchArray a[kMaxBatchArrays];
};

// queue: kBatchQueueInts ints of device memory, zero before the first launch;
// every launch leaves it zero again.  vec: every array has N % 16 == 0, a
// 16-byte aligned input and 64 * F * N < 2^31 - 16.
hipError_t launch_batch4(const BatchArgs &args, int *queue, int vec, int grid, hipStream_t s);
// The batch on the three-product kernel: every array must pass
// gauss4_batch_supported (a plan of 2, 3, 4 or 6 blocks that
// gauss4_batch_shape accepts, a 16-byte-aligned input); needs no queue.
// cus: compute units of the device.
bool gauss4_batch_shape(const Plan &pl, int F, int N);
bool gauss4_batch_supported(const BatchArray &A);
hipError_t launch_gauss4_batch(const BatchArgs &args, int cus, hipStream_t s);
hipError_t launch_fill_zero(int *p, int n, hipStream_t s);
hipError_t launch_fill_pattern(uint8_t *p, int64_t n, int eight_bit, hipStream_t s);

}  // namespace xc
