// Host side of the C ABI declared in include/xcorr.h: argument validation,
// integration bookkeeping (sample counts, sequence gaps, the int32 bound) and
// kernel dispatch.  The library allocates no device memory.
#include "xcorr.h"
#include "xcorr_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

struct xcorr_ctx {
    xcorr_config cfg;
    xc::Plan plan;
    int kc;
    void *ws;
    size_t ws_bytes;
    int64_t t_max;
    int64_t max_dump;
    int64_t acc_samples;
    int64_t total_samples;
    int64_t ingests;
    int64_t dumps;
    int64_t launches;
    uint64_t gaps;
    uint64_t gaps_total;
    uint64_t last_seq;
    bool have_seq;
};

namespace {

thread_local std::string g_last_error;

int set_error(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return set_error(XCORR_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int64_t n_pairs(int64_t N) { return N * (N + 1) / 2; }

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Default diagonal block size for the MFMA path when the config leaves it 0
// and the tune cache has no entry: one triangular region per channel while
// the whole triangle fits one work-group's registers, else 4-block segments.
int default_tile(int N)
{
    const int nb = (N + 31) / 32;
    if (nb <= 6)
        return nb <= 2 ? 2 : (nb <= 3 ? 3 : (nb <= 4 ? 4 : 6));
    return 4;
}

// Tune cache: a text file of "bits N F path tile" lines written by the
// autotuner; the path named by $XCORR_TUNE_CACHE.
int cached_tile(const xcorr_config &c)
{
    const char *path = std::getenv("XCORR_TUNE_CACHE");
    if (!path || !*path)
        return 0;
    FILE *fh = std::fopen(path, "r");
    if (!fh)
        return 0;
    int bits, n, f, p, tile, found = 0;
    while (std::fscanf(fh, "%d %d %d %d %d", &bits, &n, &f, &p, &tile) == 5)
        if (bits == c.sample_bits && n == c.n_inputs && f == c.n_chans && p == c.path &&
            xc::plan_supported(n, tile))
            found = tile;
    std::fclose(fh);
    return found;
}

int validate(const xcorr_config *c, int64_t *t_max_out)
{
    if (!c)
        return set_error(XCORR_E_INVAL, "config is NULL");
    if (c->n_inputs < 1 || c->n_chans < 1)
        return set_error(XCORR_E_INVAL, "n_inputs and n_chans must be >= 1");
    if (c->n_inputs > 8192)
        return set_error(XCORR_E_INVAL, "n_inputs above 8192 is not supported");
    if (c->sample_bits != 4 && c->sample_bits != 8)
        return set_error(XCORR_E_INVAL, "sample_bits must be 4 or 8");
    if (c->layout != XCORR_LAYOUT_TFN)
        return set_error(XCORR_E_INVAL, "unknown layout");
    if (c->path != XCORR_PATH_PLAIN && c->path != XCORR_PATH_I8_MFMA && c->path != XCORR_PATH_F16_MFMA)
        return set_error(XCORR_E_INVAL, "unknown path");
    if (c->path == XCORR_PATH_F16_MFMA && c->sample_bits != 8)
        return set_error(XCORR_E_INVAL, "the FP16 path takes 8+8-bit input only");
    if (c->tile != 0 && !xc::plan_supported(c->n_inputs, c->tile))
        return set_error(XCORR_E_INVAL, "tile must be 0, 2, 3, 4, or 6 (6 only for N <= 192)");
    const int64_t tmax = c->sample_bits == 4 ? XCORR_TMAX_4BIT : XCORR_TMAX_8BIT;
    if (c->max_samples_per_dump < 0)
        return set_error(XCORR_E_INVAL, "max_samples_per_dump must be >= 0");
    if (c->max_samples_per_dump > tmax)
        return set_error(XCORR_E_OVERFLOW, "max_samples_per_dump exceeds the int32 bound");
    if (t_max_out)
        *t_max_out = tmax;
    return XCORR_OK;
}

size_t acc_bytes(const xcorr_config &c)
{
    return (size_t)c.n_chans * (size_t)n_pairs(c.n_inputs) * 2 * 4;
}

}  // namespace

extern "C" {

int xcorr_query(const xcorr_config *cfg, size_t *workspace_bytes, size_t *out_bytes, int64_t *t_max)
{
    int64_t tm = 0;
    const int rc = validate(cfg, &tm);
    if (rc)
        return rc;
    if (workspace_bytes)
        *workspace_bytes = round_up(acc_bytes(*cfg), 256);
    if (out_bytes)
        *out_bytes = acc_bytes(*cfg);
    if (t_max)
        *t_max = tm;
    return XCORR_OK;
}

int xcorr_init(const xcorr_config *cfg, void *d_workspace, size_t ws_bytes, xcorr_ctx **out)
{
    int64_t tm = 0;
    int rc = validate(cfg, &tm);
    if (rc)
        return rc;
    if (!out)
        return set_error(XCORR_E_INVAL, "out is NULL");
    if (!d_workspace || ws_bytes < round_up(acc_bytes(*cfg), 256))
        return set_error(XCORR_E_NOMEM, "workspace missing or smaller than xcorr_query's size");
    if ((uintptr_t)d_workspace % 256)
        return set_error(XCORR_E_INVAL, "workspace must be 256-byte aligned");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_error(XCORR_E_DEVICE, std::string("device is ") + prop.gcnArchName + ", not gfx950");

    xcorr_ctx *c = new (std::nothrow) xcorr_ctx();
    if (!c)
        return set_error(XCORR_E_NOMEM, "host allocation failed");
    c->cfg = *cfg;
    c->t_max = tm;
    c->max_dump = cfg->max_samples_per_dump ? cfg->max_samples_per_dump : tm;
    c->kc = 64;
    if (cfg->path != XCORR_PATH_PLAIN) {
        int tile = cfg->tile ? cfg->tile : cached_tile(*cfg);
        if (!tile)
            tile = default_tile(cfg->n_inputs);
        c->plan = xc::make_plan(cfg->n_inputs, tile);
        // time rows staged per LDS chunk (64 or 128; 128 for D >= 4 only)
        const char *v = std::getenv("XCORR_CHUNK");
        if (v && std::strcmp(v, "128") == 0 && c->plan.D >= 4 && cfg->sample_bits == 4)
            c->kc = 128;
    }
    c->ws = d_workspace;
    c->ws_bytes = ws_bytes;
    *out = c;
    return XCORR_OK;
}

int xcorr_ingest(xcorr_ctx *ctx, const void *d_volts, int64_t n_samples, uint64_t seq, void *stream)
{
    if (!ctx || !d_volts)
        return set_error(XCORR_E_INVAL, "ctx or d_volts is NULL");
    if (n_samples < 1)
        return set_error(XCORR_E_INVAL, "n_samples must be >= 1");
    if (n_samples > ctx->max_dump - ctx->acc_samples)
        return set_error(XCORR_E_OVERFLOW, "integration would exceed max_samples_per_dump");
    const xcorr_config &c = ctx->cfg;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const uint8_t *v = static_cast<const uint8_t *>(d_volts);
    int2 *acc = static_cast<int2 *>(ctx->ws);
    const int64_t bytes_per_row = (int64_t)c.n_chans * c.n_inputs * (c.sample_bits == 4 ? 1 : 2);
    const int64_t per_launch =
        c.path == XCORR_PATH_PLAIN ? n_samples
                                   : (c.sample_bits == 4 ? xc::kMaxSamplesPerLaunch4 : xc::kMaxSamplesPerLaunch8);
    for (int64_t t0 = 0; t0 < n_samples; t0 += per_launch) {
        const int64_t tl = std::min<int64_t>(per_launch, n_samples - t0);
        const int accumulate = (ctx->acc_samples > 0 || t0 > 0) ? 1 : 0;
        const uint8_t *vp = v + t0 * bytes_per_row;
        hipError_t e;
        if (c.path == XCORR_PATH_PLAIN)
            e = xc::launch_plain(c.sample_bits, vp, tl, c.n_chans, c.n_inputs, acc, accumulate, s);
        else if (c.sample_bits == 4)
            e = xc::launch_mfma4(ctx->plan, ctx->kc, vp, tl, c.n_chans, c.n_inputs, acc, accumulate, s);
        else
            e = xc::launch_mfma8(ctx->plan, c.path == XCORR_PATH_F16_MFMA, vp, tl, c.n_chans, c.n_inputs,
                                 ctx->ws, accumulate, s);
        if (e != hipSuccess)
            return hip_fail(e, "kernel launch");
        ++ctx->launches;
    }
    if (ctx->have_seq && seq != ctx->last_seq + 1) {
        const uint64_t missing = seq > ctx->last_seq ? seq - ctx->last_seq - 1 : 1;
        ctx->gaps += missing;
        ctx->gaps_total += missing;
    }
    ctx->have_seq = true;
    ctx->last_seq = seq;
    ctx->acc_samples += n_samples;
    ctx->total_samples += n_samples;
    ++ctx->ingests;
    return XCORR_OK;
}

int xcorr_dump(xcorr_ctx *ctx, void *d_out, int64_t *n_integrated, uint64_t *n_gaps, void *stream)
{
    if (!ctx || !d_out)
        return set_error(XCORR_E_INVAL, "ctx or d_out is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const hipError_t e = xc::launch_dump(ctx->ws, d_out, (int64_t)acc_bytes(ctx->cfg),
                                         ctx->acc_samples == 0 ? 1 : 0, s);
    if (e != hipSuccess)
        return hip_fail(e, "dump launch");
    ++ctx->launches;
    if (n_integrated)
        *n_integrated = ctx->acc_samples;
    if (n_gaps)
        *n_gaps = ctx->gaps;
    ctx->acc_samples = 0;
    ctx->gaps = 0;
    ++ctx->dumps;
    return XCORR_OK;
}

int xcorr_stats(const xcorr_ctx *ctx, xcorr_stats_t *out)
{
    if (!ctx || !out)
        return set_error(XCORR_E_INVAL, "ctx or out is NULL");
    out->samples_integrated = ctx->acc_samples;
    out->samples_total = ctx->total_samples;
    out->ingests = ctx->ingests;
    out->dumps = ctx->dumps;
    out->kernel_launches = ctx->launches;
    out->seq_gaps = ctx->gaps;
    out->seq_gaps_total = ctx->gaps_total;
    out->tile = ctx->plan.D;
    out->regions_per_chan = ctx->plan.regions;
    return XCORR_OK;
}

int xcorr_destroy(xcorr_ctx *ctx)
{
    if (!ctx)
        return set_error(XCORR_E_INVAL, "ctx is NULL");
    delete ctx;
    return XCORR_OK;
}

const char *xcorr_strerror(int code)
{
    switch (code) {
    case XCORR_OK: return "ok";
    case XCORR_E_INVAL: return "invalid argument";
    case XCORR_E_NOMEM: return "workspace too small";
    case XCORR_E_OVERFLOW: return "integration exceeds the int32 bound";
    case XCORR_E_HIP: return "HIP runtime error";
    case XCORR_E_DEVICE: return "unsupported device (gfx950 required)";
    default: return "unknown error";
    }
}

const char *xcorr_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
