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
#include <vector>

// Kernel family a 4+4-bit int8-MFMA context runs (the tuner times the same).
enum class Kernel4 {
    Gauss,   // three products per tile, persistent; triangles and rectangles (default)
    Fused,   // fused products: one Re and one Im accumulator per tile ($XCORR_MFMA4_VARIANT=fused)
    Roles,   // one wave per real product ($XCORR_MFMA4_VARIANT=roles)
};

struct xcorr_ctx {
    xcorr_config cfg;
    xc::Plan plan;
    int kc;
    Kernel4 k4;
    int tile_from_cache;   // the tile came from a tune-cache line
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

}  // namespace

int xc::api_error(int code, const std::string &msg) { return set_error(code, msg); }

xc::CtxShape xc::ctx_shape(const xcorr_ctx *c)
{
    return {c->cfg.n_inputs, c->cfg.n_chans, c->cfg.sample_bits, c->cfg.path, c->max_dump};
}

namespace {

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

Kernel4 kernel4_from_env()
{
    const char *fv = std::getenv("XCORR_MFMA4_VARIANT");
    if (fv && std::strcmp(fv, "roles") == 0)
        return Kernel4::Roles;
    if (fv && std::strcmp(fv, "fused") == 0)
        return Kernel4::Fused;
    return Kernel4::Gauss;
}

// The three-product kernel takes every plan it carries (a whole triangle of
// up to 6 blocks, or segments of up to 4 blocks with the rectangles between
// them) for N a multiple of 16 (16-byte-aligned inputs are checked per call).
bool gauss_runs(Kernel4 k, const xc::Plan &pl, int F, int N)
{
    return k == Kernel4::Gauss && xc::gauss4_supported(pl, F, N);
}

int default_tile(int N);

// Name of the kernel an ingest of this config with this tile launches
// (batch = 0) or that the batched launch runs for it (batch = 1); the tuner
// times that kernel and labels its tune-cache line with this name.
const char *kernel_for(const xcorr_config &c, int tile, bool batch)
{
    if (c.path == XCORR_PATH_PLAIN)
        return "xc_plain_kernel";
    if (batch)
        return kernel4_from_env() == Kernel4::Gauss &&
                       xc::gauss4_batch_shape(xc::make_plan(c.n_inputs, tile), c.n_chans, c.n_inputs)
                   ? "xc_gauss4_batch_kernel"
                   : "xc_batch4_kernel";
    if (c.sample_bits == 8)
        return c.path == XCORR_PATH_F16_MFMA ? "xc_mfma8_kernel_f16" : "xc_mfma8_kernel_i8";
    const Kernel4 k = kernel4_from_env();
    if (k == Kernel4::Roles)
        return "xc_mfma4_kernel";
    return gauss_runs(k, xc::make_plan(c.n_inputs, tile), c.n_chans, c.n_inputs) ? "xc_gauss4_kernel"
                                                                                : "xc_mfma4f_kernel";
}

// Tiles the batched kernel carries for an array of N inputs.
bool batch_tile_supported(int N, int D) { return (D >= 2 && D <= 4) || (D == 6 && N <= 192); }

// Tune cache: a text file of "bits N F path tile kernel" lines written by the
// autotuner; the path named by $XCORR_TUNE_CACHE.  The last line for this
// config and for the kernel the caller will run wins; lines timed on another
// kernel are ignored.
int cached_tile(const xcorr_config &c, bool batch)
{
    const char *path = std::getenv("XCORR_TUNE_CACHE");
    if (!path || !*path)
        return 0;
    FILE *fh = std::fopen(path, "r");
    if (!fh)
        return 0;
    char line[256];
    int found = 0;
    while (std::fgets(line, sizeof line, fh)) {
        int bits, n, f, p, tile;
        char kern[96];
        if (std::sscanf(line, "%d %d %d %d %d %95s", &bits, &n, &f, &p, &tile, kern) != 6)
            continue;
        if (bits == c.sample_bits && n == c.n_inputs && f == c.n_chans && p == c.path &&
            (batch ? batch_tile_supported(n, tile) : xc::plan_supported(n, tile)) &&
            std::strcmp(kern, kernel_for(c, tile, batch)) == 0)
            found = tile;
    }
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
        return set_error(XCORR_E_INVAL, "tile must be 0, 2..4, 1 (N <= 32) or 5..6 (N <= 32*tile)");
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

// Tile of a batch member when the tune cache has none for the batched
// kernel: its own tile when the batched kernel carries it (2, 3, 4, or 6 with
// N <= 192), else the one of 2, 3, 4 with the fewest tiles (padding
// included), the larger on a tie.
int batch_fallback_tile(int N, int own)
{
    if (batch_tile_supported(N, own))
        return own;
    int best = 0;
    int64_t best_tiles = -1;
    for (int d = 2; d <= 4; ++d) {
        const xc::Plan p = xc::make_plan(N, d);
        const int64_t tiles = (int64_t)p.nseg * d * (d + 1) / 2 + (int64_t)p.nseg * (p.nseg - 1) / 2 * d * d;
        if (best_tiles < 0 || tiles <= best_tiles) {
            best = d;
            best_tiles = tiles;
        }
    }
    return best;
}

// Region plan of a batch member: the tile tuned for the batched kernel
// (tune cache), else the fallback above.
xc::Plan batch_plan(const xcorr_ctx *c)
{
    int d = cached_tile(c->cfg, true);
    if (!d)
        d = batch_fallback_tile(c->cfg.n_inputs, c->plan.D);
    return xc::make_plan(c->cfg.n_inputs, d);
}

int device_cus(int *cus)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    e = hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipDeviceGetAttribute");
    return XCORR_OK;
}

// Sequence-number bookkeeping shared by the single and batched ingest.
void note_ingest(xcorr_ctx *ctx, int64_t n_samples, uint64_t seq)
{
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
}

// One 4+4-bit int8-MFMA launch of the kernel family the context runs:
// results to `out`, running sums (accumulate = 1) from acc_in (default out).
hipError_t launch4(const xcorr_ctx *ctx, const uint8_t *v, int64_t T, int2 *out, int accumulate, hipStream_t s,
                   const int2 *acc_in = nullptr)
{
    const xcorr_config &c = ctx->cfg;
    if (gauss_runs(ctx->k4, ctx->plan, c.n_chans, c.n_inputs) && (uintptr_t)v % 16 == 0)
        return xc::launch_gauss4(ctx->plan, v, T, c.n_chans, c.n_inputs, out, accumulate, s, acc_in);
    return xc::launch_mfma4f(ctx->plan, v, T, c.n_chans, c.n_inputs, out, accumulate, s, acc_in);
}

// The current device must be a gfx950 GPU.
int device_check()
{
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
    return XCORR_OK;
}

// Fill a validated context; use_cache = false leaves the tune cache file
// unread (the tile is the config's or the built-in choice).
void setup_ctx(xcorr_ctx *c, const xcorr_config &cfg, int64_t tm, void *ws, size_t ws_bytes, bool use_cache)
{
    c->cfg = cfg;
    c->t_max = tm;
    c->max_dump = cfg.max_samples_per_dump ? cfg.max_samples_per_dump : tm;
    c->kc = 64;
    if (cfg.path != XCORR_PATH_PLAIN) {
        int tile = cfg.tile;
        if (!tile && use_cache) {
            tile = cached_tile(cfg, false);
            c->tile_from_cache = tile != 0;
        }
        if (!tile)
            tile = default_tile(cfg.n_inputs);
        c->plan = xc::make_plan(cfg.n_inputs, tile);
        // time rows staged per LDS chunk of the per-role kernel (64 or 128; 128 for D >= 4 only)
        const char *v = std::getenv("XCORR_CHUNK");
        if (v && std::strcmp(v, "128") == 0 && c->plan.D >= 4 && cfg.sample_bits == 4)
            c->kc = 128;
        c->k4 = kernel4_from_env();
    }
    c->ws = ws;
    c->ws_bytes = ws_bytes;
}

}  // namespace

// One integration of n_samples through a context that lives on this stack
// frame, with `ws` (ws_bytes) as its running-sum buffer when the integration
// needs one: a single 4+4-bit int8-MFMA launch writes straight to d_out, any
// other integration runs through the buffer.  Allocates nothing.
int xc::correlate_once(const xcorr_config *cfg, void *ws, size_t ws_bytes, const void *d_volts, int64_t n_samples,
                       void *d_out, int64_t *n_integrated, hipStream_t s)
{
    int64_t tm = 0;
    int rc = validate(cfg, &tm);
    if (rc)
        return rc;
    if (!d_volts || !d_out)
        return set_error(XCORR_E_INVAL, "d_volts or d_out is NULL");
    if (n_samples < 1)
        return set_error(XCORR_E_INVAL, "n_samples must be >= 1");
    if (n_samples > (cfg->max_samples_per_dump ? cfg->max_samples_per_dump : tm))
        return set_error(XCORR_E_OVERFLOW, "integration would exceed max_samples_per_dump");
    const bool one_launch = cfg->sample_bits == 4 && cfg->path == XCORR_PATH_I8_MFMA &&
                            kernel4_from_env() != Kernel4::Roles && n_samples <= kMaxSamplesPerLaunch4;
    const size_t need = round_up(acc_bytes(*cfg), 256);
    if (!one_launch && need > ws_bytes)
        return set_error(XCORR_E_NOMEM, "the integration needs " + std::to_string(need) +
                                            " bytes of running sums, more than the " + std::to_string(ws_bytes) +
                                            "-byte static scratch");
    if ((rc = device_check()) != XCORR_OK)
        return rc;
    xcorr_ctx c{};
    setup_ctx(&c, *cfg, tm, ws, ws_bytes, false);
    return xcorr_ingest_dump(&c, d_volts, n_samples, 0, d_out, n_integrated, nullptr, s);
}

struct xcorr_batch {
    std::vector<xcorr_ctx *> ctx;
    std::vector<xc::Plan> plan;
    int *queue;
    int grid;   // work-groups of the queue-driven kernel: one per CU
};

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
    if ((rc = device_check()) != XCORR_OK)
        return rc;
    xcorr_ctx *c = new (std::nothrow) xcorr_ctx();
    if (!c)
        return set_error(XCORR_E_NOMEM, "host allocation failed");
    setup_ctx(c, *cfg, tm, d_workspace, ws_bytes, true);
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
        : c.sample_bits == 8       ? xc::kMaxSamplesPerLaunch8
                                   : xc::kMaxSamplesPerLaunch4;
    for (int64_t t0 = 0; t0 < n_samples; t0 += per_launch) {
        const int64_t tl = std::min<int64_t>(per_launch, n_samples - t0);
        const int accumulate = (ctx->acc_samples > 0 || t0 > 0) ? 1 : 0;
        const uint8_t *vp = v + t0 * bytes_per_row;
        hipError_t e;
        if (c.path == XCORR_PATH_PLAIN)
            e = xc::launch_plain(c.sample_bits, vp, tl, c.n_chans, c.n_inputs, acc, accumulate, s);
        else if (c.sample_bits == 4 && ctx->k4 == Kernel4::Roles)
            e = xc::launch_mfma4(ctx->plan, ctx->kc, vp, tl, c.n_chans, c.n_inputs, acc, accumulate, s);
        else if (c.sample_bits == 4)
            e = launch4(ctx, vp, tl, acc, accumulate, s);
        else
            e = xc::launch_mfma8(ctx->plan, c.path == XCORR_PATH_F16_MFMA, vp, tl, c.n_chans, c.n_inputs,
                                 ctx->ws, accumulate, s);
        if (e != hipSuccess)
            return hip_fail(e, "kernel launch");
        ++ctx->launches;
    }
    note_ingest(ctx, n_samples, seq);
    return XCORR_OK;
}

int xcorr_ingest_dump(xcorr_ctx *ctx, const void *d_volts, int64_t n_samples, uint64_t seq, void *d_out,
                      int64_t *n_integrated, uint64_t *n_gaps, void *stream)
{
    if (!ctx || !d_volts || !d_out)
        return set_error(XCORR_E_INVAL, "ctx, d_volts or d_out is NULL");
    if (n_samples < 1)
        return set_error(XCORR_E_INVAL, "n_samples must be >= 1");
    if (n_samples > ctx->max_dump - ctx->acc_samples)
        return set_error(XCORR_E_OVERFLOW, "integration would exceed max_samples_per_dump");
    if ((uintptr_t)d_out % 16)
        return set_error(XCORR_E_INVAL, "d_out must be 16-byte aligned");
    const xcorr_config &c = ctx->cfg;
    if (!(c.sample_bits == 4 && c.path == XCORR_PATH_I8_MFMA && ctx->k4 != Kernel4::Roles)) {
        const int rc = xcorr_ingest(ctx, d_volts, n_samples, seq, stream);
        return rc ? rc : xcorr_dump(ctx, d_out, n_integrated, n_gaps, stream);
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const uint8_t *v = static_cast<const uint8_t *>(d_volts);
    int2 *acc = static_cast<int2 *>(ctx->ws);
    const int64_t bytes_per_row = (int64_t)c.n_chans * c.n_inputs;
    const int64_t L = xc::kMaxSamplesPerLaunch4;
    for (int64_t t0 = 0; t0 < n_samples; t0 += L) {
        const int64_t tl = std::min<int64_t>(L, n_samples - t0);
        const int accumulate = (ctx->acc_samples > 0 || t0 > 0) ? 1 : 0;
        const bool last = t0 + tl >= n_samples;
        // the last launch adds the running sums to its own and writes the
        // result to d_out: the integration ends without a copy
        const hipError_t e = last ? launch4(ctx, v + t0 * bytes_per_row, tl, static_cast<int2 *>(d_out),
                                            accumulate, s, acc)
                                  : launch4(ctx, v + t0 * bytes_per_row, tl, acc, accumulate, s);
        if (e != hipSuccess)
            return hip_fail(e, "kernel launch");
        ++ctx->launches;
    }
    note_ingest(ctx, n_samples, seq);
    if (n_integrated)
        *n_integrated = ctx->acc_samples;
    if (n_gaps)
        *n_gaps = ctx->gaps;
    ctx->acc_samples = 0;
    ctx->gaps = 0;
    ++ctx->dumps;
    return XCORR_OK;
}

int xcorr_ingest_blocks(xcorr_ctx *ctx, const void *const *d_blocks, int n_blocks, int64_t block_samples,
                        uint64_t first_seq, void *stream)
{
    if (!ctx || !d_blocks)
        return set_error(XCORR_E_INVAL, "ctx or d_blocks is NULL");
    if (n_blocks < 1 || block_samples < 1)
        return set_error(XCORR_E_INVAL, "n_blocks and block_samples must be >= 1");
    for (int b = 0; b < n_blocks; ++b)
        if (!d_blocks[b])
            return set_error(XCORR_E_INVAL, "NULL block");
    if (block_samples > (ctx->max_dump - ctx->acc_samples) / n_blocks)
        return set_error(XCORR_E_OVERFLOW, "integration would exceed max_samples_per_dump");
    const xcorr_config &c = ctx->cfg;
    bool fused = c.sample_bits == 4 && c.path == XCORR_PATH_I8_MFMA && ctx->k4 != Kernel4::Roles &&
                 block_samples % 64 == 0 &&
                 block_samples <= xc::kMaxSamplesPerLaunch4 && c.n_inputs % 16 == 0 &&
                 64LL * c.n_chans * c.n_inputs < (1LL << 31) - 16;
    for (int b = 0; b < n_blocks && fused; ++b)
        fused = (uintptr_t)d_blocks[b] % 16 == 0;
    if (!fused) {
        // one ingest per block (other formats and paths, ragged block sizes)
        for (int b = 0; b < n_blocks; ++b) {
            const int rc = xcorr_ingest(ctx, d_blocks[b], block_samples, first_seq + b, stream);
            if (rc)
                return rc;
        }
        return XCORR_OK;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int group = (int)std::min<int64_t>(xc::kMaxFusedBlocks, xc::kMaxSamplesPerLaunch4 / block_samples);
    for (int b0 = 0; b0 < n_blocks; b0 += group) {
        const int n = std::min(group, n_blocks - b0);
        xc::BlockTable bt{};
        for (int b = 0; b < n; ++b)
            bt.p[b] = static_cast<const uint8_t *>(d_blocks[b0 + b]);
        bt.chunks_per_block = (int)(block_samples / 64);
        const int accumulate = (ctx->acc_samples > 0 || b0 > 0) ? 1 : 0;
        const hipError_t e = gauss_runs(ctx->k4, ctx->plan, c.n_chans, c.n_inputs)
                                 ? xc::launch_gauss4_blocks(ctx->plan, bt, n, c.n_chans, c.n_inputs,
                                                            static_cast<int2 *>(ctx->ws), accumulate, s)
                                 : xc::launch_mfma4f_blocks(ctx->plan, bt, n, c.n_chans, c.n_inputs,
                                                            static_cast<int2 *>(ctx->ws), accumulate, s);
        if (e != hipSuccess)
            return hip_fail(e, "kernel launch");
        ++ctx->launches;
    }
    for (int b = 0; b < n_blocks; ++b)
        note_ingest(ctx, block_samples, first_seq + b);
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
    out->tile_from_cache = ctx->tile_from_cache;
    return XCORR_OK;
}

int xcorr_destroy(xcorr_ctx *ctx)
{
    if (!ctx)
        return set_error(XCORR_E_INVAL, "ctx is NULL");
    delete ctx;
    return XCORR_OK;
}

// ---------------------------------------------------------------------------
// Batched persistent launch

static int batch_check(xcorr_ctx *const *ctxs, int n)
{
    static_assert(XCORR_MAX_BATCH == xc::kMaxBatchArrays, "batch limit");
    if (!ctxs || n < 1 || n > xc::kMaxBatchArrays)
        return set_error(XCORR_E_INVAL, "a batch holds 1 to 16 contexts");
    for (int a = 0; a < n; ++a) {
        if (!ctxs[a])
            return set_error(XCORR_E_INVAL, "NULL context in the batch");
        if (ctxs[a]->cfg.sample_bits != 4 || ctxs[a]->cfg.path != XCORR_PATH_I8_MFMA)
            return set_error(XCORR_E_INVAL, "the batched launch takes 4+4-bit int8-MFMA contexts");
        for (int b = 0; b < a; ++b)
            if (ctxs[b] == ctxs[a])
                return set_error(XCORR_E_INVAL, "a context appears twice in the batch");
    }
    return XCORR_OK;
}

int xcorr_batch_query(xcorr_ctx *const *ctxs, int n, size_t *workspace_bytes)
{
    const int rc = batch_check(ctxs, n);
    if (rc)
        return rc;
    if (workspace_bytes)
        *workspace_bytes = 256;
    return XCORR_OK;
}

int xcorr_batch_init(xcorr_ctx *const *ctxs, int n, void *d_workspace, size_t ws_bytes, xcorr_batch **out)
{
    int rc = batch_check(ctxs, n);
    if (rc)
        return rc;
    if (!out)
        return set_error(XCORR_E_INVAL, "out is NULL");
    if (!d_workspace || ws_bytes < 256)
        return set_error(XCORR_E_NOMEM, "batch workspace missing or smaller than 256 bytes");
    if ((uintptr_t)d_workspace % 256)
        return set_error(XCORR_E_INVAL, "workspace must be 256-byte aligned");
    int cus = 0;
    rc = device_cus(&cus);
    if (rc)
        return rc;
    xcorr_batch *b = new (std::nothrow) xcorr_batch();
    if (!b)
        return set_error(XCORR_E_NOMEM, "host allocation failed");
    for (int a = 0; a < n; ++a) {
        b->ctx.push_back(ctxs[a]);
        b->plan.push_back(batch_plan(ctxs[a]));
    }
    b->queue = static_cast<int *>(d_workspace);
    b->grid = cus;   // one 512-thread work-group per CU (LDS-limited), persistent
    hipError_t e = xc::launch_fill_zero(b->queue, xc::kBatchQueueInts, nullptr);
    if (e == hipSuccess)
        e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "batch queue initialisation");
    }
    *out = b;
    return XCORR_OK;
}

int xcorr_batch_ingest(xcorr_batch *b, const void *const *d_volts, const int64_t *n_samples,
                       const uint64_t *seqs, void *stream)
{
    if (!b || !d_volts || !n_samples)
        return set_error(XCORR_E_INVAL, "batch, d_volts or n_samples is NULL");
    const int n = (int)b->ctx.size();
    int64_t longest = 0;
    for (int a = 0; a < n; ++a) {
        const xcorr_ctx *c = b->ctx[a];
        if (n_samples[a] < 0)
            return set_error(XCORR_E_INVAL, "n_samples must be >= 0");
        if (n_samples[a] > 0 && !d_volts[a])
            return set_error(XCORR_E_INVAL, "d_volts is NULL for an array with samples");
        if (n_samples[a] > c->max_dump - c->acc_samples)
            return set_error(XCORR_E_OVERFLOW, "integration would exceed max_samples_per_dump");
        longest = std::max(longest, n_samples[a]);
    }
    if (longest == 0)
        return set_error(XCORR_E_INVAL, "no array has samples to ingest");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t L = xc::kMaxSamplesPerLaunch4;
    for (int64_t t0 = 0; t0 < longest; t0 += L) {
        xc::BatchArgs args{};
        int vec = 1;
        int64_t items = 0;
        for (int a = 0; a < n; ++a) {
            if (n_samples[a] <= t0)
                continue;
            const xcorr_ctx *c = b->ctx[a];
            const xc::Plan &pl = b->plan[a];
            const int F = c->cfg.n_chans, N = c->cfg.n_inputs;
            xc::BatchArray &A = args.a[args.n++];
            A.volts = static_cast<const uint8_t *>(d_volts[a]) + t0 * (int64_t)F * N;
            A.acc = static_cast<int2 *>(c->ws);
            A.T = std::min(L, n_samples[a] - t0);
            A.F = F;
            A.N = N;
            A.D = pl.D;
            A.nseg = pl.nseg;
            A.regions = pl.regions;
            A.accumulate = (c->acc_samples > 0 || t0 > 0) ? 1 : 0;
            A.item_begin = (int)items;
            items += (int64_t)F * pl.regions;
            if (N % 16 || (uintptr_t)A.volts % 16 || 64LL * F * N >= (1LL << 31) - 16)
                vec = 0;
        }
        if (items > (1LL << 30))
            return set_error(XCORR_E_INVAL, "too many work items in one batch");
        args.total = (int)items;
        // the three-product kernel when it carries every member, else the
        // queue-driven four-product kernel
        bool gauss = kernel4_from_env() == Kernel4::Gauss;
        for (int a = 0; a < args.n && gauss; ++a)
            gauss = xc::gauss4_batch_supported(args.a[a]);
        const hipError_t e = gauss ? xc::launch_gauss4_batch(args, b->grid, s)
                                   : xc::launch_batch4(args, b->queue, vec, std::min<int64_t>(b->grid, items), s);
        if (e != hipSuccess)
            return hip_fail(e, "batch launch");
        for (int a = 0; a < n; ++a)
            if (n_samples[a] > t0)
                ++b->ctx[a]->launches;
    }
    for (int a = 0; a < n; ++a)
        if (n_samples[a] > 0) {
            xcorr_ctx *c = b->ctx[a];
            note_ingest(c, n_samples[a], seqs ? seqs[a] : (c->have_seq ? c->last_seq + 1 : 0));
        }
    return XCORR_OK;
}

int xcorr_batch_tiles(const xcorr_batch *b, int32_t *tiles)
{
    if (!b || !tiles)
        return set_error(XCORR_E_INVAL, "batch or tiles is NULL");
    for (size_t a = 0; a < b->plan.size(); ++a)
        tiles[a] = b->plan[a].D;
    return XCORR_OK;
}

int xcorr_batch_destroy(xcorr_batch *b)
{
    if (!b)
        return set_error(XCORR_E_INVAL, "batch is NULL");
    delete b;
    return XCORR_OK;
}

// ---------------------------------------------------------------------------
// Autotuner

static int64_t tune_samples() { return 2048; }

int xcorr_autotune_query(const xcorr_config *cfg, size_t *scratch_bytes)
{
    const int rc = validate(cfg, nullptr);
    if (rc)
        return rc;
    if (cfg->path == XCORR_PATH_PLAIN)
        return set_error(XCORR_E_INVAL, "the plain path has no tile to tune");
    const size_t volts = (size_t)tune_samples() * cfg->n_chans * cfg->n_inputs * (cfg->sample_bits == 4 ? 1 : 2);
    if (scratch_bytes)
        *scratch_bytes = round_up(acc_bytes(*cfg), 256) + round_up(volts, 256) + 256;
    return XCORR_OK;
}

int xcorr_autotune_kernel(const xcorr_config *cfg, int32_t batch, char *name, size_t len)
{
    const int rc = validate(cfg, nullptr);
    if (rc)
        return rc;
    if (!name || len < 1)
        return set_error(XCORR_E_INVAL, "name is NULL or empty");
    if (batch && (cfg->sample_bits != 4 || cfg->path != XCORR_PATH_I8_MFMA))
        return set_error(XCORR_E_INVAL, "the batched launch takes 4+4-bit int8-MFMA configs");
    int tile = cfg->tile;
    if (!tile && !batch)
        tile = cached_tile(*cfg, false);
    if (!tile)
        tile = default_tile(cfg->n_inputs);
    std::snprintf(name, len, "%s", kernel_for(*cfg, tile, batch != 0));
    return XCORR_OK;
}

int xcorr_plan_tile(const xcorr_config *cfg, int32_t batch, int32_t *tile, int32_t *from_cache)
{
    const int rc = validate(cfg, nullptr);
    if (rc)
        return rc;
    if (!tile)
        return set_error(XCORR_E_INVAL, "tile is NULL");
    if (cfg->path == XCORR_PATH_PLAIN)
        return set_error(XCORR_E_INVAL, "the plain path has no tile");
    if (batch && (cfg->sample_bits != 4 || cfg->path != XCORR_PATH_I8_MFMA))
        return set_error(XCORR_E_INVAL, "the batched launch takes 4+4-bit int8-MFMA configs");
    int cached = 0;
    int d = 0;
    if (batch) {
        d = cached_tile(*cfg, true);
        cached = d != 0;
        if (!d) {
            const int own = cfg->tile ? cfg->tile : cached_tile(*cfg, false);
            d = batch_fallback_tile(cfg->n_inputs, own ? own : default_tile(cfg->n_inputs));
        }
    } else {
        d = cfg->tile;
        if (!d) {
            d = cached_tile(*cfg, false);
            cached = d != 0;
        }
        if (!d)
            d = default_tile(cfg->n_inputs);
    }
    *tile = d;
    if (from_cache)
        *from_cache = cached;
    return XCORR_OK;
}

}  // extern "C"

// Time `run` (a launch of the kernel under test) with HIP events: one
// warm-up launch, then kReps launches; *ms is their total.
template <class Run>
static hipError_t time_launches(Run &&run, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, float *ms)
{
    constexpr int kReps = 5;
    hipError_t e = run(0);
    if (e == hipSuccess)
        e = hipEventRecord(ev0, s);
    for (int r = 0; r < kReps && e == hipSuccess; ++r)
        e = run(1);
    if (e == hipSuccess)
        e = hipEventRecord(ev1, s);
    if (e == hipSuccess)
        e = hipEventSynchronize(ev1);
    if (e == hipSuccess)
        e = hipEventElapsedTime(ms, ev0, ev1);
    return e;
}

extern "C" {

static int append_tune_line(const xcorr_config &c, int tile, bool batch)
{
    const char *path = std::getenv("XCORR_TUNE_CACHE");
    if (!path || !*path)
        return XCORR_OK;
    FILE *fh = std::fopen(path, "a");
    if (!fh)
        return set_error(XCORR_E_INVAL, std::string("cannot append to the tune cache ") + path);
    std::fprintf(fh, "%d %d %d %d %d %s\n", c.sample_bits, c.n_inputs, c.n_chans, c.path, tile,
                 kernel_for(c, tile, batch));
    std::fclose(fh);
    return XCORR_OK;
}

// Shared body of the two tuners: candidate tiles of the config, each timed
// on the kernel the caller will run (batch = 0: the ingest kernel of a
// context; batch = 1: the batched persistent kernel with this config as its
// only array).
static int autotune_impl(const xcorr_config *cfg, void *d_scratch, size_t scratch_bytes, void *stream,
                         int32_t *best_tile, bool batch)
{
    size_t need = 0;
    int rc = xcorr_autotune_query(cfg, &need);
    if (rc)
        return rc;
    if (!best_tile)
        return set_error(XCORR_E_INVAL, "best_tile is NULL");
    if (batch && (cfg->sample_bits != 4 || cfg->path != XCORR_PATH_I8_MFMA))
        return set_error(XCORR_E_INVAL, "the batched launch takes 4+4-bit int8-MFMA configs");
    if (!d_scratch || scratch_bytes < need)
        return set_error(XCORR_E_NOMEM, "scratch missing or smaller than xcorr_autotune_query's size");
    if ((uintptr_t)d_scratch % 256)
        return set_error(XCORR_E_INVAL, "scratch must be 256-byte aligned");
    const xcorr_config &c = *cfg;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint8_t *base = static_cast<uint8_t *>(d_scratch);
    void *acc = base;
    uint8_t *volts = base + round_up(acc_bytes(c), 256);
    const int64_t T = tune_samples();
    const int64_t vbytes = T * c.n_chans * c.n_inputs * (c.sample_bits == 4 ? 1 : 2);
    int *queue = reinterpret_cast<int *>(volts + round_up(vbytes, 256));
    int cus = 0;
    if (batch && (rc = device_cus(&cus)) != XCORR_OK)
        return rc;
    hipError_t e = xc::launch_fill_pattern(volts, vbytes, c.sample_bits == 8, s);
    if (e == hipSuccess && batch)
        e = xc::launch_fill_zero(queue, xc::kBatchQueueInts, s);
    if (e != hipSuccess)
        return hip_fail(e, "autotune set-up");
    hipEvent_t ev[2];
    if ((e = hipEventCreate(&ev[0])) != hipSuccess)
        return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&ev[1])) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return hip_fail(e, "hipEventCreate");
    }
    const Kernel4 k4 = kernel4_from_env();
    int best = 0;
    float best_ms = 0.f;
    for (int d = 1; d <= 6 && e == hipSuccess; ++d) {
        if (batch ? !batch_tile_supported(c.n_inputs, d) : !xc::plan_supported(c.n_inputs, d))
            continue;
        const xc::Plan pl = xc::make_plan(c.n_inputs, d);
        auto run = [&](int accumulate) -> hipError_t {
            if (batch) {
                xc::BatchArgs args{};
                args.n = 1;
                xc::BatchArray &A = args.a[0];
                A.volts = volts;
                A.acc = static_cast<int2 *>(acc);
                A.T = T;
                A.F = c.n_chans;
                A.N = c.n_inputs;
                A.D = pl.D;
                A.nseg = pl.nseg;
                A.regions = pl.regions;
                A.accumulate = accumulate;
                A.item_begin = 0;
                const int64_t items = (int64_t)c.n_chans * pl.regions;
                if (items > (1LL << 30))
                    return hipErrorInvalidValue;
                args.total = (int)items;
                if (k4 == Kernel4::Gauss && xc::gauss4_batch_supported(A))
                    return xc::launch_gauss4_batch(args, cus, s);
                const int vec = c.n_inputs % 16 == 0 && 64LL * c.n_chans * c.n_inputs < (1LL << 31) - 16;
                return xc::launch_batch4(args, queue, vec, (int)std::min<int64_t>(cus, items), s);
            }
            if (c.sample_bits == 8)
                return xc::launch_mfma8(pl, c.path == XCORR_PATH_F16_MFMA, volts, T, c.n_chans, c.n_inputs, acc,
                                        accumulate, s);
            if (k4 == Kernel4::Roles)
                return xc::launch_mfma4(pl, 64, volts, T, c.n_chans, c.n_inputs, static_cast<int2 *>(acc),
                                        accumulate, s);
            if (gauss_runs(k4, pl, c.n_chans, c.n_inputs))
                return xc::launch_gauss4(pl, volts, T, c.n_chans, c.n_inputs, static_cast<int2 *>(acc), accumulate,
                                         s);
            return xc::launch_mfma4f(pl, volts, T, c.n_chans, c.n_inputs, static_cast<int2 *>(acc), accumulate, s);
        };
        float ms = 0.f;
        e = time_launches(run, s, ev[0], ev[1], &ms);
        if (e == hipSuccess && (best == 0 || ms < best_ms)) {
            best = d;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (e != hipSuccess)
        return hip_fail(e, "autotune timing");
    *best_tile = best;
    return append_tune_line(c, best, batch);
}

int xcorr_autotune(const xcorr_config *cfg, void *d_scratch, size_t scratch_bytes, void *stream,
                   int32_t *best_tile)
{
    return autotune_impl(cfg, d_scratch, scratch_bytes, stream, best_tile, false);
}

int xcorr_autotune_batch(const xcorr_config *cfg, void *d_scratch, size_t scratch_bytes, void *stream,
                         int32_t *best_tile)
{
    return autotune_impl(cfg, d_scratch, scratch_bytes, stream, best_tile, true);
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
