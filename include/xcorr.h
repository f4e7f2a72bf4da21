/*
 * xcorr.h -- C ABI of the MI355X (gfx950) X-engine.
 *
 * The X-engine of an FX correlator receives channelised voltages and, per
 * frequency channel, forms the conjugate multiply-accumulate (CMAC) of every
 * input pair over an integration (paper: Section 2.3 "X-engine"; Eq. 2 of
 * Section 3.2 defines a visibility as the time average of S1* . S2).  This
 * library computes, for each channel f and each pair j <= i of the N inputs,
 *
 *     V_ij[f] = sum_t x_i[f,t] * conj(x_j[f,t])            (exact, int32)
 *
 * accumulated across ingest calls until a dump.  Pair (i, j) is stored at
 * p = i(i+1)/2 + j; autos are included, so P = N(N+1)/2 pairs per channel.
 *
 * Input formats (Section 2.1 "F-engine": 4-bit real + 4-bit imaginary after
 * requantisation; Section 2.3: the fluff step widens them to 8+8 bits):
 *   sample_bits = 4 : uint8 per sample, high nibble = real, low nibble =
 *                     imaginary, two's complement in [-8, 7].
 *   sample_bits = 8 : int8 real then int8 imaginary, each in [-127, 127]
 *                     (-128 is outside the contract: its negation does not fit).
 * Input layout XCORR_LAYOUT_TFN: time-major [T][F][N] samples, i.e. sample
 * (t, f, i) at element ((t*F + f)*N + i).
 *
 * Output of a dump: [F][P][2] (re, im) int32 for the integer paths, float32
 * for the FP16 path.  Its size is Eq. 1 of Section 2.2 with 4-byte values:
 * N(N+1)/2 * F * 2 * 4 bytes.
 *
 * Conventions.  Every call returns XCORR_OK (0) or a negative XCORR_E_* code;
 * no exception crosses the ABI.  Pointers named d_* are device pointers on
 * the current HIP device; the caller owns all device memory (the library
 * allocates none).  `stream` is a hipStream_t (NULL = the null stream); work
 * is enqueued asynchronously and the host does not synchronise.  A context is
 * not thread-safe; distinct contexts are independent.  Calls that overlap on
 * one context's workspace from different streams race.
 */
#ifndef XCORR_H
#define XCORR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define XCORR_OK 0
#define XCORR_E_INVAL (-1)    /* bad argument, shape, format or path */
#define XCORR_E_NOMEM (-2)    /* workspace too small / admission budget exceeded */
#define XCORR_E_OVERFLOW (-3) /* the integration would pass the int32 bound */
#define XCORR_E_HIP (-4)      /* a HIP runtime call failed (see xcorr_last_error) */
#define XCORR_E_DEVICE (-5)   /* the current device is not a gfx950 GPU */

/* compute paths */
#define XCORR_PATH_PLAIN 0    /* VALU int32 multiply-adds, no matrix cores */
#define XCORR_PATH_I8_MFMA 1  /* int8 MFMA, int32 accumulation (exact) */
#define XCORR_PATH_F16_MFMA 2 /* 8-bit input only: FP16 MFMA, FP32 accumulation */

/* input layouts */
#define XCORR_LAYOUT_TFN 0

/* samples the int32 accumulators can take before any entry may overflow:
 * 4-bit: |contribution| <= 128 per sample (autos at -8-8i), floor((2^31-1)/128);
 * 8-bit: |contribution| <= 2*127^2 per sample, floor((2^31-1)/32258). */
#define XCORR_TMAX_4BIT 16777215LL
#define XCORR_TMAX_8BIT 66572LL

typedef struct xcorr_ctx xcorr_ctx;
typedef struct xcorr_batch xcorr_batch;
typedef struct xcorr_pipe xcorr_pipe;

typedef struct {
    int32_t n_inputs;     /* N >= 1 (input k = 2*feed + polarisation) */
    int32_t n_chans;      /* F >= 1 */
    int32_t sample_bits;  /* 4 or 8 */
    int32_t path;         /* XCORR_PATH_* */
    int32_t layout;       /* XCORR_LAYOUT_TFN */
    int32_t tile;         /* MFMA paths: diagonal block size D in 32-input
                             blocks: 2..4 for any N (1 only when N <= 32),
                             5 or 6 only when N <= 32*D; 0 = tuned value from
                             the tune cache, else a built-in choice */
    int64_t max_samples_per_dump; /* 0 = the format's T_max; larger than
                                     T_max is XCORR_E_OVERFLOW */
} xcorr_config;

typedef struct {
    int64_t samples_integrated; /* since the last dump */
    int64_t samples_total;      /* since init */
    int64_t ingests;
    int64_t dumps;
    int64_t kernel_launches;
    uint64_t seq_gaps;          /* missing sequence numbers since the last dump */
    uint64_t seq_gaps_total;
    int32_t tile;               /* diagonal block size in use (MFMA paths) */
    int32_t regions_per_chan;   /* work-groups per channel in one ingest */
    int32_t tile_from_cache;    /* 1: the tile came from a tune-cache line */
} xcorr_stats_t;

/*
 * Sizes for admission by memory (pure host, no device call).
 *   workspace_bytes : device bytes a context needs (the accumulators,
 *                     F*P*2*4 bytes, rounded up to 256)
 *   out_bytes       : bytes one dump writes (Eq. 1 of Section 2.2, 4-byte values)
 *   t_max           : largest integration, in samples, that stays exact
 * Any output pointer may be NULL.  Errors: XCORR_E_INVAL for an invalid
 * config (N < 1, F < 1, bits not 4/8, unknown path or layout, FP16 path with
 * 4-bit input, unsupported tile); XCORR_E_OVERFLOW if
 * max_samples_per_dump > t_max.
 */
int xcorr_query(const xcorr_config *cfg, size_t *workspace_bytes, size_t *out_bytes, int64_t *t_max);

/*
 * Create a context on the current HIP device: the state of one correlator
 * instance, i.e. the accumulators the GPU thread of a hashpipe instance
 * integrates into between two hand-offs to its output thread (Section 2.3
 * "X-engine").  d_workspace (>= workspace_bytes
 * from xcorr_query) is borrowed until xcorr_destroy; its contents need no
 * initialisation.  Errors: as xcorr_query, XCORR_E_NOMEM if ws_bytes is too
 * small or d_workspace is NULL, XCORR_E_DEVICE if the device is not gfx950,
 * XCORR_E_HIP on a runtime failure.  *out is set only on success.
 */
int xcorr_init(const xcorr_config *cfg, void *d_workspace, size_t ws_bytes, xcorr_ctx **out);

/*
 * The conjugate multiply-accumulate of Section 2.3 "X-engine" on one block of
 * channelised voltages (Eq. 2 of Section 3.2 defines the product).
 * Correlate n_samples >= 1 time samples, d_volts = [n_samples][F][N] in the
 * configured format, and add them to the integration (the first ingest after
 * a dump overwrites the accumulators).  d_volts stays caller-owned and must
 * stay valid until the stream passes this call.  Any n_samples is allowed:
 * partial tiles are zero-padded, which is exact.  `seq` is the caller's block
 * sequence number; gaps (seq != previous seq + 1) are counted, not fatal.
 * Errors (checked before anything is enqueued): XCORR_E_INVAL (NULL ctx or
 * pointer, n_samples < 1), XCORR_E_OVERFLOW if samples_integrated + n_samples
 * would exceed max_samples_per_dump, XCORR_E_HIP if a launch fails.
 */
int xcorr_ingest(xcorr_ctx *ctx, const void *d_volts, int64_t n_samples, uint64_t seq, void *stream);

/*
 * Correlate n_blocks separate device blocks of block_samples samples each
 * (d_blocks[b] = [block_samples][F][N]) as consecutive parts of the
 * integration, with sequence numbers first_seq, first_seq + 1, ...  For
 * 4+4-bit int8-MFMA contexts with block_samples a multiple of 64, N a
 * multiple of 16 and 16-byte-aligned blocks, up to 8 blocks go into one
 * launch (the accumulators are read and written once per launch instead of
 * once per block); otherwise the blocks are ingested one by one.  Errors as
 * xcorr_ingest; XCORR_E_INVAL also for n_blocks < 1 or a NULL block.
 */
int xcorr_ingest_blocks(xcorr_ctx *ctx, const void *const *d_blocks, int n_blocks, int64_t block_samples,
                        uint64_t first_seq, void *stream);

/*
 * End an integration (Section 2.4 "Data storage": about 4 s per integration;
 * Section 2.3: the output thread takes the GPU thread's result buffer).
 * Write the integration to d_out ([F][P][2], out_bytes from xcorr_query) and
 * start a new one.  A dump of an empty integration writes zeros.
 * n_integrated / n_gaps (may be NULL) receive the samples and the counted
 * sequence gaps of the integration just closed.
 */
int xcorr_dump(xcorr_ctx *ctx, void *d_out, int64_t *n_integrated, uint64_t *n_gaps, void *stream);

/*
 * The last block of an integration and its hand-off (Sections 2.3 and 2.4),
 * in one call: as
 * xcorr_ingest(ctx, d_volts, n_samples, seq) followed by xcorr_dump(ctx,
 * d_out, ...), with the same results.  On the 4+4-bit int8-MFMA path the
 * final launch adds the running sums to its own and writes the visibilities
 * straight into d_out (16-byte aligned), so no separate copy runs; other
 * paths make the two calls.  Errors as the two calls.
 */
int xcorr_ingest_dump(xcorr_ctx *ctx, const void *d_volts, int64_t n_samples, uint64_t seq, void *d_out,
                      int64_t *n_integrated, uint64_t *n_gaps, void *stream);

/*
 * Counters of a context (the status values a hashpipe thread publishes each
 * cycle, Section 2.3) and its destruction (the workspace is released to the
 * caller).  Errors: XCORR_E_INVAL for NULL arguments.
 */
int xcorr_stats(const xcorr_ctx *ctx, xcorr_stats_t *out);
int xcorr_destroy(xcorr_ctx *ctx);

/*
 * Batched launch (4+4-bit, int8-MFMA contexts only).  The X-engine of
 * Section 2.3 runs once per array; a batch correlates up to XCORR_MAX_BATCH
 * arrays of uneven N, F and sample count in one kernel launch.  Where every
 * array has N a multiple of 16 and a 16-byte-aligned input, each array's
 * region shapes are jobs of the three-product kernel that every work-group
 * walks in turn; otherwise one kernel drains a work queue of (array,
 * channel, region) items.  Results, the integration bookkeeping and the
 * dumps stay per context (xcorr_dump).
 *
 * xcorr_batch_query: device bytes the batch needs (the work-queue counters).
 * xcorr_batch_init : ctxs[0..n) are borrowed (they must outlive the batch and
 *   keep their workspaces); d_workspace (>= the queried size, 256-byte
 *   aligned) is borrowed until xcorr_batch_destroy and is initialised here
 *   with a synchronous kernel on the null stream.  Each array keeps its own
 *   region plan when its tile is 2, 3, 4, or 6 with N <= 192; other tiles are
 *   replaced by whichever of 2, 3, 4 pads least (xcorr_batch_tiles reports
 *   the choice).
 *   Errors: XCORR_E_INVAL (n outside 1..XCORR_MAX_BATCH, a NULL or repeated
 *   context, a context that is not 4-bit int8-MFMA), XCORR_E_NOMEM, XCORR_E_HIP.
 * xcorr_batch_ingest: d_volts[a] = [n_samples[a]][F_a][N_a] for array a;
 *   n_samples[a] = 0 leaves array a out of this ingest.  seqs may be NULL (each
 *   array's sequence then continues without a gap).  Checks, before anything
 *   is enqueued: XCORR_E_INVAL (NULL arrays, negative counts, all counts 0),
 *   XCORR_E_OVERFLOW if any array would pass its max_samples_per_dump.  Every
 *   launch leaves the queue counters as it found them (the three-product
 *   launch uses none), so an ingest can be captured in a HIP graph and
 *   replayed; a replay repeats the overwrite /
 *   accumulate choice made at capture, so capture whole integrations (the
 *   first ingest after a dump through the dump).  Launches of one batch must
 *   not overlap (one stream at a time).
 */
#define XCORR_MAX_BATCH 16
int xcorr_batch_query(xcorr_ctx *const *ctxs, int n, size_t *workspace_bytes);
int xcorr_batch_init(xcorr_ctx *const *ctxs, int n, void *d_workspace, size_t ws_bytes, xcorr_batch **out);
int xcorr_batch_ingest(xcorr_batch *b, const void *const *d_volts, const int64_t *n_samples,
                       const uint64_t *seqs, void *stream);
int xcorr_batch_tiles(const xcorr_batch *b, int32_t *tiles);
int xcorr_batch_destroy(xcorr_batch *b);

/*
 * Autotuner (the triangle-tile choice of the work split; the paper's X-engine
 * runs a fixed tiling, Section 2.3).  xcorr_autotune times every supported
 * tile of an MFMA-path config on the kernel a context of that config runs
 * (xcorr_autotune_kernel names it), over a synthetic block of 2048 samples
 * (a fixed hash pattern written into the scratch), and returns the fastest
 * in *best_tile.  xcorr_autotune_batch does the same on the batched
 * persistent kernel, with the config as its only array, over the tiles that
 * kernel carries (2, 3, 4, and 6 when N <= 192).  When $XCORR_TUNE_CACHE
 * names a file, the line "bits N F path tile kernel" is appended to it;
 * xcorr_init with tile = 0 (and xcorr_batch_init, for each member) then uses
 * the last line of that config whose kernel is the one it will run; lines
 * timed on another kernel are ignored.  xcorr_plan_tile (pure host) reports
 * the tile xcorr_init (batch = 0) or xcorr_batch_init (batch = 1) would use
 * and whether it came from the cache.  The tuners block until their timing
 * runs on `stream` have finished.  xcorr_autotune_query gives the scratch
 * size (accumulators + input block + queue counters).
 * Errors: as xcorr_query, XCORR_E_INVAL for the plain path, a NULL output,
 * or (batch) a config that is not 4+4-bit int8 MFMA; XCORR_E_NOMEM for
 * missing or short scratch; XCORR_E_HIP.
 */
int xcorr_autotune_query(const xcorr_config *cfg, size_t *scratch_bytes);
int xcorr_autotune(const xcorr_config *cfg, void *d_scratch, size_t scratch_bytes, void *stream,
                   int32_t *best_tile);
int xcorr_autotune_batch(const xcorr_config *cfg, void *d_scratch, size_t scratch_bytes, void *stream,
                         int32_t *best_tile);
int xcorr_autotune_kernel(const xcorr_config *cfg, int32_t batch, char *name, size_t len);
int xcorr_plan_tile(const xcorr_config *cfg, int32_t batch, int32_t *tile, int32_t *from_cache);
/*
 * Streaming loop (the X-engine node's packet ring feeding the correlator,
 * which integrates and hands each integration to an output stage: Section
 * 2.3).  A pipe wraps one context: each xcorr_pipe_push submits one block of
 * block_samples samples; a host block (on_host = 1, pinned host memory) is
 * copied on `copy_stream` into the next of n_slots device ring slots (the slot
 * is reused once its previous ingest has finished), then ingested on
 * `compute_stream` after the copy; a device block (on_host = 0) is ingested
 * in place.  Every dump_every-th block the integration is dumped into d_out
 * (required on that push, *dumped = 1).  Two latencies are kept.  The service
 * time of each launch record (one block, or a held group), from the start of
 * its transfer (host blocks) or of its ingest (device blocks) to the end of
 * its ingest (and dump), comes from HIP events.  The block latency, per
 * block, runs from the host clock at its xcorr_pipe_push call to the end of
 * the ingest that holds it, so it includes queueing behind earlier blocks; a
 * GPU event maps onto the host clock through an anchor event taken at init
 * and at each xcorr_pipe_reset_latency (its uncertainty is reported).
 * xcorr_pipe_stats reports nearest-rank p50 / p99 and the maximum of both
 * over the reaped records (xcorr_pipe_drain waits for every block in
 * flight) and `held`, the device blocks whose ingest is not enqueued yet
 * (the newest `held` pushes).  Calls are
 * asynchronous except that at most max(8, 4 n_slots) blocks are in flight:
 * a push beyond that waits for the oldest.  The host block, d_out and device
 * blocks must stay valid until the streams pass them.
 *
 * xcorr_pipe_query : ring bytes (n_slots slots of 256-byte-rounded blocks).
 * xcorr_pipe_init  : ctx borrowed; d_ring may be NULL for device blocks only;
 *   dump_every = 0: dumps only through xcorr_pipe_dump.
 *   Errors: XCORR_E_INVAL, XCORR_E_NOMEM (short or misaligned ring),
 *   XCORR_E_OVERFLOW (dump_every * block_samples > max_samples_per_dump).
 *
 * Admission by memory: xcorr_admit walks cfgs[0..n) in order and admits an
 * array (admitted[a] = 1) while the running device footprint (workspace +
 * dump buffer + n_slots[a] ring slots of block_samples[a] samples; NULL
 * arrays count 0) stays within budget_bytes; *used_bytes = the admitted
 * total.  Pure host.
 */
typedef struct {
    int64_t blocks, dumps, latencies;
    double p50_ms, p99_ms, max_ms, mean_ms;   /* service time per record */
    int64_t held;                /* device blocks pushed but not yet ingested */
    int64_t submit_latencies;    /* blocks with a submit-to-done latency */
    double submit_p50_ms, submit_p99_ms, submit_max_ms;
    double clock_anchor_err_ms;  /* uncertainty of the host-clock anchor */
} xcorr_pipe_stats_t;

int xcorr_pipe_query(const xcorr_ctx *ctx, int n_slots, int64_t block_samples, size_t *ring_bytes);
int xcorr_pipe_init(xcorr_ctx *ctx, int n_slots, int64_t block_samples, int64_t dump_every, void *d_ring,
                    size_t ring_bytes, void *copy_stream, void *compute_stream, xcorr_pipe **out);
int xcorr_pipe_push(xcorr_pipe *p, const void *block, int on_host, uint64_t seq, void *d_out, int *dumped);
int xcorr_pipe_drain(xcorr_pipe *p);
int xcorr_pipe_stats(const xcorr_pipe *p, xcorr_pipe_stats_t *out);
int xcorr_pipe_reset_latency(xcorr_pipe *p);
/* Device blocks: hold up to `fuse` (1..8, default 1) pushed blocks and ingest
 * them with xcorr_ingest_blocks when the group is full, an integration ends
 * or the pipe is drained; a latency record then covers the group, from its
 * ingest's start.  Host blocks are not held.  Held blocks must stay valid
 * until they are ingested; call xcorr_pipe_drain before xcorr_pipe_destroy
 * (destroy drops held blocks). */
int xcorr_pipe_set_fuse(xcorr_pipe *p, int fuse);
/* End the integration now (sequence-aligned integrations, e.g. on an
 * XCORR_EV_DUMP event): ingest any held blocks, dump into d_out on
 * compute_stream as xcorr_dump does (n_integrated / n_gaps may be NULL) and
 * restart the count of dump_every.  With dump_every = 0 at init the pipe never
 * dumps by itself; an integration is then bounded only by the context's
 * max_samples_per_dump (an ingest past it fails with XCORR_E_OVERFLOW).
 * Errors: XCORR_E_INVAL (NULL pipe or d_out), as xcorr_dump. */
int xcorr_pipe_dump(xcorr_pipe *p, void *d_out, int64_t *n_integrated, uint64_t *n_gaps);
int xcorr_pipe_destroy(xcorr_pipe *p);
int xcorr_admit(const xcorr_config *cfgs, int n, const int64_t *block_samples, const int32_t *n_slots,
                size_t budget_bytes, int32_t *admitted, size_t *used_bytes);

/*
 * Block reassembly by sequence number (the nodes' packet counter; all nodes
 * start integrating at the same counter value so that their integrations
 * cover the same span and the calibration noise source's on/off pattern
 * falls inside one integration: Sections 2.2 and 2.3).  Pure host code, no
 * device call; a reorder object is not thread-safe.
 *
 * Integration j covers sequence numbers [seq_origin + j*blocks_per_dump,
 * seq_origin + (j+1)*blocks_per_dump).  xcorr_reorder_push takes one arriving
 * block (`block` is an opaque handle, returned untouched) and writes to
 * events[0..*n_events) what that arrival settles, in sequence order:
 *   XCORR_EV_BLOCK  release block `seq` (feed it to the correlator now);
 *   XCORR_EV_GAP    sequence numbers [seq, seq + n_blocks) are missing (one
 *                   run never crosses an integration boundary);
 *   XCORR_EV_DUMP   integration `integration` (first sequence number `seq`)
 *                   is complete: n_blocks arrived, n_missing did not; valid =
 *                   (n_missing <= max_missing).  Integrations of which no
 *                   block arrived end without any event.
 * A hole is declared missing once a block `window` or more sequence numbers
 * beyond it has arrived (window 0: no reordering).  Blocks before
 * seq_origin, blocks whose sequence number is already settled (late) and
 * duplicates of a held block are dropped and counted.  xcorr_reorder_flush
 * settles everything held (holes between held blocks become gaps) and, with
 * to_boundary != 0, declares the rest of the current integration missing so
 * that it ends.  `events` must hold xcorr_reorder_max_events(window) entries
 * (4 window + 8), the most one call can produce.
 * Errors: XCORR_E_INVAL (NULL arguments; blocks_per_dump outside [1, 2^30],
 * window outside [0, 2^20], max_missing < 0), XCORR_E_NOMEM (events too
 * short, checked before any state changes; host allocation).
 */
typedef struct xcorr_reorder xcorr_reorder;
enum { XCORR_EV_BLOCK = 1, XCORR_EV_GAP = 2, XCORR_EV_DUMP = 3 };
typedef struct {
    int32_t kind;        /* XCORR_EV_* */
    int32_t n_blocks;    /* BLOCK: 1; GAP: run length; DUMP: blocks that arrived */
    int32_t n_missing;   /* DUMP: blocks declared missing */
    int32_t valid;       /* DUMP: n_missing <= max_missing */
    uint64_t seq;        /* BLOCK, GAP: first sequence number; DUMP: the integration's first */
    int64_t integration; /* integration index of seq */
    const void *block;   /* BLOCK: the handle given to xcorr_reorder_push */
} xcorr_event;
typedef struct {
    int64_t received, released, missing, late, duplicate, before_origin, held;
    int64_t integrations, invalid_integrations, empty_integrations;
    uint64_t next_seq;   /* first sequence number not yet settled */
} xcorr_reorder_stats_t;

int32_t xcorr_reorder_max_events(int32_t window);
int xcorr_reorder_init(int64_t blocks_per_dump, int32_t window, int32_t max_missing, uint64_t seq_origin,
                       xcorr_reorder **out);
int xcorr_reorder_push(xcorr_reorder *r, uint64_t seq, const void *block, xcorr_event *events, int32_t max_events,
                       int32_t *n_events);
int xcorr_reorder_flush(xcorr_reorder *r, int32_t to_boundary, xcorr_event *events, int32_t max_events,
                        int32_t *n_events);
int xcorr_reorder_stats(const xcorr_reorder *r, xcorr_reorder_stats_t *out);
int xcorr_reorder_destroy(xcorr_reorder *r);

/*
 * One integration without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): as a context created from *cfg with tile = the
 * config's (0: the built-in choice; the tune cache is not read), followed by
 * one xcorr_ingest_dump(n_samples) into d_out, with no context, no workspace
 * and no allocation.  An integration that needs running sums (more samples
 * than one 4+4-bit int8-MFMA launch takes, 130,560, or any 8+8-bit or plain
 * integration) keeps them in a library-held device array of
 * XCORR_STATIC_SCRATCH_BYTES per GPU, held until the process ends; configs
 * whose sums (F*P*2*4 bytes, rounded up to 256) exceed it are refused with
 * XCORR_E_NOMEM before anything is enqueued.  The first launch of an
 * integration overwrites the array, so nothing needs clearing; it keeps the
 * last call's contents.  Calls that overlap on one GPU (two streams, or two
 * host threads) share the array and race.  Errors: as xcorr_query and
 * xcorr_ingest_dump, XCORR_E_NOMEM as above, XCORR_E_HIP if the array's
 * address cannot be looked up.
 */
#define XCORR_STATIC_SCRATCH_BYTES (16u << 20)
int xcorr_correlate_static(const xcorr_config *cfg, const void *d_volts, int64_t n_samples, void *d_out,
                           int64_t *n_integrated, void *stream);

/*
 * Calibrator-noise-source gating aligned to integrations (paper Section 2.5,
 * "CNS control module"): the CNS must switch on and off so that each
 * on-window falls wholly inside one integration.  Sequence numbers are the
 * block counters of xcorr_pipe / xcorr_reorder (the paper's MCNT, one per
 * block); integration j covers [seq_origin + j * blocks_per_dump,
 * seq_origin + (j + 1) * blocks_per_dump), as in xcorr_reorder.  Host only.
 *
 * xcorr_cns_plan_make: from the current sequence number `now` and a lead
 * time `lead` (the host's latency for programming the F-engine), the CNS
 * first switches on at first_on, the first integration start at or after
 * now + lead; it stays on for on_blocks (1 .. blocks_per_dump) sequence
 * numbers and repeats every period_dumps integrations (period_blocks
 * sequence numbers): first_on and period_blocks are the two values the
 * F-engine's counter block takes.  Errors: XCORR_E_INVAL for a NULL plan,
 * blocks_per_dump or period_dumps outside [1, 2^30], on_blocks outside
 * [1, blocks_per_dump], or a sequence number beyond 2^62.
 * xcorr_cns_is_on: 1 if the CNS is on at sequence number seq, else 0.
 * xcorr_cns_integration: 1 if integration j holds a CNS on-window (which
 * then starts at its first block), else 0.
 */
typedef struct {
    uint64_t seq_origin;
    int64_t blocks_per_dump;
    int64_t period_dumps;
    int64_t on_blocks;
    uint64_t first_on;          /* first sequence number with the CNS on */
    int64_t first_integration;  /* the integration that starts at first_on */
    int64_t period_blocks;      /* period_dumps * blocks_per_dump */
} xcorr_cns_plan;
int xcorr_cns_plan_make(uint64_t now, uint64_t lead, uint64_t seq_origin, int64_t blocks_per_dump,
                        int64_t period_dumps, int64_t on_blocks, xcorr_cns_plan *out);
int xcorr_cns_is_on(const xcorr_cns_plan *p, uint64_t seq);
int xcorr_cns_integration(const xcorr_cns_plan *p, int64_t j);

/*
 * F-engine front end (paper Section 2.2, "F-engine"): raw ADC samples ->
 * polyphase filter bank -> 1024 channels -> EQ -> 4+4-bit codes in the
 * X-engine's input order.  Fixed shape: 2048-point filter bank (real FFT,
 * the first 1024 bins kept), 4 taps.
 *
 * xcorr_pfb_prototype (host only): the library's prototype filter,
 * h[n] = w[n] sinc(n / n_points - taps / 2), n < taps * n_points, w the
 * symmetric Hamming window 0.54 - 0.46 cos(2 pi n / (taps n_points - 1)),
 * written as float32 to h_out (caller-owned, taps * n_points entries).
 * Errors: XCORR_E_INVAL for n_points < 2, taps < 1 or a NULL pointer.
 *
 * xcorr_fengine (async on `stream`): d_adc holds int8 ADC codes [N][S] (input
 * i's samples at i * S, S = n_samples); spectrum m (m < n_spectra) filters
 * samples [2048 m, 2048 (m + 4)) as y[q] = sum_k h[2048 k + q] x[2048 (m + k) + q]
 * with d_coeffs the 8192 prototype coefficients (float32), takes the real
 * FFT of y, multiplies channel c of input i by d_gains[i * 1024 + c]
 * (float32 EQ gain), rounds each part half to even and clips to [-8, 7], and
 * writes the packed byte (real part in the high nibble) to
 * d_out[(m * 1024 + c) * N + i]: uint8 [n_spectra][1024][N], the layout
 * xcorr_ingest reads.  Arithmetic in float32.  Requirements (else
 * XCORR_E_INVAL, nothing enqueued): N a positive multiple of 16; S a
 * multiple of 16 and at least 8192; 1 <= n_spectra <= S / 2048 - 3; d_adc,
 * d_coeffs, d_gains and d_out 16-byte aligned.  XCORR_E_HIP if the launch
 * fails.  All buffers are caller-owned and must stay valid until the stream
 * passes this call.
 *
 * xcorr_pfb_spectra: the same filter bank without EQ and requantisation;
 * writes the complex spectra as float32 (re, im) pairs to
 * d_out[((i * n_spectra + m) * 1024 + c) * 2 + {0, 1}].  Same requirements.
 */
int xcorr_pfb_prototype(int32_t n_points, int32_t taps, float *h_out);
int xcorr_fengine(const void *d_adc, int64_t n_samples, int32_t n_inputs, const float *d_coeffs,
                  const float *d_gains, int64_t n_spectra, void *d_out, void *stream);
int xcorr_pfb_spectra(const void *d_adc, int64_t n_samples, int32_t n_inputs, const float *d_coeffs,
                      int64_t n_spectra, void *d_out, void *stream);

/*
 * Full-Stokes visibilities of dual-polarisation feeds (paper Section 1:
 * full-Stokes output; Section 3.3: polarisations X north-south and Y
 * east-west).  d_vis holds a dump of N = 2 Nf inputs, int32 [F][P][2]
 * (xcorr_dump's layout), input 2 f + pol being feed f's polarisation pol
 * (0 = X, 1 = Y).  For feeds a >= b, with XX = V(2a, 2b), YY = V(2a+1, 2b+1),
 * XY = V(2a, 2b+1) (conj V(2a+1, 2a) when a = b) and YX = V(2a+1, 2b):
 * I = XX + YY, Q = XX - YY, U = XY + YX, V = -i (XY - YX), written exactly
 * as int64 (re, im) to d_out [F][Nf (Nf + 1) / 2][4][2], feed pair
 * a (a + 1) / 2 + b, Stokes order I, Q, U, V.  Async on `stream`; buffers
 * caller-owned.  Errors: XCORR_E_INVAL for an odd or < 2 input count,
 * n_chans outside [1, 65535], NULL or misaligned pointers (d_vis 8 bytes,
 * d_out 16 bytes); XCORR_E_HIP if the launch fails.
 */
int xcorr_stokes(const void *d_vis, int32_t n_inputs, int32_t n_chans, void *d_out, void *stream);

/*
 * Hardware ceilings for the roofline of a benchmark (no correlation is
 * computed).  Enqueued on `stream`; the caller times them with events.
 *   XCORR_CEILING_MFMA_I8: one work-group of 8 waves per compute unit (two
 *     per SIMD, as the correlation kernel) issues `iters` rounds of 16
 *     independent 32x32x32 int8 MFMAs per wave on operands read from d_volts
 *     (voltage bytes, at least 4096 of them, so the multipliers toggle as on
 *     real data); *ops = int8 ops done (2 per multiply-add).
 *   XCORR_CEILING_STREAM: the [n_samples][n_chans][n_inputs] packed input of
 *     a 4+4-bit launch is streamed into LDS with the correlation kernel's
 *     grid, channel mapping, 64-sample chunks, 16-byte LDS-DMA loads and
 *     cache policy, and nothing else is done with it; *ops = bytes read.
 * d_out receives one int32 checksum per thread: out_ints must be at least
 * 512 x (compute units).  Errors: XCORR_E_INVAL for an unknown kind, NULL or
 * unaligned (16 B) pointers, n_inputs outside 16..256 or not a multiple of
 * 16, 64 * n_chans * n_inputs >= 2^31 - 16, iters < 1 (MFMA) or a short
 * d_out; XCORR_E_HIP if the launch fails.
 */
#define XCORR_CEILING_MFMA_I8 0
#define XCORR_CEILING_STREAM 1
int xcorr_ceiling(int32_t kind, const void *d_volts, int64_t n_samples, int32_t n_chans, int32_t n_inputs,
                  int64_t iters, void *d_out, int64_t out_ints, double *ops, void *stream);

const char *xcorr_strerror(int code);
/* Detail of the last XCORR_E_HIP / XCORR_E_DEVICE on this thread. */
const char *xcorr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* XCORR_H */
