// Streaming runtime of the C ABI: a ring of device block slots between a
// copy stream (host -> device transfers) and a compute stream (ingest, and a
// dump every `dump_every` blocks or on request), with per-block latency taken
// from HIP events; plus admission of arrays against a device-memory budget.
//
// The paper's X-engine node runs a ring buffer of received packets feeding
// the correlator, which integrates and hands each integration to an output
// stage (Section 2.3); this file is that loop around one context.  The
// library allocates no device memory: the ring is the caller's.
#include "xcorr.h"
#include "xcorr_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <new>
#include <string>
#include <vector>

namespace {

using xc::api_error;

int hip_err(hipError_t e, const char *what)
{
    return api_error(XCORR_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// One latency record: a launch group (one block, or up to 8 held device
// blocks ingested together) between two events on the compute stream, plus
// the host clock at which each of its blocks was submitted.
struct Record {
    hipEvent_t begin, end;
    int nblk;
    double submit_s[xc::kMaxFusedBlocks];
};

double host_now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct xcorr_pipe {
    xcorr_ctx *ctx = nullptr;
    int n_slots = 0;
    int64_t block_samples = 0;
    int64_t dump_every = 0;
    size_t block_bytes = 0;
    uint8_t *ring = nullptr;
    hipStream_t copy = nullptr, compute = nullptr;
    std::vector<hipEvent_t> copied, consumed;   // per slot
    std::vector<bool> slot_used;
    std::deque<Record> pending;                 // latency records in flight
    std::vector<Record> spare;
    std::vector<float> lat_ms;         // service time per record
    std::vector<float> submit_ms;      // host submit -> end of ingest, per block
    int64_t blocks = 0, dumps = 0, since_dump = 0, host_blocks = 0;
    size_t max_pending = 0;
    int fuse = 1;                      // device blocks ingested per group
    std::vector<const void *> held;    // device blocks pushed, not yet ingested
    std::vector<double> held_submit;   // their host submit times
    uint64_t held_seq0 = 0;
    // clock anchor: an event on the idle compute stream and the host time at
    // which it ran (midpoint of record and synchronise), so that a GPU event
    // maps onto the host clock as anchor_s + elapsed(anchor, event)
    hipEvent_t anchor = nullptr;
    double anchor_s = 0.0, anchor_err_s = 0.0;
    bool have_anchor = false;
};

namespace {

void destroy_events(xcorr_pipe *p)
{
    for (auto e : p->copied)
        if (e)
            (void)hipEventDestroy(e);
    for (auto e : p->consumed)
        if (e)
            (void)hipEventDestroy(e);
    for (auto &r : p->pending) {
        (void)hipEventDestroy(r.begin);
        (void)hipEventDestroy(r.end);
    }
    for (auto &r : p->spare) {
        (void)hipEventDestroy(r.begin);
        (void)hipEventDestroy(r.end);
    }
    if (p->anchor)
        (void)hipEventDestroy(p->anchor);
    p->anchor = nullptr;
    p->have_anchor = false;
    p->copied.clear();
    p->consumed.clear();
    p->pending.clear();
    p->spare.clear();
}

// Set the clock anchor: record an event on the compute stream and wait for
// it; the event ran between the host times before the record and after the
// wait.  Work queued ahead of it (on this stream, or on another stream that
// shares its hardware queue) widens that window, so the anchor is taken
// again, up to 8 times, until the window is below 200 us; the event keeps
// the last recording, whose window is used and whose half-width is reported.
int set_anchor(xcorr_pipe *p)
{
    hipError_t e = hipSuccess;
    if (!p->anchor)
        e = hipEventCreate(&p->anchor);
    double a = 0.0, b = 0.0;
    for (int k = 0; k < 8 && e == hipSuccess; ++k) {
        a = host_now_s();
        e = hipEventRecord(p->anchor, p->compute);
        if (e == hipSuccess)
            e = hipEventSynchronize(p->anchor);
        b = host_now_s();
        if (b - a < 200e-6)
            break;
    }
    if (e != hipSuccess)
        return hip_err(e, "clock anchor event");
    p->anchor_s = 0.5 * (a + b);
    p->anchor_err_s = 0.5 * (b - a);
    p->have_anchor = true;
    return XCORR_OK;
}

// Wait for the oldest latency record and keep its durations: the service
// time of the record and, per block, the time from the host submit to the
// end of its ingest.
int reap_one(xcorr_pipe *p)
{
    Record r = p->pending.front();
    p->pending.pop_front();
    hipError_t e = hipEventSynchronize(r.end);
    float ms = 0.f, since_anchor = 0.f;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&ms, r.begin, r.end);
    if (e == hipSuccess && p->have_anchor)
        e = hipEventElapsedTime(&since_anchor, p->anchor, r.end);
    p->spare.push_back(r);
    if (e != hipSuccess)
        return hip_err(e, "latency event");
    p->lat_ms.push_back(ms);
    if (p->have_anchor) {
        const double done_s = p->anchor_s + 1e-3 * since_anchor;
        for (int k = 0; k < r.nblk; ++k)
            p->submit_ms.push_back((float)std::max(0.0, 1e3 * (done_s - r.submit_s[k])));
    }
    return XCORR_OK;
}

int get_record(xcorr_pipe *p, Record *out)
{
    if (p->pending.size() >= p->max_pending) {
        const int rc = reap_one(p);
        if (rc)
            return rc;
    }
    if (!p->spare.empty()) {
        *out = p->spare.back();
        p->spare.pop_back();
        return XCORR_OK;
    }
    hipError_t e = hipEventCreate(&out->begin);
    if (e == hipSuccess) {
        e = hipEventCreate(&out->end);
        if (e != hipSuccess)
            (void)hipEventDestroy(out->begin);
    }
    return e == hipSuccess ? XCORR_OK : hip_err(e, "hipEventCreate");
}

size_t block_bytes_of(const xcorr_ctx *ctx, int64_t block_samples)
{
    const xc::CtxShape c = xc::ctx_shape(ctx);
    return (size_t)block_samples * c.n_chans * c.n_inputs * (c.sample_bits == 4 ? 1 : 2);
}

size_t round256(size_t x) { return (x + 255) / 256 * 256; }

// Ingest the held device blocks as one group (and dump when asked), under one
// latency record.
int flush_held(xcorr_pipe *p, void *d_out, bool dump, int64_t *n_integrated = nullptr, uint64_t *n_gaps = nullptr)
{
    if (p->held.empty() && !dump)
        return XCORR_OK;
    Record r;
    int rc = get_record(p, &r);
    if (rc)
        return rc;
    r.nblk = (int)p->held.size();
    for (int k = 0; k < r.nblk; ++k)
        r.submit_s[k] = p->held_submit[k];
    hipError_t e = hipEventRecord(r.begin, p->compute);
    if (e != hipSuccess) {
        p->spare.push_back(r);
        return hip_err(e, "hipEventRecord");
    }
    if (!p->held.empty()) {
        rc = xcorr_ingest_blocks(p->ctx, p->held.data(), (int)p->held.size(), p->block_samples, p->held_seq0,
                                 p->compute);
        p->held.clear();
        p->held_submit.clear();
    }
    if (rc == XCORR_OK && dump)
        rc = xcorr_dump(p->ctx, d_out, n_integrated, n_gaps, p->compute);
    if (rc) {
        p->spare.push_back(r);
        return rc;
    }
    e = hipEventRecord(r.end, p->compute);
    if (e != hipSuccess) {
        p->spare.push_back(r);
        return hip_err(e, "hipEventRecord");
    }
    p->pending.push_back(r);
    return XCORR_OK;
}

}  // namespace

extern "C" {

int xcorr_pipe_query(const xcorr_ctx *ctx, int n_slots, int64_t block_samples, size_t *ring_bytes)
{
    if (!ctx || n_slots < 1 || block_samples < 1)
        return api_error(XCORR_E_INVAL, "ctx is NULL, n_slots < 1 or block_samples < 1");
    if (ring_bytes)
        *ring_bytes = (size_t)n_slots * round256(block_bytes_of(ctx, block_samples));
    return XCORR_OK;
}

int xcorr_pipe_init(xcorr_ctx *ctx, int n_slots, int64_t block_samples, int64_t dump_every, void *d_ring,
                    size_t ring_bytes, void *copy_stream, void *compute_stream, xcorr_pipe **out)
{
    size_t need = 0;
    int rc = xcorr_pipe_query(ctx, n_slots, block_samples, &need);
    if (rc)
        return rc;
    if (!out || dump_every < 0)
        return api_error(XCORR_E_INVAL, "out is NULL or dump_every < 0");
    if (dump_every > xc::ctx_shape(ctx).max_samples_per_dump / block_samples)
        return api_error(XCORR_E_OVERFLOW, "dump_every blocks exceed the context's max_samples_per_dump");
    if (n_slots > 1024)
        return api_error(XCORR_E_INVAL, "at most 1024 ring slots");
    if (d_ring && ((uintptr_t)d_ring % 256 || ring_bytes < need))
        return api_error(XCORR_E_NOMEM, "ring smaller than xcorr_pipe_query's size or not 256-byte aligned");
    xcorr_pipe *p = new (std::nothrow) xcorr_pipe();
    if (!p)
        return api_error(XCORR_E_NOMEM, "host allocation failed");
    p->ctx = ctx;
    p->n_slots = n_slots;
    p->block_samples = block_samples;
    p->dump_every = dump_every;
    p->block_bytes = block_bytes_of(ctx, block_samples);
    p->ring = static_cast<uint8_t *>(d_ring);
    p->copy = reinterpret_cast<hipStream_t>(copy_stream);
    p->compute = reinterpret_cast<hipStream_t>(compute_stream);
    p->max_pending = (size_t)std::max(8, 4 * n_slots);
    p->copied.assign(n_slots, nullptr);
    p->consumed.assign(n_slots, nullptr);
    p->slot_used.assign(n_slots, false);
    for (int k = 0; k < n_slots; ++k) {
        hipError_t e = hipEventCreateWithFlags(&p->copied[k], hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&p->consumed[k], hipEventDisableTiming);
        if (e != hipSuccess) {
            destroy_events(p);
            delete p;
            return hip_err(e, "hipEventCreate");
        }
    }
    rc = set_anchor(p);
    if (rc) {
        destroy_events(p);
        delete p;
        return rc;
    }
    *out = p;
    return XCORR_OK;
}

int xcorr_pipe_push(xcorr_pipe *p, const void *block, int on_host, uint64_t seq, void *d_out, int *dumped)
{
    const double submit = host_now_s();
    if (!p || !block)
        return api_error(XCORR_E_INVAL, "pipe or block is NULL");
    if (on_host && !p->ring)
        return api_error(XCORR_E_INVAL, "host blocks need a ring");
    const bool dump_due = p->dump_every > 0 && p->since_dump + 1 >= p->dump_every;
    if (dump_due && !d_out)
        return api_error(XCORR_E_INVAL, "this block completes an integration: d_out is required");
    if (!on_host && p->fuse > 1) {
        // a group holds consecutive sequence numbers
        if (!p->held.empty() && seq != p->held_seq0 + p->held.size()) {
            const int rc = flush_held(p, nullptr, false);
            if (rc)
                return rc;
        }
        if (p->held.empty())
            p->held_seq0 = seq;
        p->held.push_back(block);
        p->held_submit.push_back(submit);
        ++p->blocks;
        ++p->since_dump;
        int rc = XCORR_OK;
        if (dump_due) {
            rc = flush_held(p, d_out, true);
            if (rc == XCORR_OK) {
                p->since_dump = 0;
                ++p->dumps;
            }
        } else if ((int)p->held.size() >= p->fuse) {
            rc = flush_held(p, nullptr, false);
        }
        if (dumped)
            *dumped = rc == XCORR_OK && dump_due;
        return rc;
    }
    if (!p->held.empty()) {   // keep the integration's order
        const int rc = flush_held(p, nullptr, false);
        if (rc)
            return rc;
    }
    Record r;
    int rc = get_record(p, &r);
    if (rc)
        return rc;
    r.nblk = 1;
    r.submit_s[0] = submit;
    hipError_t e = hipSuccess;
    const void *src = block;
    if (on_host) {
        const int k = (int)(p->host_blocks % p->n_slots);
        uint8_t *slot = p->ring + (size_t)k * round256(p->block_bytes);
        if (p->slot_used[k])
            e = hipStreamWaitEvent(p->copy, p->consumed[k], 0);   // the slot's last ingest is done
        if (e == hipSuccess)
            e = hipEventRecord(r.begin, p->copy);
        if (e == hipSuccess)
            e = hipMemcpyAsync(slot, block, p->block_bytes, hipMemcpyHostToDevice, p->copy);
        if (e == hipSuccess)
            e = hipEventRecord(p->copied[k], p->copy);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(p->compute, p->copied[k], 0);
        if (e != hipSuccess) {
            p->spare.push_back(r);
            return hip_err(e, "block transfer");
        }
        src = slot;
        rc = xcorr_ingest(p->ctx, src, p->block_samples, seq, p->compute);
        if (rc == XCORR_OK) {
            e = hipEventRecord(p->consumed[k], p->compute);
            p->slot_used[k] = true;
            ++p->host_blocks;
        }
    } else {
        e = hipEventRecord(r.begin, p->compute);
        if (e != hipSuccess) {
            p->spare.push_back(r);
            return hip_err(e, "hipEventRecord");
        }
        rc = xcorr_ingest(p->ctx, src, p->block_samples, seq, p->compute);
    }
    if (rc) {
        p->spare.push_back(r);
        return rc;
    }
    if (e != hipSuccess) {
        p->spare.push_back(r);
        return hip_err(e, "hipEventRecord");
    }
    ++p->blocks;
    ++p->since_dump;
    int did = 0;
    if (dump_due) {
        rc = xcorr_dump(p->ctx, d_out, nullptr, nullptr, p->compute);
        if (rc) {
            p->spare.push_back(r);
            return rc;
        }
        p->since_dump = 0;
        ++p->dumps;
        did = 1;
    }
    e = hipEventRecord(r.end, p->compute);
    if (e != hipSuccess) {
        p->spare.push_back(r);
        return hip_err(e, "hipEventRecord");
    }
    p->pending.push_back(r);
    if (dumped)
        *dumped = did;
    return XCORR_OK;
}

int xcorr_pipe_dump(xcorr_pipe *p, void *d_out, int64_t *n_integrated, uint64_t *n_gaps)
{
    if (!p || !d_out)
        return api_error(XCORR_E_INVAL, "pipe or d_out is NULL");
    const int rc = flush_held(p, d_out, true, n_integrated, n_gaps);
    if (rc == XCORR_OK) {
        p->since_dump = 0;
        ++p->dumps;
    }
    return rc;
}

int xcorr_pipe_set_fuse(xcorr_pipe *p, int fuse)
{
    if (!p || fuse < 1 || fuse > 8)
        return api_error(XCORR_E_INVAL, "pipe is NULL or fuse outside 1..8");
    const int rc = flush_held(p, nullptr, false);
    if (rc)
        return rc;
    p->fuse = fuse;
    return XCORR_OK;
}

int xcorr_pipe_drain(xcorr_pipe *p)
{
    if (!p)
        return api_error(XCORR_E_INVAL, "pipe is NULL");
    const int rc = flush_held(p, nullptr, false);
    if (rc)
        return rc;
    while (!p->pending.empty()) {
        const int rc = reap_one(p);
        if (rc)
            return rc;
    }
    return XCORR_OK;
}

int xcorr_pipe_stats(const xcorr_pipe *p, xcorr_pipe_stats_t *out)
{
    if (!p || !out)
        return api_error(XCORR_E_INVAL, "pipe or out is NULL");
    out->blocks = p->blocks;
    out->dumps = p->dumps;
    out->latencies = (int64_t)p->lat_ms.size();
    out->held = (int64_t)p->held.size();
    // nearest-rank percentiles, maximum and mean of a sample
    auto summarise = [](const std::vector<float> &lat, double *p50, double *p99, double *mx, double *mean) {
        *p50 = *p99 = *mx = *mean = 0.0;
        if (lat.empty())
            return;
        std::vector<float> v(lat);
        std::sort(v.begin(), v.end());
        auto rank = [&](double q) {
            const size_t k = (size_t)std::ceil(q * v.size());
            return (double)v[std::min(v.size(), std::max<size_t>(k, 1)) - 1];
        };
        *p50 = rank(0.50);
        *p99 = rank(0.99);
        *mx = v.back();
        double s = 0;
        for (float x : v)
            s += x;
        *mean = s / v.size();
    };
    summarise(p->lat_ms, &out->p50_ms, &out->p99_ms, &out->max_ms, &out->mean_ms);
    double unused_mean = 0.0;
    out->submit_latencies = (int64_t)p->submit_ms.size();
    summarise(p->submit_ms, &out->submit_p50_ms, &out->submit_p99_ms, &out->submit_max_ms, &unused_mean);
    out->clock_anchor_err_ms = 1e3 * p->anchor_err_s;
    return XCORR_OK;
}

int xcorr_pipe_reset_latency(xcorr_pipe *p)
{
    if (!p)
        return api_error(XCORR_E_INVAL, "pipe is NULL");
    int rc = xcorr_pipe_drain(p);
    p->lat_ms.clear();
    p->submit_ms.clear();
    if (rc == XCORR_OK)
        rc = set_anchor(p);   // the compute stream is idle after the drain
    return rc;
}

int xcorr_pipe_destroy(xcorr_pipe *p)
{
    if (!p)
        return api_error(XCORR_E_INVAL, "pipe is NULL");
    for (auto &r : p->pending)
        (void)hipEventSynchronize(r.end);
    for (int k = 0; k < p->n_slots; ++k)
        if (p->slot_used[k])
            (void)hipEventSynchronize(p->consumed[k]);
    destroy_events(p);
    delete p;
    return XCORR_OK;
}

int xcorr_admit(const xcorr_config *cfgs, int n, const int64_t *block_samples, const int32_t *n_slots,
                size_t budget_bytes, int32_t *admitted, size_t *used_bytes)
{
    if (!cfgs || n < 0 || !admitted)
        return api_error(XCORR_E_INVAL, "cfgs or admitted is NULL, or n < 0");
    size_t used = 0;
    for (int a = 0; a < n; ++a) {
        size_t ws = 0, outb = 0;
        const int rc = xcorr_query(&cfgs[a], &ws, &outb, nullptr);
        if (rc)
            return rc;
        const int64_t bs = block_samples ? block_samples[a] : 0;
        const int slots = n_slots ? n_slots[a] : 0;
        if (bs < 0 || slots < 0)
            return api_error(XCORR_E_INVAL, "negative block size or slot count");
        const size_t block = (size_t)bs * cfgs[a].n_chans * cfgs[a].n_inputs * (cfgs[a].sample_bits == 4 ? 1 : 2);
        const size_t need = ws + round256(outb) + (size_t)slots * round256(block);
        if (used + need <= budget_bytes) {
            used += need;
            admitted[a] = 1;
        } else {
            admitted[a] = 0;
        }
    }
    if (used_bytes)
        *used_bytes = used;
    return XCORR_OK;
}

}  // extern "C"
