// Block reassembly by sequence number ahead of the streaming loop: blocks
// that arrive out of order are released in order, blocks that never arrive
// are declared missing once a window of later blocks has been seen, and
// integrations are cut at fixed sequence numbers, the same for every node
// that uses the same origin.
//
// The paper's nodes receive packets carrying a packet counter and start
// integrating at the same counter value, so that every node's integrations
// cover the same time span and the calibration noise source's on/off pattern
// falls inside one integration (Sections 2.2 and 2.3).  Pure host code: no
// device call, no allocation after init beyond the hold map.
#include "xcorr.h"
#include "xcorr_internal.h"

#include <cstdint>
#include <map>
#include <new>

using xc::api_error;

struct xcorr_reorder {
    int64_t k = 0;              // blocks per integration
    int32_t window = 0;         // later blocks seen before a hole is declared missing
    int32_t max_missing = 0;    // an integration with more missing blocks is flagged invalid
    uint64_t origin = 0;        // first sequence number of integration 0
    uint64_t next = 0;          // next sequence number to release or declare missing
    std::map<uint64_t, const void *> held;
    int64_t cur_blocks = 0, cur_missing = 0;   // of the integration `next` belongs to
    xcorr_reorder_stats_t st{};
};

namespace {

int64_t integration_of(const xcorr_reorder *r, uint64_t seq) { return (int64_t)((seq - r->origin) / r->k); }
uint64_t integration_begin(const xcorr_reorder *r, int64_t j) { return r->origin + (uint64_t)j * (uint64_t)r->k; }

// Events of one call.  xcorr_reorder_max_events bounds what one call can
// produce (per released block one BLOCK, at most two GAP runs before it and
// one DUMP after it); the capacity check only guards that bound.
struct Out {
    xcorr_event *ev;
    int32_t cap;
    int32_t n = 0;
    bool overflow = false;
    void add(const xcorr_event &e)
    {
        if (n < cap)
            ev[n++] = e;
        else
            overflow = true;
    }
};

// The integration of `next - 1` has just ended: report it if any of its
// blocks arrived (integrations with none are skipped without an event).
void close_integration(xcorr_reorder *r, Out &o)
{
    const int64_t j = integration_of(r, r->next - 1);
    if (r->cur_blocks > 0) {
        xcorr_event e{};
        e.kind = XCORR_EV_DUMP;
        e.seq = integration_begin(r, j);
        e.integration = j;
        e.n_blocks = (int32_t)r->cur_blocks;
        e.n_missing = (int32_t)r->cur_missing;
        e.valid = r->cur_missing <= r->max_missing;
        o.add(e);
        ++r->st.integrations;
        if (!e.valid)
            ++r->st.invalid_integrations;
    } else {
        ++r->st.empty_integrations;
    }
    r->cur_blocks = r->cur_missing = 0;
}

// Release the held block at `next`, or declare `next` and every following
// unheld sequence number up to `limit` (exclusive) missing as one run that
// ends at an integration boundary at the latest.
void advance_one(xcorr_reorder *r, uint64_t limit, Out &o)
{
    auto it = r->held.find(r->next);
    if (it != r->held.end()) {
        xcorr_event e{};
        e.kind = XCORR_EV_BLOCK;
        e.seq = r->next;
        e.integration = integration_of(r, r->next);
        e.n_blocks = 1;
        e.block = it->second;
        o.add(e);
        r->held.erase(it);
        ++r->st.released;
        ++r->cur_blocks;
        ++r->next;
    } else {
        // the run stops at the next held block, at `limit` and at the end of
        // this integration
        const uint64_t end_of_int = integration_begin(r, integration_of(r, r->next) + 1);
        uint64_t stop = limit < end_of_int ? limit : end_of_int;
        auto nx = r->held.lower_bound(r->next);
        if (nx != r->held.end() && nx->first < stop)
            stop = nx->first;
        const uint64_t n = stop - r->next;
        xcorr_event e{};
        e.kind = XCORR_EV_GAP;
        e.seq = r->next;
        e.integration = integration_of(r, r->next);
        e.n_blocks = (int32_t)n;
        o.add(e);
        r->st.missing += (int64_t)n;
        r->cur_missing += (int64_t)n;
        r->next = stop;
    }
    if ((r->next - r->origin) % (uint64_t)r->k == 0)
        close_integration(r, o);
}

// At an integration boundary, skip the whole integrations before the one
// holding `target` (nothing is held before `target`): they are missing
// entirely and produce no event.
void skip_empty(xcorr_reorder *r, uint64_t target)
{
    if ((r->next - r->origin) % (uint64_t)r->k != 0)
        return;
    const int64_t jt = integration_of(r, target), jn = integration_of(r, r->next);
    if (jt > jn) {
        r->st.missing += (jt - jn) * r->k;
        r->st.empty_integrations += jt - jn;
        r->next = integration_begin(r, jt);
    }
}

// Settle every sequence number below `limit`: release what is held, declare
// the rest missing.
void settle(xcorr_reorder *r, uint64_t limit, Out &o)
{
    while (r->next < limit) {
        uint64_t target = limit;
        auto nx = r->held.lower_bound(r->next);
        if (nx != r->held.end() && nx->first < target)
            target = nx->first;
        skip_empty(r, target);
        if (r->next < limit)
            advance_one(r, limit, o);
    }
}

}  // namespace

extern "C" {

int32_t xcorr_reorder_max_events(int32_t window) { return window < 0 ? 0 : 4 * window + 8; }

int xcorr_reorder_init(int64_t blocks_per_dump, int32_t window, int32_t max_missing, uint64_t seq_origin,
                       xcorr_reorder **out)
{
    if (!out || blocks_per_dump < 1 || blocks_per_dump > (1 << 30) || window < 0 || window > (1 << 20) ||
        max_missing < 0)
        return api_error(XCORR_E_INVAL, "out is NULL, blocks_per_dump outside [1, 2^30], window outside "
                                        "[0, 2^20] or max_missing < 0");
    xcorr_reorder *r = new (std::nothrow) xcorr_reorder();
    if (!r)
        return api_error(XCORR_E_NOMEM, "host allocation failed");
    r->k = blocks_per_dump;
    r->window = window;
    r->max_missing = max_missing;
    r->origin = r->next = seq_origin;
    *out = r;
    return XCORR_OK;
}

int xcorr_reorder_push(xcorr_reorder *r, uint64_t seq, const void *block, xcorr_event *events, int32_t max_events,
                       int32_t *n_events)
{
    if (!r || !events || !n_events)
        return api_error(XCORR_E_INVAL, "reorder, events or n_events is NULL");
    if (max_events < xcorr_reorder_max_events(r->window))
        return api_error(XCORR_E_NOMEM, "events holds fewer than xcorr_reorder_max_events(window) entries");
    Out o{events, max_events};
    ++r->st.received;
    if (seq < r->origin) {
        ++r->st.before_origin;
    } else if (seq < r->next) {
        ++r->st.late;
    } else if (r->held.count(seq)) {
        ++r->st.duplicate;
    } else {
        r->held.emplace(seq, block);
        // a block `window` or more ahead of `next` settles every earlier hole
        if (seq - r->next >= (uint64_t)r->window + 1)
            settle(r, seq - (uint64_t)r->window, o);
        while (!r->held.empty() && r->held.begin()->first == r->next)
            advance_one(r, r->next + 1, o);
    }
    r->st.held = (int64_t)r->held.size();
    *n_events = o.n;
    return o.overflow ? api_error(XCORR_E_NOMEM, "event bound exceeded") : XCORR_OK;
}

int xcorr_reorder_flush(xcorr_reorder *r, int32_t to_boundary, xcorr_event *events, int32_t max_events,
                        int32_t *n_events)
{
    if (!r || !events || !n_events)
        return api_error(XCORR_E_INVAL, "reorder, events or n_events is NULL");
    if (max_events < xcorr_reorder_max_events(r->window))
        return api_error(XCORR_E_NOMEM, "events holds fewer than xcorr_reorder_max_events(window) entries");
    Out o{events, max_events};
    if (!r->held.empty())
        settle(r, r->held.rbegin()->first + 1, o);
    if (to_boundary && (r->next - r->origin) % (uint64_t)r->k != 0)
        settle(r, integration_begin(r, integration_of(r, r->next) + 1), o);
    r->st.held = 0;
    *n_events = o.n;
    return o.overflow ? api_error(XCORR_E_NOMEM, "event bound exceeded") : XCORR_OK;
}

int xcorr_reorder_stats(const xcorr_reorder *r, xcorr_reorder_stats_t *out)
{
    if (!r || !out)
        return api_error(XCORR_E_INVAL, "reorder or out is NULL");
    *out = r->st;
    out->next_seq = r->next;
    return XCORR_OK;
}

int xcorr_reorder_destroy(xcorr_reorder *r)
{
    delete r;
    return XCORR_OK;
}

}  // extern "C"
