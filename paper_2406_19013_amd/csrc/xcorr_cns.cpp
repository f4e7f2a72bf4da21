// Calibrator-noise-source (CNS) gating aligned to integrations (paper
// Section 2.5, "CNS control module"): the host reads the current sequence
// number, picks a future sequence number at an integration boundary for the
// CNS to switch on, and a period in sequence numbers; the F-engine then
// switches the CNS on and off by its own counter, so that each on-window falls
// wholly inside one integration.  Pure host code.
#include "xcorr.h"
#include "xcorr_internal.h"

#include <limits>

namespace {

constexpr uint64_t kMaxSeq = std::numeric_limits<uint64_t>::max() / 4;

}  // namespace

extern "C" int xcorr_cns_plan_make(uint64_t now, uint64_t lead, uint64_t seq_origin, int64_t blocks_per_dump,
                                   int64_t period_dumps, int64_t on_blocks, xcorr_cns_plan *out)
{
    using xc::api_error;
    if (!out)
        return api_error(XCORR_E_INVAL, "out is NULL");
    if (blocks_per_dump < 1 || blocks_per_dump > (1 << 30) || period_dumps < 1 || period_dumps > (1 << 30) ||
        on_blocks < 1 || on_blocks > blocks_per_dump)
        return api_error(XCORR_E_INVAL, "blocks_per_dump or period_dumps outside [1, 2^30], or on_blocks "
                                        "outside [1, blocks_per_dump]");
    if (now > kMaxSeq || lead > kMaxSeq || seq_origin > kMaxSeq)
        return api_error(XCORR_E_INVAL, "sequence numbers beyond 2^62");
    const uint64_t k = (uint64_t)blocks_per_dump;
    const uint64_t earliest = now + lead;
    // the first integration start at or after `earliest`
    uint64_t j = 0;
    if (earliest > seq_origin)
        j = (earliest - seq_origin + k - 1) / k;
    xcorr_cns_plan p{};
    p.seq_origin = seq_origin;
    p.blocks_per_dump = blocks_per_dump;
    p.period_dumps = period_dumps;
    p.on_blocks = on_blocks;
    p.first_on = seq_origin + j * k;
    p.first_integration = (int64_t)j;
    p.period_blocks = period_dumps * blocks_per_dump;
    *out = p;
    return XCORR_OK;
}

extern "C" int xcorr_cns_is_on(const xcorr_cns_plan *p, uint64_t seq)
{
    if (!p || p->period_blocks < 1)
        return 0;
    if (seq < p->first_on)
        return 0;
    return (seq - p->first_on) % (uint64_t)p->period_blocks < (uint64_t)p->on_blocks;
}

extern "C" int xcorr_cns_integration(const xcorr_cns_plan *p, int64_t j)
{
    if (!p || p->period_dumps < 1 || j < p->first_integration)
        return 0;
    return (j - p->first_integration) % p->period_dumps == 0;
}
