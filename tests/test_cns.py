"""Calibrator-noise-source gating aligned to integrations (paper Section 2.5,
"CNS control module"): every on-window lies wholly inside one integration and
starts at its first block, the first window is the earliest integration start
the host can still program, the period is whole integrations, and the
integrations the schedule flags are exactly those whose blocks carry the CNS
when the blocks go through sequence-number reassembly."""
import random

import pytest

from paper_2406_19013_amd import xcorr as X


def _windows(p, upto):
    """On-windows [s, e) that start before `upto`, enumerated from the plan."""
    out, s = [], p.first_on
    while s < upto:
        out.append((s, s + p.on_blocks))
        s += p.period_blocks
    return out


@pytest.mark.parametrize("seed", range(40))
def test_windows_fall_inside_one_integration(seed):
    rng = random.Random(seed)
    k = rng.choice([1, 2, 7, 128, 1000])
    origin = rng.randrange(0, 10 ** 6)
    now = origin + rng.randrange(-5000, 10 ** 6)
    now = max(now, 0)
    lead = rng.randrange(0, 3 * k + 5)
    period = rng.randrange(1, 6)
    on = rng.randrange(1, k + 1)
    p = X.xcorr_cns_plan_make(now, lead, origin, k, period, on)
    # first window: an integration start, not before now + lead, and the
    # earliest such start
    assert p.first_on >= now + lead and p.first_on >= origin
    assert (p.first_on - origin) % k == 0
    assert p.first_on - k < max(now + lead, origin) or p.first_on == origin
    assert p.first_integration == (p.first_on - origin) // k
    assert p.period_blocks == period * k
    upto = origin + (p.first_integration + 4 * period + 3) * k   # past every integration checked below
    for s, e in _windows(p, upto):
        j = (s - origin) // k
        assert s == origin + j * k                       # starts an integration
        assert e <= origin + (j + 1) * k                 # ends inside it
        assert p.integration(j)
    # the on/off state block by block agrees with the windows, and each
    # integration is flagged exactly when it holds on-blocks
    on_set = {seq for s, e in _windows(p, upto) for seq in range(s, e)}
    lo = max(origin, p.first_on - 2 * k)
    for seq in range(lo, min(upto, lo + 12 * k + 50)):
        assert p.is_on(seq) == (seq in on_set), seq
    for j in range(max(0, p.first_integration - 2), p.first_integration + 4 * period + 2):
        blocks = range(origin + j * k, origin + (j + 1) * k)
        assert p.integration(j) == any(b in on_set for b in blocks), j


def test_edge_cases():
    # now + lead exactly on a boundary: that boundary
    p = X.xcorr_cns_plan_make(1000, 0, 0, 100, 3, 100)
    assert p.first_on == 1000 and p.first_integration == 10
    # one past a boundary: the next one
    p = X.xcorr_cns_plan_make(1001, 0, 0, 100, 3, 100)
    assert p.first_on == 1100
    # before the origin: integration 0
    p = X.xcorr_cns_plan_make(5, 10, 500, 64, 1, 1)
    assert p.first_on == 500 and p.first_integration == 0
    # on for a whole integration, every integration
    p = X.xcorr_cns_plan_make(0, 0, 0, 8, 1, 8)
    assert all(p.is_on(s) for s in range(64))
    # before the first window nothing is on
    p = X.xcorr_cns_plan_make(700, 0, 0, 100, 2, 30)
    assert not any(p.is_on(s) for s in range(0, 700))
    assert [s for s in range(700, 1200) if p.is_on(s)] == list(range(700, 730)) + list(range(900, 930)) + \
        list(range(1100, 1130))


def test_refusals():
    for args in [(0, 0, 0, 0, 1, 1), (0, 0, 0, 8, 0, 1), (0, 0, 0, 8, 1, 0), (0, 0, 0, 8, 1, 9),
                 (1 << 63, 0, 0, 8, 1, 1)]:
        with pytest.raises(X.XcorrError):
            X.xcorr_cns_plan_make(*args)


def test_cns_blocks_through_reassembly():
    """Blocks tagged by the schedule (CNS on) arrive shuffled and with losses;
    after reassembly each integration holds CNS blocks only if the schedule
    flags it, and then exactly on_blocks of them unless some were lost."""
    k, period, on, origin = 16, 3, 5, 1000
    p = X.xcorr_cns_plan_make(1013, 20, origin, k, period, on)
    rng = random.Random(4)
    seqs = [s for s in range(origin, origin + 40 * k) if rng.random() > 0.02]
    arrivals = sorted(seqs, key=lambda s: s + rng.uniform(0, 6))
    r = X.Reorder(k, 8, max_missing=k, seq_origin=origin)
    per_int = {}
    lost = set(range(origin, origin + 40 * k)) - set(seqs)

    def take(events):
        for e in events:
            if e["kind"] == "block":
                j = (e["seq"] - origin) // k
                per_int.setdefault(j, []).append(e["block"])

    for s in arrivals:
        take(r.push(s, p.is_on(s)))
    take(r.flush(True))
    r.close()
    for j in range(40):
        n_on = sum(1 for b in per_int.get(j, []) if b)
        blocks = range(origin + j * k, origin + (j + 1) * k)
        if p.integration(j):
            assert n_on == on - sum(1 for b in blocks if b in lost and p.is_on(b)), j
        else:
            assert n_on == 0, j
