"""Per-module capacities on the GPU against the oracle (-m gpu).

With capacities set, each stage's objects of a module beyond its capacity
are removed (the smallest hit tuples kept) before the next stage; the
oracle does the same on the CPU (its rule is pinned against a filter of the
uncapped chain in test_oracle_truncation.py).  Object sets, candidate
counts and per-kind drop counts must be equal, per stage launch, replayed
hipGraph and tuned launch shape, for single events and batches; without
capacities the chain is the plain one again.
"""
import numpy as np
import pytest

import oracle
from synth import events as E
from synth import geometry as G
from synth import params as PR
from tests.parity import assert_parity
from tests.test_oracle_truncation import _filtered

pytestmark = pytest.mark.gpu


def _check(ctx, e, orc, ev, caps):
    ref = orc.run_event(ev)
    got = {k: ctx.objects(e, k) for k in range(5)}
    assert_parity(got, ref)
    c = ctx.counts(e)
    assert [c["cand_md"], c["cand_seg"], c["cand_t3"], c["cand_t5"]] == ref.cands.tolist()
    assert c["dropped"] == orc.dropped().tolist(), (e, caps, c["dropped"], orc.dropped())
    return orc.dropped()


@pytest.mark.parametrize("cid,event,n_tracks,q", [(1, 0, None, 0.9), (2, 0, None, 0.97),
                                                  (2, 1, None, 0.999), (5, 0, 1500, 0.99)])
def test_capped_event_matches_oracle(cid, event, n_tracks, q):
    import paper_2209_13711_amd as lst
    cfg = E.CONFIGS[cid]
    geo = G.get(cfg.geometry)
    params = PR.make(w=cfg.window)
    ev = E.generate(cid, event, n_tracks=n_tracks)
    orc = oracle.Oracle(params, geo.f32, geo.i32)
    caps = _filtered(orc.run_event(ev), ev, q, *orc.module_map())["caps"]
    orc.set_truncation(caps)
    print(f"case capacities cfg{cid} event {event} caps {caps}", flush=True)
    ctx = lst.Context(params, geo.f32, geo.i32, device=0)
    ctx.set_capacities(caps)
    offs = np.array([0, ev.n_hits], np.int32)
    ctx.run_batch(offs, ev.x, ev.y, ev.z, ev.module, ev.sensor)
    d = _check(ctx, 0, orc, ev, caps)
    assert d.sum() > 0
    # stage by stage, then as a replayed graph, then with a tuned launch shape
    ctx.load_hits(offs, ev.x, ev.y, ev.z, ev.module, ev.sensor)
    for fn in (ctx.run_sort, ctx.run_md, ctx.run_segments, ctx.run_triplets, ctx.run_quintuplets,
               ctx.run_dedup):
        fn()
    _check(ctx, 0, orc, ev, caps)
    for _ in range(2):
        ctx.run_chain_graph()
        _check(ctx, 0, orc, ev, caps)
    ctx.tune(reps=1)
    ctx.run_chain_graph()
    _check(ctx, 0, orc, ev, caps)
    with pytest.raises(lst.LSTError) as ei:
        ctx.run_chain_persistent()
    assert ei.value.code == lst.LST_E_STATE
    # capacities off: the plain chain again
    ctx.set_capacities(None)
    orc.set_truncation(None)
    ctx.run_chain_graph()
    _check(ctx, 0, orc, ev, caps)
    assert ctx.counts(0)["dropped"] == [0, 0, 0, 0]


@pytest.mark.parametrize("cid,n_events", [(3, 4), (2, 9)])
def test_capped_batch_matches_oracle(cid, n_events):
    """a ragged batch (config 3) and a batch grouped per event in LDS (nine
    PU200-like events, one empty): the same capacities in every event"""
    import paper_2209_13711_amd as lst
    cfg = E.CONFIGS[cid]
    geo = G.get(cfg.geometry)
    params = PR.make(w=cfg.window)
    evs = [E.generate(cid, 40 + e, n_tracks=(0 if e == 3 and n_events > 4 else None))
           for e in range(n_events)]
    orc = oracle.Oracle(params, geo.f32, geo.i32)
    caps = _filtered(orc.run_event(evs[0]), evs[0], 0.97, *orc.module_map())["caps"]
    orc.set_truncation(caps)
    b = E.concat(evs)
    print(f"case capped batch cfg{cid} x{n_events} caps {caps}", flush=True)
    ctx = lst.Context(params, geo.f32, geo.i32, device=0)
    ctx.set_capacities(caps)
    ctx.run_batch(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
    tot = np.zeros(4, np.int64)
    for e, ev in enumerate(evs):
        tot += _check(ctx, e, orc, ev, caps)
    assert tot.sum() > 0
    ctx.run_chain_graph()
    for e, ev in enumerate(evs):
        _check(ctx, e, orc, ev, caps)
