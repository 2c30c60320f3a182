"""Pixel objects and track candidates on the GPU against the oracle (-m gpu).

The pT5 and pT3 link candidates must be the oracle's (seed and outer hit
tuple), with bit-equal scores and equal survival flags, and the track
candidates must be equal as (type, seed, hit tuple) rows, for single events
(barrel toy, full geometry, stress configuration), batches (ragged, and
grouped per event in LDS), after per-stage, graph and persistent chains.
The oracle counts its pixel decisions within 1e-5 of a threshold; none is
expected, and any difference must be explained by one.
"""
import numpy as np
import pytest

import oracle
from synth import events as E
from synth import geometry as G
from synth import params as PR

pytestmark = pytest.mark.gpu

PP = PR.make_pixel()


def _rows(a):
    return set(map(tuple, np.asarray(a).tolist()))


def _compare(ctx, e, pr):
    for what, ref in ((0, pr.pt5), (1, pr.pt3)):
        got = ctx.pixel_candidates(e, what)
        assert _rows(got) == _rows(ref) or pr.near > 0, (e, what, len(got), len(ref),
                                                         len(_rows(got) ^ _rows(ref)))
    tc = ctx.track_candidates(e)
    assert _rows(tc) == _rows(pr.tc) or pr.near > 0, (e, len(tc), len(pr.tc))
    c = ctx.counts(e)
    assert c["n_tc"] == len(pr.tc) or pr.near > 0
    return tc


@pytest.mark.parametrize("cid,event,n_tracks", [(1, 0, None), (2, 0, None), (5, 0, 1500)])
def test_pixel_stage_matches_oracle(cid, event, n_tracks):
    import paper_2209_13711_amd as lst
    cfg = E.CONFIGS[cid]
    geo = G.get(cfg.geometry)
    params = PR.make(w=cfg.window)
    ev = E.generate(cid, event, n_tracks=n_tracks)
    px = E.pixel_seeds(ev, cid, event)
    orc = oracle.Oracle(params, geo.f32, geo.i32)
    orc.run_event(ev)
    pr = orc.run_pixel(PP, px)
    print(f"case pixel cfg{cid} event {event}: seeds {px.n_seeds} tc {len(pr.tc)} "
          f"near {pr.near}", flush=True)
    ctx = lst.Context(params, geo.f32, geo.i32, device=0)
    ctx.run_event_pixel(ev, px, PP)
    tc = _compare(ctx, 0, pr)
    assert len(tc) > 0 and set(tc[:, 0].tolist()) >= {lst.LST_TC_PT5}
    # after a replayed graph and after the persistent kernel
    offs = np.array([0, ev.n_hits], np.int32)
    for chain in (ctx.run_chain_graph, ctx.run_chain_persistent):
        ctx.load_hits(offs, ev.x, ev.y, ev.z, ev.module, ev.sensor)
        chain()
        ctx.load_pixel(np.array([0, px.n_hits], np.int32), px.x, px.y, px.z,
                       np.array([0, px.n_seeds], np.int32), px.seeds, PP)
        ctx.run_pixel()
        _compare(ctx, 0, pr)


@pytest.mark.parametrize("cid,n_events,n_tracks", [(3, 4, None), (2, 9, 400)])
def test_pixel_stage_batch_matches_oracle(cid, n_events, n_tracks):
    import paper_2209_13711_amd as lst
    cfg = E.CONFIGS[cid]
    geo = G.get(cfg.geometry)
    params = PR.make(w=cfg.window)
    evs = [E.generate(cid, 50 + e, n_tracks=n_tracks) for e in range(n_events)]
    pxs = [E.pixel_seeds(ev, cid, 50 + e) for e, ev in enumerate(evs)]
    b = E.concat(evs)
    poff = np.r_[0, np.cumsum([p.n_hits for p in pxs])].astype(np.int32)
    soff = np.r_[0, np.cumsum([p.n_seeds for p in pxs])].astype(np.int32)
    cat = lambda a: np.concatenate([getattr(p, a) for p in pxs])
    seeds = np.concatenate([p.seeds for p in pxs])
    print(f"case pixel batch cfg{cid} x{n_events} seeds {soff[-1]}", flush=True)
    ctx = lst.Context(params, geo.f32, geo.i32, device=0)
    ctx.reserve(lst.default_caps(n_events, int(b.offsets[-1])))
    ctx.pixel_caps(int(poff[-1]), int(soff[-1]))
    ctx.run_batch(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
    ctx.load_pixel(poff, cat("x"), cat("y"), cat("z"), soff, seeds, PP)
    ctx.run_pixel()
    orc = oracle.Oracle(params, geo.f32, geo.i32)
    for e, (ev, px) in enumerate(zip(evs, pxs)):
        orc.run_event(ev)
        _compare(ctx, e, orc.run_pixel(PP, px))


def test_pixel_stage_state_and_input_errors():
    import paper_2209_13711_amd as lst
    geo = G.get("barrel_toy")
    ev = E.generate(1, 0)
    px = E.pixel_seeds(ev, 1, 0)
    ctx = lst.Context(PR.make(), geo.f32, geo.i32, device=0)
    ctx.run_event(ev)            # arena without pixel capacities
    one = np.array([0, px.n_hits], np.int32)
    sone = np.array([0, px.n_seeds], np.int32)
    with pytest.raises(lst.LSTError) as ei:
        ctx.load_pixel(one, px.x, px.y, px.z, sone, px.seeds, PP)
    assert ei.value.code == lst.LST_E_CAPACITY
    ctx.run_event_pixel(ev, px, PP)
    with pytest.raises(lst.LSTError) as ei:      # twice
        ctx.run_pixel()
    assert ei.value.code == lst.LST_E_STATE
    ctx.load_hits(np.array([0, ev.n_hits], np.int32), ev.x, ev.y, ev.z, ev.module, ev.sensor)
    ctx.run_chain()
    with pytest.raises(lst.LSTError) as ei:      # seeds of the earlier batch are gone
        ctx.run_pixel()
    assert ei.value.code == lst.LST_E_STATE
    bad = px.seeds.copy()
    bad[3, 2] = px.n_hits
    with pytest.raises(lst.LSTError) as ei:
        ctx.load_pixel(one, px.x, px.y, px.z, sone, bad, PP)
    assert ei.value.code == lst.LST_E_INVALID
    with pytest.raises(lst.LSTError) as ei:      # before the chain's dedup
        ctx.load_hits(np.array([0, ev.n_hits], np.int32), ev.x, ev.y, ev.z, ev.module, ev.sensor)
        ctx.run_sort()
        ctx.load_pixel(one, px.x, px.y, px.z, sone, px.seeds, PP)
        ctx.run_pixel()
    assert ei.value.code == lst.LST_E_STATE


def test_pixel_stage_full_size_batch_of_16_pu200():
    """16 PU200-like events (the full-size batch) with their pixel seeds in
    one launch, every event against the oracle"""
    import paper_2209_13711_amd as lst
    geo = G.get("full")
    params = PR.make()
    evs = [E.generate(2, 100 + e) for e in range(16)]
    pxs = [E.pixel_seeds(ev, 2, 100 + e) for e, ev in enumerate(evs)]
    b = E.concat(evs)
    poff = np.r_[0, np.cumsum([p.n_hits for p in pxs])].astype(np.int32)
    soff = np.r_[0, np.cumsum([p.n_seeds for p in pxs])].astype(np.int32)
    cat = lambda a: np.concatenate([getattr(p, a) for p in pxs])
    print(f"case pixel full-size batch: 16 events, {soff[-1]} seeds", flush=True)
    ctx = lst.Context(params, geo.f32, geo.i32, device=0)
    ctx.reserve(lst.default_caps(16, int(b.offsets[-1])))
    ctx.pixel_caps(int(poff[-1]), int(soff[-1]))
    ctx.run_batch(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
    ctx.tune(reps=1)
    ctx.load_hits(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
    ctx.run_chain_graph()
    ctx.load_pixel(poff, cat("x"), cat("y"), cat("z"), soff, np.concatenate([p.seeds for p in pxs]), PP)
    ctx.run_pixel()
    orc = oracle.Oracle(params, geo.f32, geo.i32)
    for e, (ev, px) in enumerate(zip(evs, pxs)):
        orc.run_event(ev)
        _compare(ctx, e, orc.run_pixel(PP, px))
        assert ctx.counts(e)["error_flags"] == 0
