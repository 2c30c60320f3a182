"""Parity of the HIP chain with the CPU oracle (run with -m gpu on an MI355X).

Object sets are compared as sorted hit-index tuples per stage; the only
allowed mismatches are decisions whose FP64 margin is below 1e-5 and their
descendants (none are expected: both sides round every FP32 operation the
same way).  Candidate counts are integers and must match exactly.
"""
import numpy as np
import pytest

import oracle
from synth import events as E
from synth import geometry as G
from synth import params as PR
from tests.parity import assert_parity

pytestmark = pytest.mark.gpu


def _ctx(geo, params):
    import paper_2209_13711_amd as lst
    return lst.Context(params, geo.f32, geo.i32, device=0)


def _run_both(cid, event=0, n_tracks=None, params=None):
    cfg = E.CONFIGS[cid]
    geo = G.get(cfg.geometry)
    params = PR.make(w=cfg.window) if params is None else params
    ev = E.generate(cid, event, n_tracks=n_tracks)
    print(f"case cfg{cid} event {event} hits {ev.n_hits}", flush=True)
    ctx = _ctx(geo, params)
    got = ctx.run_event(ev)
    cnt = ctx.counts(0)
    ref = oracle.Oracle(params, geo.f32, geo.i32).run_event(ev)
    return ctx, got, cnt, ref, ev


@pytest.mark.parametrize("cid,event,n_tracks", [(1, 0, None), (1, 1, None), (2, 0, 600),
                                                (2, 0, None), (5, 0, 800)])
def test_chain_matches_oracle(cid, event, n_tracks):
    ctx, got, cnt, ref, ev = _run_both(cid, event, n_tracks)
    assert_parity(got, ref)
    # algorithmic candidate counts are exact integers
    assert [cnt["cand_md"], cnt["cand_seg"], cnt["cand_t3"], cnt["cand_t5"]] == ref.cands.tolist()
    assert cnt["n_t5_kept"] == len(ref.tuples[4])


def test_t5_scores_bitwise():
    ctx, got, cnt, ref, ev = _run_both(2, 1, 1500)
    s_gpu = ctx.t5_scores(0)
    t_gpu = ctx.objects(0, 3)
    gmap = {tuple(t): s for t, s in zip(t_gpu.tolist(), s_gpu.view(np.uint32).tolist())}
    omap = {tuple(t): s for t, s in zip(ref.tuples[3].tolist(), ref.t5_scores.view(np.uint32).tolist())}
    assert gmap.keys() == omap.keys()
    assert all(gmap[k] == omap[k] for k in gmap)


def test_batch_of_uneven_events_matches_per_event_oracle():
    cfg = E.CONFIGS[3]
    geo = G.get(cfg.geometry)
    params = PR.make()
    evs = [E.generate(3, e) for e in range(4)]
    b = E.concat(evs)
    print("case batch cfg3 x4 hits", b.offsets.tolist(), flush=True)
    ctx = _ctx(geo, params)
    ctx.run_batch(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
    orc = oracle.Oracle(params, geo.f32, geo.i32)
    for e, ev in enumerate(evs):
        got = {k: ctx.objects(e, k) for k in range(5)}
        ref = orc.run_event(ev)
        assert_parity(got, ref)
        cnt = ctx.counts(e)
        assert [cnt["cand_md"], cnt["cand_seg"], cnt["cand_t3"], cnt["cand_t5"]] == ref.cands.tolist()


@pytest.mark.parametrize("geometry,cid,n_tracks", [("barrel_toy", 1, None), ("full", 2, 300)])
def test_batch_sorted_per_event_matches_oracle(geometry, cid, n_tracks):
    """Batches of 8 or more events group their hits per event in LDS (a
    quarter of the event's bins per block); the batch holds
    an empty event and a hit with a bad module id, and a second batch on the
    same context checks that the first one left every bin at zero."""
    geo = G.get(geometry)
    params = PR.make()
    orc = oracle.Oracle(params, geo.f32, geo.i32)
    ctx = _ctx(geo, params)
    for first in (0, 20):
        evs = [E.generate(cid, first + e, n_tracks=n_tracks) for e in range(9)]
        evs[3] = E.generate(cid, first + 3, n_tracks=0)
        b = E.concat(evs)
        mod = b.module.copy()
        bad = int(b.offsets[5]) + 1            # second hit of event 5
        mod[bad] = geo.n_mod + 3
        print(f"case per-event sort {geometry} first {first} hits {b.offsets.tolist()}", flush=True)
        ctx.run_batch(b.offsets, b.x, b.y, b.z, mod, b.sensor)
        assert ctx.caps["events"] >= 8
        for e, ev in enumerate(evs):
            cnt = ctx.counts(e)
            assert cnt["error_flags"] & 1
            if e == 5:
                keep = np.ones(ev.n_hits, bool)
                keep[1] = False
                ref = orc.run(ev.x[keep], ev.y[keep], ev.z[keep], ev.module[keep], ev.sensor[keep])
                back = np.nonzero(keep)[0]
                for k in range(5):
                    ref.tuples[k] = back[ref.tuples[k]] if len(ref.tuples[k]) else ref.tuples[k]
                for k in range(4):
                    if len(ref.near[k][0]):
                        ref.near[k] = (back[ref.near[k][0]], ref.near[k][1], ref.near[k][2])
            else:
                ref = orc.run_event(ev)
                assert [cnt["cand_md"], cnt["cand_seg"], cnt["cand_t3"],
                        cnt["cand_t5"]] == ref.cands.tolist()
            assert_parity({k: ctx.objects(e, k) for k in range(5)}, ref)
        assert len(ctx.objects(3, 0)) == 0


def test_empty_and_degenerate_events():
    geo = G.get("barrel_toy")
    params = PR.make()
    ctx = _ctx(geo, params)
    print("case empty", flush=True)
    z = np.zeros(0, np.float32)
    ctx.run_batch(np.array([0, 0], np.int32), z, z, z, np.zeros(0, np.int32), np.zeros(0, np.uint8))
    for k in range(5):
        assert len(ctx.objects(0, k)) == 0
    # hits on lower sensors only: no mini-doublet can form
    ev = E.generate(1, 2)
    lo = ev.sensor == 0
    print("case lower-only", flush=True)
    ctx.run_batch(np.array([0, int(lo.sum())], np.int32), ev.x[lo], ev.y[lo], ev.z[lo],
                  ev.module[lo], ev.sensor[lo])
    assert len(ctx.objects(0, 0)) == 0
    # an event between two empty ones
    print("case ragged batch", flush=True)
    offs = np.array([0, 0, ev.n_hits, ev.n_hits], np.int32)
    ctx.run_batch(offs, ev.x, ev.y, ev.z, ev.module, ev.sensor)
    ref = oracle.Oracle(params, geo.f32, geo.i32).run_event(ev)
    assert_parity({k: ctx.objects(1, k) for k in range(5)}, ref)
    assert len(ctx.objects(0, 0)) == 0 and len(ctx.objects(2, 0)) == 0


def test_invalid_hits_are_flagged_and_skipped():
    geo = G.get("barrel_toy")
    params = PR.make()
    ctx = _ctx(geo, params)
    ev = E.generate(1, 3)
    mod = ev.module.copy()
    mod[0] = geo.n_mod + 5          # out of range
    sen = ev.sensor.copy()
    sen[1] = 7                       # bad sensor id
    print("case invalid ids", flush=True)
    ctx.run_batch(np.array([0, ev.n_hits], np.int32), ev.x, ev.y, ev.z, mod, sen)
    c = ctx.counts(0)
    assert c["error_flags"] & 1
    keep = np.ones(ev.n_hits, bool); keep[:2] = False
    ref = oracle.Oracle(params, geo.f32, geo.i32).run(ev.x[keep], ev.y[keep], ev.z[keep],
                                                       ev.module[keep], ev.sensor[keep])
    # oracle indices refer to the filtered arrays: map them back
    back = np.nonzero(keep)[0]
    for k in range(5):
        ref.tuples[k] = back[ref.tuples[k]] if len(ref.tuples[k]) else ref.tuples[k]
    for k in range(4):
        if len(ref.near[k][0]):
            ref.near[k] = (back[ref.near[k][0]], ref.near[k][1], ref.near[k][2])
    assert_parity({k: ctx.objects(0, k) for k in range(5)}, ref)


def test_capacity_overflow_is_reported_then_recovered():
    import paper_2209_13711_amd as lst
    geo = G.get("barrel_toy")
    params = PR.make()
    ctx = _ctx(geo, params)
    ev = E.generate(1, 4)
    print("case tiny capacity", flush=True)
    ctx.reserve(dict(events=1, hits=ev.n_hits, md=64, seg=64, t3=64, t5=64))
    ctx.load_hits(np.array([0, ev.n_hits], np.int32), ev.x, ev.y, ev.z, ev.module, ev.sensor)
    ctx.run_chain()
    c = ctx.counts(0, check=False)
    assert c["rc"] == lst.lst.LST_E_CAPACITY and c["overflow_mask"] & 1
    assert c["n_md"] > 64
    with pytest.raises(lst.LSTError):
        ctx.objects(0, 0)
    got = ctx.run_event(ev)
    ref = oracle.Oracle(params, geo.f32, geo.i32).run_event(ev)
    assert_parity(got, ref)


def test_module_map_on_device_context_equals_oracle():
    geo = G.get("full")
    params = PR.make()
    ctx = _ctx(geo, params)
    ptr, col = ctx.module_map()
    optr, ocol = oracle.Oracle(params, geo.f32, geo.i32).module_map()
    np.testing.assert_array_equal(ptr, optr)
    np.testing.assert_array_equal(col, ocol)


def test_graph_chain_replays_match_eager_and_oracle():
    """The captured chain is replayed several times with eager work in
    between, then fed a batch of a different size; every replay must equal
    the eager chain and the oracle."""
    import torch
    geo = G.get("full")
    params = PR.make()
    orc = oracle.Oracle(params, geo.f32, geo.i32)
    ctx = _ctx(geo, params)
    ev0, ev1 = E.generate(2, 5, n_tracks=2500), E.generate(2, 6, n_tracks=1200)
    print("case graph replays", ev0.n_hits, ev1.n_hits, flush=True)
    eager = ctx.run_event(ev0)
    ref0 = orc.run_event(ev0)
    assert_parity(eager, ref0)
    for rep in range(3):
        got = ctx.run_event(ev0, graph=True)
        assert_parity(got, ref0)
        for k in range(5):
            assert set(map(tuple, got[k].tolist())) == set(map(tuple, eager[k].tolist()))
        # eager work on the same stream between replays
        t = torch.arange(1 << 20, device="cuda", dtype=torch.float32)
        assert float(t.sum().item()) == float((1 << 20) * ((1 << 20) - 1) / 2)
        ctx.run_event(ev1)
    got1 = ctx.run_event(ev1, graph=True)
    assert_parity(got1, orc.run_event(ev1))


def _batch_parity(ctx, evs, orc):
    for e, ev in enumerate(evs):
        assert_parity({k: ctx.objects(e, k) for k in range(5)}, orc.run_event(ev))
        assert (ctx.counts(e)["error_flags"] & 2) == 0     # no barrier time-out


def test_persistent_chain_matches_oracle():
    """The whole chain as one persistent kernel (eager launch and inside a
    hipGraph), on a ragged batch of uneven events and on a PU200-like event."""
    geo = G.get("barrel_toy")
    params = PR.make()
    orc = oracle.Oracle(params, geo.f32, geo.i32)
    evs = [E.generate(3, e) for e in range(6)] + [E.generate(1, 7)]
    b = E.concat(evs)
    print("case persistent batch", b.offsets.tolist(), flush=True)
    ctx = _ctx(geo, params)
    ctx.run_batch(b.offsets, b.x, b.y, b.z, b.module, b.sensor)      # sizes the arena
    t = ctx.tuning()
    for bpc in sorted({1, t["blocks_per_cu"]}):
        ctx.set_tuning(t["grid"], persistent=1, blocks_per_cu=bpc)
        ctx.load_hits(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
        ctx.run_chain_persistent()
        _batch_parity(ctx, evs, orc)
        ctx.load_hits(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
        ctx.run_chain_graph()
        _batch_parity(ctx, evs, orc)
    geo2 = G.get("full")
    ev = E.generate(2, 0)
    print("case persistent pu200", flush=True)
    ctx2 = _ctx(geo2, params)
    ctx2.run_event(ev)
    t2 = ctx2.tuning()
    ctx2.set_tuning(t2["grid"], persistent=1, blocks_per_cu=t2["blocks_per_cu"])
    got = ctx2.run_event(ev)
    assert_parity(got, oracle.Oracle(params, geo2.f32, geo2.i32).run_event(ev))


@pytest.mark.parametrize("lanes", [8, 16, 32, 64])
def test_group_widths_match_oracle(lanes):
    """Every group width of the object stages (lanes per inner object), per
    stage launches and the persistent kernel, on a PU200-like event and a
    ragged batch."""
    import paper_2209_13711_amd as lst
    params = PR.make()
    geo = G.get("full")
    ev = E.generate(2, 2, n_tracks=1500)
    print(f"case lanes {lanes} pu200-1500", flush=True)
    ref = oracle.Oracle(params, geo.f32, geo.i32).run_event(ev)
    ctx = _ctx(geo, params)
    ctx.run_event(ev)
    t = ctx.tuning()
    widths = [64, lanes, lanes, lanes, lanes, 64]
    ctx.set_tuning(t["grid"], persistent=0, blocks_per_cu=1, lanes=widths)
    assert ctx.tuning()["lanes"] == widths
    assert_parity(ctx.run_event(ev), ref)
    ctx.set_tuning(t["grid"], persistent=1, blocks_per_cu=1, lanes=widths)
    assert_parity(ctx.run_event(ev), ref)
    geo_b = G.get("barrel_toy")
    orc = oracle.Oracle(params, geo_b.f32, geo_b.i32)
    evs = [E.generate(3, 20 + e) for e in range(3)] + [E.generate(1, 3)]
    b = E.concat(evs)
    ctx_b = _ctx(geo_b, params)
    ctx_b.run_batch(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
    ctx_b.set_tuning(ctx_b.tuning()["grid"], persistent=0, blocks_per_cu=1, lanes=widths)
    ctx_b.run_batch(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
    _batch_parity(ctx_b, evs, orc)


@pytest.mark.parametrize("lanes", [16, 32])
def test_one_pass_and_many_pass_orders_match_oracle(lanes):
    """The MD, segment, triplet and quintuplet stages spread a sector's inner
    objects over the waves when the grid covers the sector in one pass, and
    keep their consecutive order when each wave makes several passes: both
    orders (grids of 8192 and 8 blocks) give the oracle's objects on the same
    PU200-like event."""
    params = PR.make()
    geo = G.get("full")
    ev = E.generate(2, 4)
    ref = oracle.Oracle(params, geo.f32, geo.i32).run_event(ev)
    ctx = _ctx(geo, params)
    ctx.run_event(ev)
    t = ctx.tuning()
    widths = [64, lanes, lanes, lanes, lanes, 64]
    for g in (8192, 8):
        print(f"case lanes {lanes} object-stage grid {g}", flush=True)
        ctx.set_tuning([t["grid"][0], g, g, g, g, t["grid"][5]], persistent=0, blocks_per_cu=1,
                       lanes=widths)
        assert ctx.tuning()["grid"][1:5] == [g] * 4
        assert_parity(ctx.run_event(ev), ref)


@pytest.mark.parametrize("lanes", [8, 16, 32])
def test_batch_shared_segment_enumeration_matches_oracle(lanes):
    """Arenas of several events use the segment kernel whose runs of inner MDs
    of one module share their candidates; with a grid of 8 blocks every wave
    takes consecutive MDs, so runs of one module are common.  Two PU200-like
    events (one of them with 2500 tracks) in one batch against the oracle,
    then the same batch with a one-pass grid (spread order, nothing
    shared)."""
    params = PR.make()
    geo = G.get("full")
    orc = oracle.Oracle(params, geo.f32, geo.i32)
    evs = [E.generate(2, 6), E.generate(2, 7, n_tracks=2500)]
    b = E.concat(evs)
    ctx = _ctx(geo, params)
    ctx.run_batch(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
    t = ctx.tuning()
    widths = [64, lanes, lanes, lanes, lanes, 64]
    for g in (8, 8192):
        print(f"case lanes {lanes} batch of 2 object-stage grid {g}", flush=True)
        ctx.set_tuning([t["grid"][0], g, g, g, g, t["grid"][5]], persistent=0, blocks_per_cu=1,
                       lanes=widths)
        ctx.run_batch(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
        _batch_parity(ctx, evs, orc)


def test_autotuner_keeps_results_and_caches(tmp_path):
    geo = G.get("barrel_toy")
    params = PR.make()
    orc = oracle.Oracle(params, geo.f32, geo.i32)
    evs = [E.generate(3, 10 + e) for e in range(3)]
    b = E.concat(evs)
    print("case tuner", b.offsets.tolist(), flush=True)
    ctx = _ctx(geo, params)
    ctx.run_batch(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
    cache = str(tmp_path / "tune.jsonl")
    res = ctx.tune(cache_path=cache, reps=2)
    print("tuned", res, flush=True)
    assert res["report_us"][0] > 0
    _batch_parity(ctx, evs, orc)
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and '"tuning"' in lines[0]
    ctx2 = _ctx(geo, params)
    ctx2.run_batch(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
    res2 = ctx2.tune(cache_path=cache, reps=2)
    assert res2["report_us"][0] == -1.0
    assert res2["grid"] == res["grid"] and res2["persistent"] == res["persistent"]
    assert res2["lanes"] == res["lanes"]
    ctx2.load_hits(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
    ctx2.run_chain_graph()
    _batch_parity(ctx2, evs, orc)


@pytest.mark.parametrize("cid,n_tracks", [(2, 1500), (5, 600)])
def test_t5_features_bitwise(cid, n_tracks):
    cfg = E.CONFIGS[cid]
    geo = G.get(cfg.geometry)
    params = PR.make(w=cfg.window)
    ev = E.generate(cid, 2, n_tracks=n_tracks)
    print(f"case features cfg{cid}", ev.n_hits, flush=True)
    ctx = _ctx(geo, params)
    caps = dict(ctx.lib and __import__("paper_2209_13711_amd").default_caps(1, ev.n_hits))
    caps["features"] = 1
    ctx.reserve(caps)
    ctx.run_event(ev)
    ctx.run_t5_features()
    tup = ctx.objects(0, 3)
    feat = ctx.t5_features(0)
    ref = oracle.Oracle(params, geo.f32, geo.i32).run_event(ev)
    omap = {tuple(t): f for t, f in zip(ref.tuples[3].tolist(), ref.t5_features.view(np.uint32))}
    assert len(tup) == len(omap) > 50
    for t, f in zip(tup.tolist(), feat.view(np.uint32)):
        np.testing.assert_array_equal(f, omap[tuple(t)])


def test_dedup_with_many_score_ties_matches_oracle():
    """Upper hits of 20 tracks duplicated in place: every mini-doublet of
    those tracks has two upper-hit choices with identical coordinates, so up
    to 32 quintuplets share one score and their hits (more ties per hit than
    the inline slots hold); the survivor is decided by the hit tuple."""
    import paper_2209_13711_amd as lst
    geo = G.get("barrel_toy")
    params = PR.make()
    ev = E.generate(1, 0)
    sel = np.flatnonzero((ev.sensor == 1) & (ev.truth >= 0) & (ev.truth < 20))
    arrs = [np.concatenate([a, a[sel]]) for a in (ev.x, ev.y, ev.z, ev.module, ev.sensor)]
    print(f"case tie-heavy event hits {len(arrs[0])}", flush=True)
    ref = oracle.Oracle(params, geo.f32, geo.i32).run(*arrs)
    ctx = lst.Context(params, geo.f32, geo.i32, device=0)
    offs = np.array([0, len(arrs[0])], np.int32)
    for run in ("chain", "persistent"):
        ctx.run_batch(offs, *arrs)
        if run == "persistent":
            ctx.run_chain_persistent()
        for kind in (lst.LST_T5, lst.LST_T5_KEPT):
            got = {tuple(t) for t in ctx.objects(0, kind).tolist()}
            assert got == {tuple(t) for t in ref.tuples[kind].tolist()}, (run, kind)
