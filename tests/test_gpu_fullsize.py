"""Parity with the oracle at the full sizes of the measured workloads, in the
launch configuration that bench.py times: the launch shape picked by the
autotuner, the chain replayed as one hipGraph (per-stage kernels or the
persistent kernel, whichever the tuner picked) and the persistent kernel on
the same batch.  Events are compared with the oracle run on that event
alone (object sets as hit-index tuples, candidate counts exactly): every
event of the PU200-like batch, every fourth of the 64-event batch and every
second of the stress batch; on all events the persistent kernel's counts
must equal the graph's, no error flag may be raised and the kept
quintuplets must be pairwise hit-disjoint.
"""
import time

import numpy as np
import pytest

import oracle
from synth import events as E
from synth import geometry as G
from synth import params as PR
from tests.parity import assert_parity

pytestmark = pytest.mark.gpu


def _tuned(cid, seeds):
    import torch
    import paper_2209_13711_amd as lst
    cfg = E.CONFIGS[cid]
    geo = G.get(cfg.geometry)
    params = PR.make(w=cfg.window)
    t0 = time.perf_counter()
    evs = [E.generate(cid, s) for s in seeds]
    b = E.concat(evs)
    print(f"case full size config {cid}: {len(evs)} events, {int(b.offsets[-1])} hits "
          f"(generated in {time.perf_counter() - t0:.1f} s)", flush=True)
    ctx = lst.Context(params, geo.f32, geo.i32, device=0)
    ctx.run_batch(b.offsets, b.x, b.y, b.z, b.module, b.sensor)     # sizes the arena
    t0 = time.perf_counter()
    t = ctx.tune(reps=1)
    print("tuned", {k: t[k] for k in ("grid", "lanes", "persistent", "blocks_per_cu")},
          f"in {time.perf_counter() - t0:.1f} s", flush=True)
    stream = torch.cuda.current_stream()
    load = lambda: ctx.load_hits(b.offsets, b.x, b.y, b.z, b.module, b.sensor, stream)
    return ctx, evs, oracle.Oracle(params, geo.f32, geo.i32), load, stream


COUNT_KEYS = ("n_md", "n_seg", "n_t3", "n_t5", "n_t5_kept", "cand_md", "cand_seg", "cand_t3",
              "cand_t5", "error_flags")


def _objects(ctx, events):
    return {e: {k: ctx.objects(e, k) for k in range(5)} for e in events}


def _counts(ctx, n_events):
    return [{k: ctx.counts(e)[k] for k in COUNT_KEYS} for e in range(n_events)]


def _against_oracle(ctx, evs, orc, sample):
    """the sampled events against the oracle; every event: no error flag and
    kept quintuplets pairwise hit-disjoint (duplicate removal's invariant)"""
    t0 = time.perf_counter()
    got = _objects(ctx, sample)
    for e in sample:
        ref = orc.run_event(evs[e])
        assert_parity(got[e], ref)
        c = ctx.counts(e)
        assert [c["cand_md"], c["cand_seg"], c["cand_t3"], c["cand_t5"]] == ref.cands.tolist(), e
        assert c["n_t5_kept"] == len(ref.tuples[4]), e
    cnt = _counts(ctx, len(evs))
    for e in range(len(evs)):
        assert cnt[e]["error_flags"] == 0, e
        kept = ctx.objects(e, 4)
        assert len(kept) == cnt[e]["n_t5_kept"], e
        assert len(np.unique(kept)) == kept.size, e
    print(f"oracle parity of {len(sample)} of {len(evs)} events in {time.perf_counter() - t0:.1f} s",
          flush=True)
    return got, cnt


def _same(ctx, want, want_counts):
    for e, objs in _objects(ctx, want).items():
        for k in range(5):
            assert set(map(tuple, objs[k].tolist())) == set(map(tuple, want[e][k].tolist())), (e, k)
    assert _counts(ctx, len(want_counts)) == want_counts


def _graph_then_persistent(cid, seeds, every):
    """every `every`-th event of the batch against the oracle, all of them
    against the persistent kernel's counts"""
    import torch
    ctx, evs, orc, load, stream = _tuned(cid, seeds)
    for _ in range(3):       # several replays of the captured chain
        load()
        ctx.run_chain_graph(stream)
    torch.cuda.synchronize()
    want, want_counts = _against_oracle(ctx, evs, orc, range(0, len(evs), every))
    print("case persistent kernel on the same batch", flush=True)
    load()
    ctx.run_chain_persistent(stream)
    torch.cuda.synchronize()
    _same(ctx, want, want_counts)


def test_pu200_event_tuned_graph_matches_oracle():
    """the headline workload: one PU200-like event (full geometry), per-stage
    eager calls and graph replays after tuning"""
    import torch
    ctx, evs, orc, load, stream = _tuned(2, [0])
    load()
    for fn in (ctx.run_sort, ctx.run_md, ctx.run_segments, ctx.run_triplets,
               ctx.run_quintuplets, ctx.run_dedup):
        fn(stream)
    torch.cuda.synchronize()
    want, want_counts = _against_oracle(ctx, evs, orc, [0])
    for _ in range(5):
        ctx.run_chain_graph(stream)
    torch.cuda.synchronize()
    _same(ctx, want, want_counts)


def test_batch_of_64_uneven_events_full_size():
    """64 events of uneven pileup (barrel toy) in one launch"""
    _graph_then_persistent(3, range(64), every=4)


def test_pu200_batch_of_16_full_size():
    """16 PU200-like events (full geometry) in one launch: per-event hit
    grouping in LDS"""
    _graph_then_persistent(2, range(100, 116), every=1)


def test_stress_batch_of_16_full_size():
    """16 PU300-like events with displaced tracks, 10 % noise and windows
    widened 1.5x, in one launch"""
    _graph_then_persistent(5, range(16), every=2)
