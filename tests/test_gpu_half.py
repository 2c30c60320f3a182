"""Half-precision hit storage on the GPU against the oracle's storage mode
(-m gpu).

With lst_set_hit_storage(1) the grouping stage keeps every hit as binary16
module-local (u, v) plus its index and the mini-doublet stage rebuilds the
FP32 position; the oracle applies the same rounding and rebuild before its
chain (pinned against NumPy's float16 on the CPU).  Object sets, candidate
counts and scores must be equal: single events, batches grouped on the
device and per event in LDS, graph replays, the persistent kernel, hits
planted with u in the binary16 subnormal range, and switching the mode back.
"""
import numpy as np
import pytest

import oracle
from synth import events as E
from synth import geometry as G
from synth import params as PR
from tests.parity import assert_parity

pytestmark = pytest.mark.gpu


def _oracles(cid):
    cfg = E.CONFIGS[cid]
    geo = G.get(cfg.geometry)
    params = PR.make(w=cfg.window)
    half = oracle.Oracle(params, geo.f32, geo.i32)
    half.set_hit_storage(True)
    return geo, params, half, oracle.Oracle(params, geo.f32, geo.i32)


@pytest.mark.parametrize("cid,event,n_tracks", [(1, 0, None), (2, 0, None), (5, 0, 1500)])
def test_half_storage_chain_matches_oracle(cid, event, n_tracks):
    import paper_2209_13711_amd as lst
    geo, params, half, plain = _oracles(cid)
    ev = E.generate(cid, event, n_tracks=n_tracks)
    print(f"case fp16 storage cfg{cid} event {event}", flush=True)
    ctx = lst.Context(params, geo.f32, geo.i32, device=0)
    ctx.set_hit_storage(True)
    got = ctx.run_event(ev)
    ref = half.run_event(ev)
    assert_parity(got, ref)
    c = ctx.counts(0)
    assert [c["cand_md"], c["cand_seg"], c["cand_t3"], c["cand_t5"]] == ref.cands.tolist()
    s_gpu = {tuple(t): s for t, s in zip(ctx.objects(0, 3).tolist(), ctx.t5_scores(0).view(np.uint32))}
    s_ref = {tuple(t): s for t, s in zip(ref.tuples[3].tolist(), ref.t5_scores.view(np.uint32))}
    assert s_gpu == s_ref
    offs = np.array([0, ev.n_hits], np.int32)
    for chain in (ctx.run_chain_graph, ctx.run_chain_graph, ctx.run_chain_persistent):
        ctx.load_hits(offs, ev.x, ev.y, ev.z, ev.module, ev.sensor)
        chain()
        assert_parity({k: ctx.objects(0, k) for k in range(5)}, ref)
    # back to FP32 storage: the plain oracle's objects
    ctx.set_hit_storage(False)
    assert_parity(ctx.run_event(ev), plain.run_event(ev))


@pytest.mark.parametrize("cid,n_events,n_tracks", [(3, 4, None), (2, 9, 300)])
def test_half_storage_batches_match_oracle(cid, n_events, n_tracks):
    import paper_2209_13711_amd as lst
    geo, params, half, _ = _oracles(cid)
    evs = [E.generate(cid, 70 + e, n_tracks=n_tracks) for e in range(n_events)]
    b = E.concat(evs)
    print(f"case fp16 storage batch cfg{cid} x{n_events}", flush=True)
    ctx = lst.Context(params, geo.f32, geo.i32, device=0)
    ctx.set_hit_storage(True)
    ctx.run_batch(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
    for e, ev in enumerate(evs):
        assert_parity({k: ctx.objects(e, k) for k in range(5)}, half.run_event(ev))


def test_half_storage_subnormal_coordinates_match_oracle():
    """lower hits moved onto their module's v axis, with u of 3e-6, -5e-7 and
    1e-8 cm (binary16 subnormals and below)"""
    import paper_2209_13711_amd as lst
    geo, params, half, _ = _oracles(1)
    ev = E.generate(1, 6)
    f = geo.f32
    x, y, z = ev.x.copy(), ev.y.copy(), ev.z.copy()
    lows = np.nonzero(ev.sensor == 0)[0][:300]
    for i, h in enumerate(lows):
        m = ev.module[h]
        u = np.float32([3e-6, -5e-7, 1e-8][i % 3])
        c = f[G.F_CX:G.F_CZ + 1, m].astype(np.float64)
        U = f[G.F_UX:G.F_UZ + 1, m].astype(np.float64)
        V = f[G.F_VX:G.F_VZ + 1, m].astype(np.float64)
        W = f[G.F_WX:G.F_WZ + 1, m].astype(np.float64)
        v = ((np.array([x[h], y[h], z[h]], np.float64) - c) @ V)
        p = c + u * U + v * V - 0.5 * f[G.F_GAP, m] * W
        x[h], y[h], z[h] = p.astype(np.float32)
    ctx = lst.Context(params, geo.f32, geo.i32, device=0)
    ctx.set_hit_storage(True)
    ctx.run_batch(np.array([0, ev.n_hits], np.int32), x, y, z, ev.module, ev.sensor)
    assert_parity({k: ctx.objects(0, k) for k in range(5)}, half.run(x, y, z, ev.module, ev.sensor))
