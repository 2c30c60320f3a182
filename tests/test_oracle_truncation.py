"""Pins of the oracle's per-module capacities (Sec. 3: object arrays of a
fixed capacity per module, truncated at an occupancy quantile).

Each cut decides a candidate from its own mini-doublets only, so the chain
with capacities equals a filter of the chain without them, stage by stage:
the MDs a module keeps are its `cap` smallest (lower, upper) hit pairs; the
segments built are exactly the uncapped segments whose two MDs were kept,
of which each inner module keeps its `cap` smallest hit tuples; triplets are
the uncapped triplets whose two segments were kept, then capped; quintuplets
likewise from kept triplets; duplicate removal runs on the kept quintuplets.
That filter is written here in Python from the uncapped oracle's output and
must give the capped oracle's object sets, candidate counts and drop counts.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as M
from synth import events as E
from synth import geometry as G
from synth import params as PR


def _quantile_cap(tuples, module, q):
    """capacity at the q-quantile of the per-module counts of the modules
    holding at least one object, so that some modules exceed it"""
    cnt = np.bincount(module[tuples[:, 0]]) if len(tuples) else np.zeros(1, np.int64)
    cnt = cnt[cnt > 0]
    if len(cnt) == 0:
        return 1
    return max(1, min(int(np.quantile(cnt, q)), int(cnt.max()) - 1))


def _cap(tuples, module, cap, caps=None, q=None):
    """per module (that of the first hit), the `cap` smallest tuples; with q,
    the capacity is first set at that quantile and appended to caps"""
    if q is not None:
        cap = _quantile_cap(tuples, module, q)
        caps.append(cap)
    if cap <= 0 or len(tuples) == 0:
        return tuples, 0
    keep = []
    mods = module[tuples[:, 0]]
    for m in np.unique(mods):
        rows = tuples[mods == m]
        rows = rows[np.lexsort(rows.T[::-1])]
        keep.append(rows[:cap])
    kept = np.concatenate(keep)
    return kept, len(tuples) - len(kept)


def _as_set(t):
    return set(map(tuple, np.asarray(t).tolist()))


def _filtered(ref, ev, q, ptr, col):
    """the capped chain, from the uncapped oracle's objects, with each kind's
    capacity at the q-quantile of its per-module counts in the capped chain"""
    mod = ev.module
    caps = []
    md, d0 = _cap(ref.tuples[oracle.MD], mod, 0, caps, q)
    mds = _as_set(md)
    seg = np.array([t for t in ref.tuples[oracle.SEG].tolist()
                    if tuple(t[:2]) in mds and tuple(t[2:]) in mds], np.int64).reshape(-1, 4)
    seg, d1 = _cap(seg, mod, 0, caps, q)
    segs = _as_set(seg)
    t3 = np.array([t for t in ref.tuples[oracle.T3].tolist()
                   if tuple(t[:4]) in segs and tuple(t[2:]) in segs], np.int64).reshape(-1, 6)
    t3, d2 = _cap(t3, mod, 0, caps, q)
    t3s = _as_set(t3)
    score = {tuple(t): s for t, s in zip(ref.tuples[oracle.T5].tolist(), ref.t5_scores)}
    t5 = np.array([t for t in ref.tuples[oracle.T5].tolist()
                   if tuple(t[:6]) in t3s and tuple(t[4:]) in t3s], np.int64).reshape(-1, 10)
    t5, d3 = _cap(t5, mod, 0, caps, q)
    sc = np.array([score[tuple(t)] for t in t5.tolist()], np.float32)
    keep = M.dedup(t5, sc, np.zeros(len(t5), bool)) if len(t5) else np.zeros(0, bool)
    # algorithmic candidate counts of the capped chain
    md_mod = mod[md[:, 0]] if len(md) else np.zeros(0, np.int64)
    n_md = np.bincount(md_mod, minlength=len(ptr) - 1)
    c_seg = sum(int(n_md[a]) * int(n_md[col[ptr[a]:ptr[a + 1]]].sum())
                for a in np.flatnonzero(n_md))
    out_seg = {}
    for t in seg.tolist():
        out_seg[tuple(t[:2])] = out_seg.get(tuple(t[:2]), 0) + 1
    c_t3 = sum(out_seg.get(tuple(t[2:]), 0) for t in seg.tolist())
    out_t3 = {}
    for t in t3.tolist():
        out_t3[tuple(t[:2])] = out_t3.get(tuple(t[:2]), 0) + 1
    c_t5 = sum(out_t3.get(tuple(t[4:]), 0) for t in t3.tolist())
    return dict(caps=caps, sets=[_as_set(x) for x in (md, seg, t3, t5, t5[keep])],
                dropped=[d0, d1, d2, d3], cands=[int(ref.cands[0]), c_seg, c_t3, c_t5])


@pytest.mark.parametrize("cid,event,q", [(1, 0, 0.9), (1, 1, 0.95), (2, 0, 0.97), (5, 0, 0.99)])
def test_capped_chain_is_the_filtered_chain(cid, event, q):
    cfg = E.CONFIGS[cid]
    geo = G.get(cfg.geometry)
    params = PR.make(w=cfg.window)
    ev = E.generate(cid, event, n_tracks=1500 if cid == 5 else None)
    orc = oracle.Oracle(params, geo.f32, geo.i32)
    ref = orc.run_event(ev)
    want = _filtered(ref, ev, q, *orc.module_map())
    caps = want["caps"]
    orc.set_truncation(caps)
    got = orc.run_event(ev)
    for k in range(5):
        assert _as_set(got.tuples[k]) == want["sets"][k], (k, caps)
    assert orc.dropped().tolist() == want["dropped"], (caps, orc.dropped(), want["dropped"])
    assert got.cands.tolist() == want["cands"]
    assert all(d > 0 for d in want["dropped"]), want["dropped"]     # every kind was capped
    # survivors stay pairwise hit-disjoint
    kept = got.tuples[oracle.T5_KEPT]
    assert len(np.unique(kept)) == kept.size
    # capacities off again: the uncapped chain
    orc.set_truncation(None)
    again = orc.run_event(ev)
    assert all(_as_set(again.tuples[k]) == _as_set(ref.tuples[k]) for k in range(5))
    assert orc.dropped().tolist() == [0, 0, 0, 0]


def test_capacity_above_occupancy_changes_nothing():
    geo = G.get("barrel_toy")
    ev = E.generate(1, 0)
    orc = oracle.Oracle(PR.make(), geo.f32, geo.i32)
    ref = orc.run_event(ev)
    orc.set_truncation([10 ** 6] * 4)
    got = orc.run_event(ev)
    assert all(_as_set(got.tuples[k]) == _as_set(ref.tuples[k]) for k in range(5))
    assert orc.dropped().tolist() == [0, 0, 0, 0]
    with pytest.raises(ValueError):
        orc.set_truncation([1, -1, 1, 1])
