"""Pins of the oracle's enumeration, indexing, module map and duplicate removal.

* brute force on tiny events: every candidate of every stage re-enumerated in
  Python without the oracle's grouping or its module map, each decided by the
  oracle's single-candidate evaluator -> identical object sets;
* truth: on noise-free isolated tracks every true object is built;
* invariants on a full PU200-like event;
* the module map contains every module pair that true tracks above threshold
  link (its purpose, Sec. 2.1).
"""
import itertools

import numpy as np
import pytest

import oracle
from synth import events as E
from synth import geometry as G
from synth import params as PR
from synth import truth as T
from tests.helpers import NEXT, as_set


def _tiny_event(geo_name, n_tracks, seed, noise=0.0, eta=0.8, sigma=True):
    cfg = E.EventConfig(99, geo_name, 1, n_tracks, "logu", 0.9, 10.0, eta, noise_frac=noise)
    rng = E.rng_for(99, seed, 0)
    trk = E._draw_tracks(cfg, rng, n_tracks)
    hel = E.Helices(**trk)
    ev = E.simulate(G.get(geo_name), hel, rng if sigma else None, noise_frac=noise)
    trk["R"] = hel.R
    ev.tracks = trk
    return ev


def _hits6(ev, lo, up):
    return np.r_[ev.x[lo], ev.y[lo], ev.z[lo], ev.x[up], ev.y[up], ev.z[up]]


@pytest.mark.parametrize("geo_name,n_tracks,seed,noise,eta",
                         [("barrel_toy", 12, 1, 0.3, 0.8), ("full", 10, 2, 0.2, 2.4)])
def test_brute_force_equals_oracle(geo_name, n_tracks, seed, noise, eta):
    geo = G.get(geo_name)
    orc = oracle.Oracle(PR.make(), geo.f32, geo.i32)
    ev = _tiny_event(geo_name, n_tracks, seed, noise, eta)
    res = orc.run_event(ev)
    layer = geo.i32[G.I_LAYER]
    ptr, col = orc.module_map()
    edges = set()
    for a in range(geo.n_mod):
        for b in col[ptr[a]:ptr[a + 1]]:
            edges.add((a, int(b)))

    # mini-doublets: all lower x upper pairs of every module
    md = []
    n_cand = [0, 0, 0, 0]
    for lo in np.nonzero(ev.sensor == 0)[0]:
        for up in np.nonzero((ev.sensor == 1) & (ev.module == ev.module[lo]))[0]:
            n_cand[0] += 1
            p, _ = orc.eval_md(int(ev.module[lo]), _hits6(ev, lo, up)[:3], _hits6(ev, lo, up)[3:])
            if p:
                md.append((int(lo), int(up)))
    assert as_set(md) == as_set(res.tuples[oracle.MD])

    # segments: all MD pairs on successive logical layers, no map
    mod_of = {m: int(ev.module[m[0]]) for m in md}
    brute, in_map = set(), set()
    for i, o in itertools.product(md, md):
        a, b = mod_of[i], mod_of[o]
        if layer[b] not in NEXT.get(int(layer[a]), []):
            continue
        p, _ = orc.eval_seg([a, b], np.r_[_hits6(ev, *i), _hits6(ev, *o)])
        if (a, b) in edges:
            n_cand[1] += 1
        if p:
            brute.add(i + o)
            if (a, b) in edges:
                in_map.add(i + o)
    seg = as_set(res.tuples[oracle.SEG])
    assert in_map == seg
    # outside the map only objects that no single track made
    for s in brute - seg:
        t = ev.truth[list(s)]
        assert not (np.all(t == t[0]) and t[0] >= 0 and ev.tracks["pt"][t[0]] >= 0.8)

    # triplets: all segment pairs sharing an MD
    t3 = set()
    segl = sorted(seg)
    by_in = {}
    for s in segl:
        by_in.setdefault(s[:2], []).append(s)
    for s1 in segl:
        for s2 in by_in.get(s1[2:], []):
            n_cand[2] += 1
            mds = [s1[:2], s1[2:], s2[2:]]
            p, _ = orc.eval_t3([mod_of[m] for m in mds], np.concatenate([_hits6(ev, *m) for m in mds]))
            if p:
                t3.add(s1 + s2[2:])
    assert t3 == as_set(res.tuples[oracle.T3])

    # quintuplets: all triplet pairs sharing an MD
    t5 = set()
    by_first = {}
    for t in t3:
        by_first.setdefault(t[:2], []).append(t)
    for t in sorted(t3):
        for u in by_first.get(t[4:], []):
            n_cand[3] += 1
            mds = [t[0:2], t[2:4], t[4:6], u[2:4], u[4:6]]
            p, _ = orc.eval_t5([mod_of[m] for m in mds], np.concatenate([_hits6(ev, *m) for m in mds]))
            if p:
                t5.add(t + u[2:])
    assert t5 == as_set(res.tuples[oracle.T5])
    assert n_cand == res.cands.tolist()


def test_duplicate_removal_all_pairs():
    geo = G.get("full")
    orc = oracle.Oracle(PR.make(), geo.f32, geo.i32)
    ev = E.generate(2, 3)
    res = orc.run_event(ev)
    tup, sc = res.tuples[oracle.T5], res.t5_scores
    n = len(tup)
    assert n > 1000
    sets = [set(r) for r in tup.tolist()]
    keys = [(float(sc[i]), tuple(tup[i])) for i in range(n)]
    owner = {}
    for i, r in enumerate(tup.tolist()):
        for h in r:
            owner.setdefault(h, []).append(i)
    keep = np.ones(n, bool)
    for i in range(n):
        for h in sets[i]:
            for j in owner[h]:
                if j != i and keys[j] < keys[i]:
                    keep[i] = False
    np.testing.assert_array_equal(keep, res.t5_keep)
    # survivors are pairwise hit-disjoint
    seen = set()
    for r in tup[keep].tolist():
        assert not (set(r) & seen)
        seen |= set(r)


def test_invariants_pu200_event():
    geo = G.get("full")
    orc = oracle.Oracle(PR.make(), geo.f32, geo.i32)
    ev = E.generate(2, 0)
    res = orc.run_event(ev)
    md, seg = as_set(res.tuples[oracle.MD]), as_set(res.tuples[oracle.SEG])
    t3, t5 = as_set(res.tuples[oracle.T3]), as_set(res.tuples[oracle.T5])
    for lo, up in md:
        assert ev.module[lo] == ev.module[up] and ev.sensor[lo] == 0 and ev.sensor[up] == 1
    for s in seg:
        assert s[:2] in md and s[2:] in md
    for t in t3:
        assert t[:4] in seg and t[2:] in seg
    for q in t5:
        assert q[:6] in t3 and q[4:] in t3
        assert len(set(q)) == 10
    kept = as_set(res.tuples[oracle.T5_KEPT])
    assert kept <= t5 and len(kept) == int(res.t5_keep.sum())
    # near-threshold records really are near threshold
    for kind in range(4):
        assert np.all(res.near[kind][1] < 1e-5)


def test_margins_off_changes_no_object():
    """the FP64 instance only records near-threshold candidates: switched off,
    every object, candidate count and score is the same and no near record
    is left"""
    geo = G.get("full")
    ev = E.generate(2, 3, n_tracks=600)
    on = oracle.Oracle(PR.make(), geo.f32, geo.i32)
    off = oracle.Oracle(PR.make(), geo.f32, geo.i32)
    off.set_margins(False)
    a, b = on.run_event(ev), off.run_event(ev)
    for k in range(5):
        assert np.array_equal(a.tuples[k], b.tuples[k])
    assert np.array_equal(a.cands, b.cands)
    assert np.array_equal(a.t5_scores.view(np.uint32), b.t5_scores.view(np.uint32))
    assert sum(len(a.near[k][1]) for k in range(4)) > 0
    assert all(len(b.near[k][1]) == 0 for k in range(4))


def test_noise_free_isolated_tracks_are_all_built():
    geo = G.get("barrel_toy")
    orc = oracle.Oracle(PR.make(), geo.f32, geo.i32)
    for seed in range(3):
        ev = _tiny_event("barrel_toy", 8, 10 + seed, noise=0.0, sigma=False)
        res = orc.run_event(ev)
        m = T.metrics(res.tuples[oracle.T5_KEPT], ev, geo)
        assert m["n_findable"] >= 4
        assert m["eff"] == 1.0 and m["fake"] == 0.0
        # every true MD is built
        got = as_set(res.tuples[oracle.MD])
        for lo in np.nonzero(ev.sensor == 0)[0]:
            for up in np.nonzero((ev.sensor == 1) & (ev.module == ev.module[lo]))[0]:
                if ev.truth[lo] == ev.truth[up]:
                    assert (lo, up) in got


def test_module_map_covers_true_links():
    geo = G.get("full")
    orc = oracle.Oracle(PR.make(), geo.f32, geo.i32)
    ptr, col = orc.module_map()
    edges = set()
    for a in range(geo.n_mod):
        edges.update((a, int(b)) for b in col[ptr[a]:ptr[a + 1]])
    layer = geo.i32[G.I_LAYER]
    n_links = 0
    for e in range(3):
        ev = E.generate(2, e, purpose=E.PURPOSE_MAPCHECK)
        pt, z0 = ev.tracks["pt"], ev.tracks["z0"]
        ok = ev.truth >= 0
        per = {}
        for h in np.nonzero(ok)[0]:
            per.setdefault(int(ev.truth[h]), set()).add(int(ev.module[h]))
        for t, mods in per.items():
            if pt[t] < 0.8 or abs(z0[t]) > 15.0:
                continue
            for a in mods:
                for b in mods:
                    if layer[b] in NEXT.get(int(layer[a]), []):
                        n_links += 1
                        assert (a, b) in edges, (t, a, b)
    assert n_links > 10000
