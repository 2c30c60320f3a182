"""Truth matching of output objects against the simulated tracks.

Reporting only (no Segment Linking arithmetic): efficiency, fake rate and
duplicate rate of quintuplets, with the definitions this project adopts since
the paper states none (Sec. 2.2): an object matches a simulated track when at
least 8 of its 10 hits come from it; a track is findable when p_T >= 0.8 GeV
and it left a lower+upper hit pair in one module on at least five
consecutive logical layers; a fake is an object matching no track; a
duplicate is any further object matching an already matched track.
"""
from __future__ import annotations

import numpy as np

from . import geometry as G

# chains of consecutive logical layers (barrel 1..6 then the disks of one side)
_NEXT = {l: ([l + 1] if l < 6 else []) + [7, 12] for l in range(1, 7)}
_NEXT.update({l: [l + 1] for l in list(range(7, 11)) + list(range(12, 16))})


def true_md_layers(ev, geo: G.Geometry):
    """track id -> set of logical layers where it has a lower+upper pair in one module."""
    t = ev.truth
    ok = t >= 0
    key = (t[ok].astype(np.int64) << 20) | ev.module[ok].astype(np.int64)
    sen = ev.sensor[ok]
    lo = set(key[sen == 0].tolist())
    up = set(key[sen == 1].tolist())
    out = {}
    layer = geo.i32[G.I_LAYER]
    for k in lo & up:
        tr, m = k >> 20, k & ((1 << 20) - 1)
        out.setdefault(int(tr), set()).add(int(layer[m]))
    return out


def _longest_chain(layers: set) -> int:
    best = {}
    for l in sorted(layers, reverse=True):
        best[l] = 1 + max([best[n] for n in _NEXT.get(l, []) if n in best], default=0)
    return max(best.values(), default=0)


def findable(ev, geo: G.Geometry, pt_min=0.8, n_layers=5):
    lays = true_md_layers(ev, geo)
    pt = ev.tracks["pt"]
    return np.array(sorted(t for t, ls in lays.items()
                           if pt[t] >= pt_min and _longest_chain(ls) >= n_layers), dtype=np.int64)


def match(tuples: np.ndarray, truth: np.ndarray, min_hits=8):
    """track id matched by each object (-1 when none)."""
    if len(tuples) == 0:
        return np.zeros(0, np.int64)
    tt = truth[tuples]
    out = np.full(len(tuples), -1, np.int64)
    for i, row in enumerate(tt):
        ids, cnt = np.unique(row[row >= 0], return_counts=True)
        if len(cnt) and cnt.max() >= min_hits:
            out[i] = ids[np.argmax(cnt)]
    return out


def metrics(t5_tuples: np.ndarray, ev, geo: G.Geometry) -> dict:
    fnd = findable(ev, geo)
    m = match(t5_tuples, ev.truth)
    matched = set(m[m >= 0].tolist())
    n = len(t5_tuples)
    found = len(set(fnd.tolist()) & matched)
    n_fake = int(np.sum(m < 0))
    n_dup = int(np.sum(m >= 0) - len(matched))
    return dict(n_obj=n, n_findable=int(len(fnd)), n_found=found,
                eff=found / max(len(fnd), 1), fake=n_fake / max(n, 1), dup=n_dup / max(n, 1),
                n_fake=n_fake, n_dup=n_dup)


def tc_metrics(tc, ev, px, geo: G.Geometry) -> dict:
    """Track candidates (rows: type, seed, 10 outer hits -1 padded) against
    the simulated tracks.  A candidate matches a track when at least 75 % of
    its hits (outer hits and its seed's four pixel hits) come from it;
    findable = p_T >= 0.8 GeV and either quintuplet-findable (five
    consecutive layers with a hit pair) or with a hit on all four pixel
    layers."""
    tc = np.asarray(tc).reshape(-1, 12)
    ptr = ev.tracks["pt"]
    fnd = set(findable(ev, geo).tolist())
    px_tr = {}
    for h, t in enumerate(px.truth.tolist()):
        px_tr[t] = px_tr.get(t, 0) + 1
    fnd |= {t for t, n in px_tr.items() if n == 4 and ptr[t] >= 0.8}
    match = []
    for row in tc:
        hits = [int(ev.truth[h]) for h in row[2:] if h >= 0]
        if row[1] >= 0:
            hits += [int(px.truth[h]) for h in px.seeds[row[1]]]
        ids, cnt = np.unique([h for h in hits if h >= 0], return_counts=True)
        ok = len(cnt) and cnt.max() >= 0.75 * len(hits)
        match.append(int(ids[np.argmax(cnt)]) if ok else -1)
    match = np.array(match, np.int64)
    matched = set(match[match >= 0].tolist())
    n = len(tc)
    n_fake = int(np.sum(match < 0))
    n_dup = int(np.sum(match >= 0) - len(matched))
    found = len(fnd & matched)
    by_type = {int(t): int(np.sum(tc[:, 0] == t)) for t in range(4)}
    return dict(n_obj=n, n_findable=len(fnd), n_found=found, eff=found / max(len(fnd), 1),
                fake=n_fake / max(n, 1), dup=n_dup / max(n, 1), n_fake=n_fake, n_dup=n_dup,
                by_type=by_type)
