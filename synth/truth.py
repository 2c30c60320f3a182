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
