"""Shared test utilities: exact helices, per-layer true mini-doublets, tuple sets."""
import numpy as np

from synth import events as E
from synth import geometry as G

NEXT = {l: ([l + 1] if l < 6 else []) + [7, 12] for l in range(1, 7)}
NEXT.update({l: [l + 1] for l in list(range(7, 11)) + list(range(12, 16))})


def helix(pt, eta, phi0, q, z0=0.0, d0=0.0):
    return E.Helices([pt], [eta], [phi0], [q], [z0], [d0])


def track_mds(geo, ev):
    """First (module, lower hit, upper hit) per logical layer, ordered along the track."""
    layer = geo.i32[G.I_LAYER]
    out = {}
    for h in np.nonzero(ev.sensor == 0)[0]:
        ups = np.nonzero((ev.sensor == 1) & (ev.module == ev.module[h]))[0]
        if len(ups):
            out.setdefault(int(layer[ev.module[h]]), (int(ev.module[h]), int(h), int(ups[0])))
    # order along the track: barrel layers by radius, then disks by |z|
    return [out[l] for l in sorted(out, key=lambda l: (l > 6, l if l <= 11 else l - 5))]


def md_hits(ev, md):
    _, lo, up = md
    return np.r_[ev.x[lo], ev.y[lo], ev.z[lo], ev.x[up], ev.y[up], ev.z[up]].astype(np.float32)


def chain_hits(ev, mds):
    return np.concatenate([md_hits(ev, m) for m in mds])


def as_set(tuples):
    return set(map(tuple, np.asarray(tuples).tolist()))
