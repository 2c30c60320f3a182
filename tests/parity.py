"""Object-set comparison of the HIP chain with the oracle, with the
near-threshold and cascade accounting of mismatches."""
import numpy as np

KINDS = ("MD", "SEG", "T3", "T5", "T5_KEPT")
SUB = {1: (0, [(0, 2), (2, 4)]), 2: (1, [(0, 4), (2, 6)]), 3: (2, [(0, 6), (4, 10)])}


def _set(a):
    return set(map(tuple, np.asarray(a).tolist()))


def compare(gpu: dict, ref, verbose=True):
    """gpu: kind -> int32 tuples; ref: oracle.Result.  Returns a report dict;
    'unexplained' counts mismatches that are neither near threshold nor
    descendants of an upstream mismatch."""
    report = {}
    diffs = {}
    for kind in range(5):
        g, o = _set(gpu[kind]), _set(ref.tuples[kind])
        d = g ^ o
        diffs[kind] = d
        near = set()
        if kind < 4:
            near = _set(ref.near[kind][0]) if len(ref.near[kind][0]) else set()
        casc = set()
        if kind in SUB:
            up, parts = SUB[kind]
            for t in d:
                if any(tuple(t[a:b]) in diffs[up] for a, b in parts):
                    casc.add(t)
        if kind == 4:
            # duplicate removal decides a quintuplet from the quintuplets that
            # share one of its hits (one pass), so a kept-set difference is a
            # cascade only when the quintuplet itself, or one sharing a hit
            # with it, differs between the two sides
            dhits = {h for q in diffs[3] for h in q}
            casc = {t for t in d if t in diffs[3] or (set(t) & dhits)}
        near_d = {t for t in d if t in near}
        unexplained = d - near_d - casc
        report[KINDS[kind]] = dict(gpu=len(g), oracle=len(o), mismatch=len(d), near=len(near_d),
                                   cascade=len(casc - near_d), unexplained=len(unexplained))
    if verbose:
        print(report, flush=True)
    return report


def assert_parity(gpu: dict, ref):
    rep = compare(gpu, ref)
    for k, v in rep.items():
        assert v["unexplained"] == 0, (k, rep)
    return rep
