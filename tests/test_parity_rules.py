"""CPU checks of the mismatch accounting used by the GPU parity tests: a
difference is excused only as a near-threshold decision or as the cascade
of a difference one stage up (for the kept quintuplets: the quintuplet
itself or one sharing a hit with it)."""
import numpy as np

import oracle
from synth import events as E
from synth import geometry as G
from synth import params as PR
from tests.parity import compare


def _ref():
    geo = G.get("barrel_toy")
    return oracle.Oracle(PR.make(), geo.f32, geo.i32).run_event(E.generate(1, 0))


def _copy(ref):
    return {k: ref.tuples[k].copy() for k in range(5)}


def test_identical_sets_have_no_mismatch():
    ref = _ref()
    rep = compare(_copy(ref), ref, verbose=False)
    assert all(v["mismatch"] == 0 for v in rep.values())


def test_kept_difference_next_to_a_missing_quintuplet_is_a_cascade():
    ref = _ref()
    t5, kept = ref.tuples[oracle.T5], ref.tuples[oracle.T5_KEPT]
    kept_set = set(map(tuple, kept.tolist()))
    # a removed quintuplet that shares hits with a kept one it did not beat
    for i, q in enumerate(t5.tolist()):
        if tuple(q) in kept_set:
            continue
        nb = [k for k in kept.tolist() if set(k) & set(q)]
        if nb:
            break
    else:
        raise AssertionError("no removed quintuplet next to a kept one")
    got = _copy(ref)
    got[oracle.T5] = np.delete(t5, i, axis=0)
    got[oracle.T5_KEPT] = np.array([k for k in kept.tolist() if k != nb[0]], np.int32)
    rep = compare(got, ref, verbose=False)
    assert rep["T5"]["unexplained"] == 1           # the quintuplet itself: no upstream cause
    assert rep["T5_KEPT"]["mismatch"] == 1 and rep["T5_KEPT"]["cascade"] == 1
    assert rep["T5_KEPT"]["unexplained"] == 0


def test_kept_difference_far_from_any_quintuplet_difference_is_unexplained():
    ref = _ref()
    t5, kept = ref.tuples[oracle.T5], ref.tuples[oracle.T5_KEPT]
    got = _copy(ref)
    # one quintuplet differs, and a kept one sharing no hit with it is dropped
    q = t5[0]
    far = [k for k in kept.tolist() if not set(k) & set(q.tolist())]
    got[oracle.T5] = t5[1:]
    got[oracle.T5_KEPT] = np.array([k for k in kept.tolist() if k != far[0]], np.int32)
    rep = compare(got, ref, verbose=False)
    assert rep["T5_KEPT"]["unexplained"] >= 1
