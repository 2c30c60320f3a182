"""Half-precision storage of hit positions (the paper's outlook, Sec. 4),
measured with the oracle on PU200-like events of the full geometry.

A hit is stored as its two in-plane coordinates in the module's local frame
(u along the precise axis, v along the coarse axis, relative to the module
centre) rounded to FP16, and its sensor; the FP32 position is rebuilt as
centre + u U + v V + (+-gap/2) W.  Module half-sizes are at most 5.5 cm, so
each FP16 coordinate is within half an ulp of 2^-8 cm (19.5 um) of its
FP32 value.  Rounding the global coordinates to FP16 instead costs up to
2^-6 cm per coordinate at r = 110 cm and is shown for contrast.

Measured on 8 events (seeds 300..307; the tests run the first four): FP16
local storage changes 0.7 % of
the mini-doublets, 2.4 % of the segments, 1 % of the triplets, 0.7 % of the
quintuplets and 6 % of the kept quintuplets (mostly which of two near-equal
duplicates survives); efficiency 97.01 % -> 96.93 %, fake rate unchanged.
Global FP16: efficiency 67 %.

The module-local storage is built: the oracle's storage mode
(`Oracle.set_hit_storage`) is pinned here against NumPy's FP16 conversion
and the positions rebuilt below, and the library's mode
(`lst_set_hit_storage`) is compared with it on the GPU.
"""
import numpy as np
import pytest

import oracle
from synth import events as E
from synth import geometry as G
from synth import params as PR
from synth import truth as T

SEEDS = range(300, 304)
HALF_ULP = 2.0 ** -9      # half an FP16 ulp for 4 <= |u| < 8 cm


def _frame(geo, m):
    f = geo.f32
    col = lambda *ks: [f[k][m] for k in ks]
    return (col(G.F_CX, G.F_CY, G.F_CZ), col(G.F_UX, G.F_UY, G.F_UZ),
            col(G.F_VX, G.F_VY, G.F_VZ), col(G.F_WX, G.F_WY, G.F_WZ), f[G.F_GAP][m])


def _rebuild(geo, ev, store):
    """FP32 positions rebuilt from module-local (u, v) passed through `store`"""
    c, U, V, W, gap = _frame(geo, ev.module)
    d = [(p - c[k]).astype(np.float32) for k, p in enumerate((ev.x, ev.y, ev.z))]
    u = (d[0] * U[0] + d[1] * U[1]) + d[2] * U[2]
    v = (d[0] * V[0] + d[1] * V[1]) + d[2] * V[2]
    u, v = store(u), store(v)
    w = np.where(ev.sensor == 1, np.float32(0.5), np.float32(-0.5)) * gap
    return [(((c[k] + u * U[k]) + v * V[k]) + w * W[k]).astype(np.float32) for k in range(3)]


def _half(a):
    return a.astype(np.float16).astype(np.float32)


VARIANTS = {
    "local_f32": lambda geo, ev: _rebuild(geo, ev, lambda a: a),
    "local_f16": lambda geo, ev: _rebuild(geo, ev, _half),
    "global_f16": lambda geo, ev: [_half(a) for a in (ev.x, ev.y, ev.z)],
}


@pytest.fixture(scope="module")
def study():
    geo = G.get("full")
    orc = oracle.Oracle(PR.make(), geo.f32, geo.i32)
    tup = lambda a: set(map(tuple, a.tolist()))
    out = {k: dict(err=0.0, changed=np.zeros(5), n=np.zeros(5), found=0, fake=0, obj=0)
           for k in ("ref",) + tuple(VARIANTS)}
    n_findable = 0
    for s in SEEDS:
        ev = E.generate(2, s)
        ref = orc.run_event(ev)
        runs = {"ref": ref}
        for name, fn in VARIANTS.items():
            x, y, z = fn(geo, ev)
            err = np.sqrt((x - ev.x).astype(np.float64) ** 2 + (y - ev.y) ** 2 + (z - ev.z) ** 2)
            out[name]["err"] = max(out[name]["err"], float(err.max()))
            runs[name] = orc.run(x, y, z, ev.module, ev.sensor)
        for name, r in runs.items():
            o = out[name]
            for k in range(5):
                o["changed"][k] += len(tup(r.tuples[k]) ^ tup(ref.tuples[k]))
                o["n"][k] += len(ref.tuples[k])
            m = T.metrics(r.tuples[4], ev, geo)
            o["found"] += m["n_found"]
            o["fake"] += m["n_fake"]
            o["obj"] += m["n_obj"]
            if name == "ref":
                n_findable += m["n_findable"]
    for o in out.values():
        o["frac"] = o["changed"] / o["n"]
        o["eff"] = o["found"] / n_findable
        o["fake_rate"] = o["fake"] / max(o["obj"], 1)
    print({k: dict(err_um=1e4 * v["err"], frac=np.round(v["frac"], 5).tolist(), eff=v["eff"],
                   fake=v["fake_rate"]) for k, v in out.items()})
    return out


def test_local_fp16_rounding_stays_within_half_an_ulp(study):
    # u and v each within half an FP16 ulp; the FP32 rebuild adds < 0.2 um
    assert study["local_f16"]["err"] <= np.sqrt(2.0) * HALF_ULP + 2e-5
    assert study["local_f32"]["err"] < 2e-5


def test_the_rebuild_alone_changes_almost_nothing(study):
    # the FP32 round trip through the module frame moves hits by < 0.2 um
    assert np.all(study["local_f32"]["frac"][:4] < 1e-3)
    assert study["local_f32"]["eff"] == pytest.approx(study["ref"]["eff"], abs=1e-3)


def test_local_fp16_costs_little_efficiency(study):
    ref, h = study["ref"], study["local_f16"]
    assert np.all(h["frac"][:4] < 0.05)             # a few % of objects change
    assert h["eff"] >= ref["eff"] - 0.005           # < 0.5 points of efficiency
    assert h["fake_rate"] <= 2 * ref["fake_rate"] + 1e-3


def test_global_fp16_is_far_too_coarse(study):
    assert study["global_f16"]["err"] > 0.05        # > 0.5 mm at the outer layers
    assert study["global_f16"]["eff"] < study["ref"]["eff"] - 0.1


# ---------------------------------------------------------------- the storage mode
def test_oracle_fp16_conversion_is_numpys():
    """the oracle's binary32 -> binary16 rounding (nearest, ties to even) and
    its inverse against NumPy's own conversion: random values over every
    exponent a module coordinate can take and beyond, exact ties between two
    binary16 values, subnormals, and every binary16 bit pattern back"""
    rng = np.random.default_rng(71)
    v = (rng.uniform(-1, 1, 60000) * 2.0 ** rng.integers(-28, 17, 60000)).astype(np.float32)
    h16 = np.arange(0, 0x7c00, 7, dtype=np.uint16)            # finite positive patterns
    lo = h16[:-1].view(np.float16).astype(np.float64)
    hi = (h16[:-1] + 1).view(np.float16).astype(np.float64)
    ties = (0.5 * (lo + hi)).astype(np.float32)                # exact in binary32
    vals = np.concatenate([v, ties, -ties, np.float32([0.0, -0.0, 65504.0, 1e-8])])
    assert np.array_equal(oracle.f32_to_f16_bits(vals), vals.astype(np.float16).view(np.uint16))
    allh = np.arange(0, 0x10000, dtype=np.uint32).astype(np.uint16)
    allh = allh[(allh & 0x7c00) != 0x7c00]                     # no Inf/NaN
    assert np.array_equal(oracle.f16_bits_to_f32(allh).view(np.uint32),
                          allh.view(np.float16).astype(np.float32).view(np.uint32))


@pytest.mark.parametrize("cid,event", [(1, 0), (2, 300)])
def test_oracle_storage_mode_is_the_rebuilt_positions(cid, event):
    """the oracle with half-precision hit storage equals the plain oracle run
    on the positions rebuilt here from NumPy's FP16 rounding of the
    module-local coordinates (same FP32 operation order)"""
    cfg = E.CONFIGS[cid]
    geo = G.get(cfg.geometry)
    params = PR.make(w=cfg.window)
    ev = E.generate(cid, event)
    plain = oracle.Oracle(params, geo.f32, geo.i32)
    x, y, z = _rebuild(geo, ev, _half)
    want = plain.run(x, y, z, ev.module, ev.sensor)
    half = oracle.Oracle(params, geo.f32, geo.i32)
    half.set_hit_storage(True)
    got = half.run_event(ev)
    tup = lambda a: set(map(tuple, a.tolist()))
    for k in range(5):
        assert tup(got.tuples[k]) == tup(want.tuples[k]), k
    assert np.array_equal(got.cands, want.cands)
    # and the mode does change the chain (the rounding is not a no-op)
    ref = plain.run_event(ev)
    assert any(tup(ref.tuples[k]) != tup(got.tuples[k]) for k in range(4))
