"""Pins of the oracle's scorer features and of its triplet veto.

Features of exact helix tracks are compared with what the helix fixes:
anchor coordinates and module types, curvature 1/R, a zero pull for every
residual of an exact track, slope dz/ds = sinh(eta), chord lengths from the
hits, and the impact parameter of displaced tracks.  The triplet veto is
checked against the relation it must keep: a quintuplet survives a veto iff
neither of its two triplets is vetoed, and duplicate removal then acts on the
survivors alone.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp as M
from synth import events as E
from synth import geometry as G
from synth import params as PR
from tests.helpers import chain_hits, helix, track_mds


@pytest.fixture(scope="module")
def geo_b():
    return G.get("barrel_toy")


@pytest.fixture(scope="module")
def geo_f():
    return G.get("full")


def _track(geo, rng, eta_rng, d0=0.0, z0=None, pt_min=1.0):
    while True:
        pt = math.exp(rng.uniform(math.log(pt_min), math.log(10.0)))
        eta = rng.uniform(*eta_rng)
        hel = helix(pt, eta, rng.uniform(0, 2 * np.pi), rng.choice([-1, 1]),
                    rng.normal(0, 5) if z0 is None else z0, d0)
        ev = E.simulate(geo, hel, None)
        mds = track_mds(geo, ev)
        if len(mds) >= 5:
            return hel, eta, ev, mds


def _anchor(ev, md):
    h = md[1]
    return float(ev.x[h]), float(ev.y[h]), float(ev.z[h])


def _per_md_block(f, geo, ev, mds, n):
    for j in range(n):
        x, y, z = _anchor(ev, mds[j])
        m = mds[j][0]
        assert f[5 * j + 0] == pytest.approx(math.hypot(x, y) / 100, rel=1e-5)
        assert f[5 * j + 1] == pytest.approx(z / 100, rel=1e-5, abs=1e-7)
        assert abs(f[5 * j + 2]) <= 1.0 + 1e-6          # bend pull inside the window
        assert f[5 * j + 3] == float(geo.i32[G.I_SUBDET][m] == 1)
        assert f[5 * j + 4] == float(geo.i32[G.I_TYPE][m] == 1)


@pytest.mark.parametrize("which", ["barrel", "endcap"])
def test_t5_features_of_exact_tracks(which, geo_b, geo_f):
    geo, eta_rng, tol = ((geo_b, (-0.8, 0.8), 2e-4) if which == "barrel"
                         else (geo_f, (1.7, 2.3), 5e-3))
    orc = oracle.Oracle(PR.make(), geo.f32, geo.i32)
    rng = np.random.default_rng(51)
    kmax = orc.consts()["kmax"]
    for _ in range(25):
        hel, eta, ev, mds = _track(geo, rng, eta_rng)
        ok, f = orc.eval_t5_features([m[0] for m in mds[:5]], chain_hits(ev, mds[:5]))
        assert ok
        _per_md_block(f, geo, ev, mds, 5)
        k_true = hel.h[0] / hel.R[0]
        for j in (25, 26, 27):                         # inner, outer, bridge curvature
            assert abs(f[j] * kmax / k_true - 1.0) < tol
        assert f[28] < 1e-2 and f[29] < 1e-2            # chi2/(1+chi2) of an exact track
        assert np.all(np.abs(f[30:37]) < 1e-2)          # pulls and curvature agreement
        assert f[37] == pytest.approx(math.sinh(eta), rel=2e-3)
        xa, ya, _ = _anchor(ev, mds[0])
        xe, ye, _ = _anchor(ev, mds[4])
        assert f[38] == pytest.approx(math.hypot(xe - xa, ye - ya) / 100, rel=1e-5)
        assert abs(f[39]) < 2e-3                        # prompt: no impact parameter


def test_t5_feature_measures_impact_parameter(geo_b):
    """(k_bridge - k_origin) r_a r_e / 2 is the impact parameter to first order
    in d0 and in k r_e: tracks above 3 GeV keep k r_e below 0.35"""
    orc = oracle.Oracle(PR.make(d0max=20.0), geo_b.f32, geo_b.i32)
    rng = np.random.default_rng(52)
    for d0 in (0.5, 1.0, 2.0):
        for _ in range(15):
            hel, eta, ev, mds = _track(geo_b, rng, (-0.5, 0.5), d0=d0 * rng.choice([-1, 1]), z0=0.0,
                                       pt_min=3.0)
            _, f = orc.eval_t5_features([m[0] for m in mds[:5]], chain_hits(ev, mds[:5]))
            assert abs(abs(f[39]) / d0 - 1.0) < 0.05


@pytest.mark.parametrize("which", ["barrel", "endcap"])
def test_t3_features_of_exact_tracks(which, geo_b, geo_f):
    geo, eta_rng, tol = ((geo_b, (-0.8, 0.8), 2e-4) if which == "barrel"
                         else (geo_f, (1.7, 2.3), 5e-3))
    params = PR.make()
    orc = oracle.Oracle(params, geo.f32, geo.i32)
    c = orc.consts()
    rng = np.random.default_rng(53)
    for _ in range(25):
        hel, eta, ev, mds = _track(geo, rng, eta_rng)
        ok, f = orc.eval_t3_features([m[0] for m in mds[:3]], chain_hits(ev, mds[:3]))
        assert ok
        _per_md_block(f, geo, ev, mds, 3)
        k_true = hel.h[0] / hel.R[0]
        assert abs(f[15] * c["kmax"] / k_true - 1.0) < tol
        # T1 ratio: |k| over the threshold bound (plus its resolution term)
        assert 0.0 < f[16] <= 1.0 and f[16] <= (1.0 / hel.R[0]) / c["klim"] * (1 + tol)
        assert abs(f[17]) < 2e-3 and abs(f[18]) < 1e-2   # beam-line and r-z residuals
        assert f[19] == pytest.approx(math.sinh(eta), rel=2e-3)
        xa, ya, _ = _anchor(ev, mds[0])
        xc, yc, _ = _anchor(ev, mds[2])
        assert f[20] == pytest.approx(math.hypot(xc - xa, yc - ya) / 100, rel=1e-5)
        assert abs(f[21]) < 2e-3
        assert not np.any(f[22:])                        # padding


def test_t3_feature_measures_impact_parameter(geo_b):
    orc = oracle.Oracle(PR.make(d0max=20.0), geo_b.f32, geo_b.i32)
    rng = np.random.default_rng(54)
    for d0 in (0.5, 1.0, 2.0):
        for _ in range(15):
            hel, eta, ev, mds = _track(geo_b, rng, (-0.5, 0.5), d0=d0 * rng.choice([-1, 1]), z0=0.0)
            _, f = orc.eval_t3_features([m[0] for m in mds[:3]], chain_hits(ev, mds[:3]))
            assert abs(abs(f[21]) / d0 - 1.0) < 0.05


def test_chain_features_equal_single_candidate_evaluation(geo_b):
    """the features stored by the chain are those of the evaluator for the
    same MDs (checks the bookkeeping, not the formulas)"""
    orc = oracle.Oracle(PR.make(), geo_b.f32, geo_b.i32)
    ev = E.generate(1, 0)
    r = orc.run_event(ev)
    hits = np.stack([ev.x, ev.y, ev.z], 1).astype(np.float32)
    for kind, feats, fn, n in ((oracle.T3, r.t3_features, orc.eval_t3_features, 3),
                               (oracle.T5, r.t5_features, orc.eval_t5_features, 5)):
        tup = r.tuples[kind]
        for i in np.random.default_rng(1).choice(len(tup), 25, replace=False):
            t = tup[i]
            mods = ev.module[t[0::2]]
            hh = np.concatenate([np.r_[hits[t[2 * j]], hits[t[2 * j + 1]]] for j in range(n)])
            _, f = fn(mods, hh)
            assert np.array_equal(f.view(np.uint32), feats[i].view(np.uint32))


# ---------------------------------------------------------------- triplet veto
def test_rerun_without_veto_reproduces_the_chain(geo_b):
    orc = oracle.Oracle(PR.make(), geo_b.f32, geo_b.i32)
    r = orc.run_event(E.generate(1, 1))
    r2 = orc.rerun_t5(None)
    for k in (oracle.T5, oracle.T5_KEPT):
        assert np.array_equal(r.tuples[k], r2.tuples[k])
    assert np.array_equal(r.t5_scores.view(np.uint32), r2.t5_scores.view(np.uint32))
    assert np.array_equal(r.cands, r2.cands)


@pytest.mark.parametrize("cid", [1, 2])
def test_triplet_veto_keeps_exactly_the_quintuplets_of_surviving_triplets(cid):
    geo = G.get(E.CONFIGS[cid].geometry)
    orc = oracle.Oracle(PR.make(), geo.f32, geo.i32)
    r = orc.run_event(E.generate(cid, 0))
    t3 = r.tuples[oracle.T3]
    rng = np.random.default_rng(cid)
    veto = rng.random(len(t3)) < 0.3
    vetoed = {tuple(t) for t in t3[veto].tolist()}
    r2 = orc.rerun_t5(veto)
    # a T5 (a, b, c, d, e) is built from triplets (a, b, c) and (c, d, e)
    def parts(t):
        return tuple(t[:6]), tuple(t[4:])
    want = [i for i, t in enumerate(r.tuples[oracle.T5].tolist())
            if not (set(parts(t)) & vetoed)]
    assert {tuple(t) for t in r2.tuples[oracle.T5].tolist()} == \
        {tuple(r.tuples[oracle.T5][i]) for i in want}
    # candidate pairs are counted with or without the veto
    assert np.array_equal(r.cands, r2.cands)
    # duplicate removal acts on the survivors alone
    keep = M.dedup(r2.tuples[oracle.T5], r2.t5_scores, np.zeros(len(r2.tuples[oracle.T5]), bool))
    assert np.array_equal(keep, r2.t5_keep)
    assert len(orc.rerun_t5(np.ones(len(t3), np.uint8)).tuples[oracle.T5]) == 0
