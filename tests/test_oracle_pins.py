"""Pins of the CPU oracle against closed forms, thresholds and statistics.

None of these re-types an oracle formula: each compares what the oracle
computes with a fact fixed by geometry or by the method's definition
(threshold p_T, circle through three points, straight line in arc length,
chi-square with the right number of degrees of freedom).
"""
import math

import numpy as np
import pytest

import oracle
from synth import events as E
from synth import geometry as G
from synth import params as PR
from tests.helpers import chain_hits, helix, track_mds

PT_THR = 0.8


@pytest.fixture(scope="module")
def geo_b():
    return G.get("barrel_toy")


@pytest.fixture(scope="module")
def geo_f():
    return G.get("full")


def _sharp(geo, **over):
    """resolution-free, margin-free parameters: windows are the bare helix bounds"""
    p = dict(sigu=1e-7, sigv=1e-7, epsk=0.0, epsa=0.0)
    p.update(over)
    return oracle.Oracle(PR.make(**p), geo.f32, geo.i32)


# ---------------------------------------------------------------- generator
def test_generator_exact_hits_on_helix_and_planes(geo_b, geo_f):
    rng = np.random.default_rng(3)
    for geo, etamax in ((geo_b, 0.8), (geo_f, 2.4)):
        for _ in range(40):
            pt, eta = rng.uniform(1, 10), rng.uniform(-etamax, etamax)
            phi0, q, z0 = rng.uniform(0, 2 * np.pi), rng.choice([-1, 1]), rng.normal(0, 5)
            hel = helix(pt, eta, phi0, q, z0)
            ev = E.simulate(geo, hel, None)
            assert ev.n_hits >= 6
            R = pt / (E.K_B * E.B_FIELD)            # p_T = 0.2998 B[T] R[m]
            h = -q
            cx, cy = h * R * (-np.sin(phi0)), h * R * np.cos(phi0)
            x, y, z = ev.x.astype(float), ev.y.astype(float), ev.z.astype(float)
            np.testing.assert_allclose(np.hypot(x - cx, y - cy), R, rtol=2e-6)
            r = np.hypot(x, y)
            s = 2 * R * np.arcsin(r / (2 * R))       # arc length from the beam line
            np.testing.assert_allclose(z, z0 + s * np.sinh(eta), atol=2e-4)
            f = geo.f64
            m = ev.module
            d = (x - f[G.F_CX, m]) * f[G.F_WX, m] + (y - f[G.F_CY, m]) * f[G.F_WY, m] + \
                (z - f[G.F_CZ, m]) * f[G.F_WZ, m]
            np.testing.assert_allclose(d, (ev.sensor - 0.5) * f[G.F_GAP, m], atol=2e-4)


def test_derived_constants_closed_form(geo_b):
    k = oracle.Oracle(PR.make(), geo_b.f32, geo_b.i32).consts()
    # kappa_max = 0.299792458 B / p_T[GeV] per metre: R_min = 70.22 cm at 0.8 GeV, 3.8 T
    assert abs(1.0 / k["kmax"] - 70.2245) < 1e-3
    assert abs(k["kh"] - 0.5 * k["kmax"] * 1.05) < 1e-8


# ---------------------------------------------------------------- MD window
@pytest.mark.parametrize("which", ["barrel", "endcap"])
def test_md_window_is_the_pt_threshold(which, geo_b, geo_f):
    geo = geo_b if which == "barrel" else geo_f
    # the endcap step length between sensors depends on the vertex z, so the
    # window is only sharp with the luminous region shrunk to a point
    orc = _sharp(geo) if which == "barrel" else _sharp(geo, z0max=1e-3)
    rng = np.random.default_rng(5)
    n_checked = 0
    for _ in range(30):
        phi0, q = rng.uniform(0, 2 * np.pi), rng.choice([-1, 1])
        eta = rng.uniform(-0.6, 0.6) if which == "barrel" else rng.uniform(1.7, 2.2)
        for scale, expect in ((1.02, True), (0.85, False)):
            ev = E.simulate(geo, helix(PT_THR * scale, eta, phi0, q, 0.0), None)
            mds = track_mds(geo, ev)
            if which == "endcap":
                mds = [m for m in mds if geo.i32[G.I_SUBDET, m[0]] == 1]
            for m in mds:
                p, out = orc.eval_md(m[0], chain_hits(ev, [m])[:3], chain_hits(ev, [m])[3:])
                bend_ok = out[0] <= out[1]
                assert bend_ok == expect, (scale, out)
                n_checked += 1
    assert n_checked > 100


# ---------------------------------------------------------------- segment
def _track(geo, rng, eta_rng, pt_rng=(1.0, 10.0), z0=None, d0=0.0):
    while True:
        pt = math.exp(rng.uniform(math.log(pt_rng[0]), math.log(pt_rng[1])))
        eta = rng.uniform(*eta_rng)
        phi0, q = rng.uniform(0, 2 * np.pi), rng.choice([-1, 1])
        zz = rng.normal(0, 5) if z0 is None else z0
        hel = helix(pt, eta, phi0, q, zz, d0)
        ev = E.simulate(geo, hel, None)
        mds = track_mds(geo, ev)
        if len(mds) >= 5:
            return hel, ev, mds


@pytest.mark.parametrize("which", ["barrel", "endcap"])
def test_segment_azimuth_window_is_the_pt_threshold(which, geo_b, geo_f):
    geo = geo_b if which == "barrel" else geo_f
    orc = _sharp(geo)
    rng = np.random.default_rng(11)
    eta_rng = (-0.6, 0.6) if which == "barrel" else (1.8, 2.2)
    n = 0
    for _ in range(25):
        phi0, q, eta = rng.uniform(0, 2 * np.pi), rng.choice([-1, 1]), rng.uniform(*eta_rng)
        for scale, expect in ((1.002, True), (0.99, False)):
            ev = E.simulate(geo, helix(PT_THR * scale, eta, phi0, q, 0.0), None)
            mds = track_mds(geo, ev)
            for a, b in zip(mds[:-1], mds[1:]):
                _, out = orc.eval_seg([a[0], b[0]], chain_hits(ev, [a, b]))
                assert (out[2] <= out[3]) == expect, (scale, out[2], out[3])
                n += 1
    assert n > 50


@pytest.mark.parametrize("which", ["barrel", "endcap"])
def test_segment_pointing_recovers_z0_and_prompt_circle(which, geo_b, geo_f):
    geo = geo_b if which == "barrel" else geo_f
    orc = oracle.Oracle(PR.make(), geo.f32, geo.i32)
    rng = np.random.default_rng(12)
    eta_rng = (-0.8, 0.8) if which == "barrel" else (1.7, 2.3)
    for _ in range(40):
        hel, ev, mds = _track(geo, rng, eta_rng, pt_rng=(2.0, 10.0))
        R, h, z0 = hel.R[0], hel.h[0], hel.z0[0]
        for a, b in zip(mds[:-1], mds[1:]):
            p, out = orc.eval_seg([a[0], b[0]], chain_hits(ev, [a, b]))
            assert p
            # circle through the beam line and both anchors = the track circle
            assert abs(out[11] * R * h - 1.0) < (2e-3 if which == "endcap" else 1e-4)
            # straight line in arc length points back to the true z0
            tol = 2e-2 if which == "endcap" else 2e-3
            assert abs(out[10] - z0) < tol, (out[10], z0)
            # relative angle: MD direction vs chord equals the prompt-circle prediction
            kappa = 1.0 / R
            if out[7] > 0:
                assert out[6] <= kappa * 0.5 + 2e-4
            if out[9] > 0:
                assert out[8] <= kappa * 0.5 + 2e-4


# ---------------------------------------------------------------- triplet
def test_triplet_circle_and_line_closed_forms(geo_b, geo_f):
    rng = np.random.default_rng(21)
    for geo, eta_rng in ((geo_b, (-0.8, 0.8)), (geo_f, (1.7, 2.3))):
        orc = oracle.Oracle(PR.make(), geo.f32, geo.i32)
        for _ in range(40):
            hel, ev, mds = _track(geo, rng, eta_rng)
            R, h = hel.R[0], hel.h[0]
            for j in range(len(mds) - 2):
                p, out = orc.eval_t3([m[0] for m in mds[j:j + 3]], chain_hits(ev, mds[j:j + 3]))
                assert p
                # curvature of the circle through three points of a helix = 1/R, signed
                assert abs(out[6] * R * h - 1.0) < (2e-4 if geo is geo_b else 5e-3)
                # prompt: the circle also passes through the beam line
                assert out[2] < 2e-6
                # z linear in arc length: the middle anchor is on the line
                assert out[4] < 2e-4


def test_triplet_beamline_cut_measures_impact_parameter(geo_b):
    orc = oracle.Oracle(PR.make(), geo_b.f32, geo_b.i32)
    rng = np.random.default_rng(22)
    for d0 in (0.5, 1.0, 2.0):
        for _ in range(20):
            hel, ev, mds = _track(geo_b, rng, (-0.5, 0.5), z0=0.0,
                                  d0=d0 * rng.choice([-1, 1]))
            _, out = orc.eval_t3([m[0] for m in mds[:3]], chain_hits(ev, mds[:3]))
            ra = np.hypot(ev.x[mds[0][1]], ev.y[mds[0][1]])
            rc = np.hypot(ev.x[mds[2][1]], ev.y[mds[2][1]])
            # first order: |k - k_origin| = 2 |d0| / (r_a r_c)
            assert abs(out[2] / (2 * d0 / (ra * rc)) - 1.0) < 0.05


def test_triplet_curvature_cut_is_the_pt_threshold(geo_b):
    orc = _sharp(geo_b)
    rng = np.random.default_rng(23)
    n = 0
    for _ in range(30):
        phi0, q, eta = rng.uniform(0, 2 * np.pi), rng.choice([-1, 1]), rng.uniform(-0.6, 0.6)
        for scale, expect in ((1.001, True), (0.99, False)):
            ev = E.simulate(geo_b, helix(PT_THR * scale, eta, phi0, q, 0.0), None)
            mds = track_mds(geo_b, ev)
            for j in range(len(mds) - 2):
                _, out = orc.eval_t3([m[0] for m in mds[j:j + 3]], chain_hits(ev, mds[j:j + 3]))
                assert (out[0] <= out[1]) == expect
                n += 1
    assert n > 50


# ---------------------------------------------------------------- quintuplet
def test_quintuplet_exact_track_has_zero_residuals(geo_b, geo_f):
    rng = np.random.default_rng(31)
    for geo, eta_rng in ((geo_b, (-0.8, 0.8)), (geo_f, (1.7, 2.3))):
        orc = oracle.Oracle(PR.make(), geo.f32, geo.i32)
        for _ in range(30):
            hel, ev, mds = _track(geo, rng, eta_rng)
            R, h = hel.R[0], hel.h[0]
            p, out = orc.eval_t5([m[0] for m in mds[:5]], chain_hits(ev, mds[:5]))
            assert p
            assert abs(out[12] * R * h - 1.0) < (2e-4 if geo is geo_b else 5e-3)
            assert abs(out[13]) < 1e-4 and abs(out[14]) < 1e-4
            assert out[15] < 1e-2 and out[16] < 1e-2


@pytest.mark.parametrize("which", ["barrel", "endcap"])
def test_quintuplet_chi2_has_its_degrees_of_freedom(which, geo_b, geo_f):
    """With the nominal Gaussian smearing the r-phi chi2 (two residuals) must
    average 2 and the r-z chi2 (three residuals) 3: pins every variance term."""
    geo = geo_b if which == "barrel" else geo_f
    orc = oracle.Oracle(PR.make(), geo.f32, geo.i32)
    rng = np.random.default_rng(41)
    eta_rng = (-0.8, 0.8) if which == "barrel" else (1.9, 2.3)
    c2p, c2z = [], []
    while len(c2p) < 1200:
        pt = math.exp(rng.uniform(0.0, math.log(10)))
        hel = helix(pt, rng.uniform(*eta_rng), rng.uniform(0, 2 * np.pi), rng.choice([-1, 1]),
                    rng.normal(0, 5))
        ev = E.simulate(geo, hel, rng, shuffle=False)
        mds = track_mds(geo, ev)
        if len(mds) < 5:
            continue
        _, out = orc.eval_t5([m[0] for m in mds[:5]], chain_hits(ev, mds[:5]))
        c2p.append(out[15]); c2z.append(out[16])
    c2p, c2z = np.array(c2p), np.array(c2z)
    assert abs(c2p.mean() - 2.0) < 0.2, c2p.mean()
    assert abs(c2z.mean() - 3.0) < 0.25, c2z.mean()


# ---------------------------------------------------------------- MD coarse window
Z0MAX = 15.0


def _straight(geo, eta, phi0, q, z0):
    """an (almost) straight track: p_T 10 TeV, so arc length equals radius to 1e-9"""
    ev = E.simulate(geo, helix(1e4, eta, phi0, q, z0), None)
    return ev, track_mds(geo, ev)


def _coarse_ok(orc, ev, m):
    h = chain_hits(ev, [m])
    _, out = orc.eval_md(m[0], h[:3], h[3:])
    return out[2] <= out[3]


def test_md_coarse_window_is_the_luminous_region_barrel(geo_b):
    """Sec. 2: a stub points back to the luminous region.  For a straight
    track from (0, 0, z0) the displacement between the sensors along z is
    the transverse step times (z_L - z0)/r_L, so with the resolution term
    removed the coarse half of the MD window passes exactly when
    |z0| <= Z0MAX, on every barrel layer and on both sides of the vertex."""
    orc = _sharp(geo_b)
    rng = np.random.default_rng(51)
    n = 0
    for _ in range(25):
        phi0, q, s = rng.uniform(0, 2 * np.pi), rng.choice([-1, 1]), rng.choice([-1.0, 1.0])
        eta = rng.uniform(-0.6, 0.6)
        for d in (0.01, 0.3, 2.0):
            for z0, expect in ((s * (Z0MAX - d), True), (s * (Z0MAX + d), False)):
                ev, mds = _straight(geo_b, eta, phi0, q, z0)
                for m in mds:
                    assert _coarse_ok(orc, ev, m) == expect, (z0, m)
                    n += 1
    assert n > 800


def test_md_coarse_window_is_the_luminous_region_endcap(geo_f):
    """Endcap (coarse axis radial, sensors stacked along z): the transverse
    step over the gap g is D = g r_L / (|z_L| - s z0) for a straight track
    (s = side of the disk).  The window runs from the straight track of the
    far vertex edge, s z0 = -Z0MAX (smallest step), to the threshold-p_T helix
    from the near edge, whose step is longer by its arc-over-chord factor
    F = asin(a)/a, a = r_L kappa_max / 2: a straight track passes up to
    s z0 = |z_L| - (|z_L| - Z0MAX) / F.  Both edges are checked on exact
    hits; the high edge within 0.1 cm, because the chain's arc-length series
    bounds asin(a)/a from above by at most 3e-4 relative, and the far edge
    from 0.05 cm on."""
    orc = _sharp(geo_f)
    kmax = float(orc.consts()["kmax"])
    rng = np.random.default_rng(52)

    def zlim(ev, m):
        h = chain_hits(ev, [m])
        rl, zl = math.hypot(h[0], h[1]), abs(float(h[2]))
        a = 0.5 * rl * kmax
        return zl - (zl - Z0MAX) / (math.asin(a) / a)

    def disk_mds(ev, mds):
        return [m for m in mds if geo_f.i32[G.I_SUBDET, m[0]] == 1]

    n_lo, hi = 0, {True: 0, False: 0}
    for _ in range(25):
        phi0, q, s = rng.uniform(0, 2 * np.pi), rng.choice([-1, 1]), rng.choice([-1.0, 1.0])
        eta = s * rng.uniform(1.7, 2.3)
        # far edge: s z0 = -Z0MAX (0.05 cm moves the step by ~2e-5 cm, eight
        # times the FP32 rounding of the hit coordinates)
        for d in (0.05, 0.3, 2.0):
            for z0, expect in ((-s * (Z0MAX - d), True), (-s * (Z0MAX + d), False)):
                ev, mds = _straight(geo_f, eta, phi0, q, z0)
                for m in disk_mds(ev, mds):
                    assert _coarse_ok(orc, ev, m) == expect, (z0, m)
                    n_lo += 1
        # near edge: the threshold-helix limit of each disk MD's module
        ev0, mds0 = _straight(geo_f, eta, phi0, q, s * 20.0)
        for m0 in disk_mds(ev0, mds0):
            for d in (0.15, -0.15, 0.4, -0.4, 1.0, -1.0):
                z0 = s * (zlim(ev0, m0) - d)
                ev, mds = _straight(geo_f, eta, phi0, q, z0)
                for m in disk_mds(ev, mds):
                    if m[0] != m0[0]:
                        continue
                    # the limit of the hit this vertex produces
                    lim = zlim(ev, m)
                    if abs(lim - s * z0) < 0.1:
                        continue
                    inside = bool(s * z0 < lim)
                    assert _coarse_ok(orc, ev, m) == inside, (z0, lim, m)
                    hi[inside] += 1
    assert n_lo > 400 and min(hi.values()) > 40, (n_lo, hi)


@pytest.mark.parametrize("which", ["barrel", "endcap"])
def test_md_coarse_window_contains_threshold_helices(which, geo_b, geo_f):
    """The coarse window is written for straight tracks; a helix at the
    threshold p_T arrives with its arc longer than its radius and its step
    turned away from the radial axis.  With the nominal resolution term the
    window still holds every exact helix from the edge of the luminous region
    (|z0| = 14.9 cm) at 0.8 GeV and above, both charges, every layer and disk,
    using at most a quarter of its width."""
    geo = geo_b if which == "barrel" else geo_f
    orc = oracle.Oracle(PR.make(), geo.f32, geo.i32)
    rng = np.random.default_rng(53)
    worst, n = 0.0, 0
    for _ in range(150):
        phi0, q = rng.uniform(0, 2 * np.pi), rng.choice([-1, 1])
        eta = rng.uniform(-0.9, 0.9) if which == "barrel" else \
            rng.uniform(1.2, 2.4) * rng.choice([-1, 1])
        pt = PT_THR * rng.choice([1.0, 1.001, 1.5, 3.0, 100.0])
        ev = E.simulate(geo, helix(pt, eta, phi0, q, rng.choice([-1, 1]) * 14.9), None)
        for m in track_mds(geo, ev):
            h = chain_hits(ev, [m])
            _, out = orc.eval_md(m[0], h[:3], h[3:])
            worst = max(worst, out[2] / out[3])
            n += 1
    assert n > 800 and worst < 0.25, (n, worst)


# ---------------------------------------------------------------- quintuplet bridge curvature
@pytest.mark.parametrize("which", ["barrel", "endcap"])
@pytest.mark.parametrize("epsk", [0.0, 0.05])
def test_quintuplet_bridge_curvature_cut_is_the_pt_threshold(which, epsk, geo_b, geo_f):
    """Q2: the circle through the first, middle and last anchors has the
    track's curvature, so the bridge cut passes exactly the helices with p_T
    above the threshold lowered by the curvature margin, 0.8 / (1 + EPSK) GeV.
    Exact helices at 1.001x that p_T pass Q2 and at 0.999x fail it, while
    the other four quintuplet cuts pass on both sides."""
    geo = geo_b if which == "barrel" else geo_f
    orc = oracle.Oracle(PR.make(epsk=epsk), geo.f32, geo.i32)
    p_edge = PT_THR / (1.0 + epsk)
    rng = np.random.default_rng(54)
    n = 0
    for _ in range(30):
        phi0, q = rng.uniform(0, 2 * np.pi), rng.choice([-1, 1])
        eta = rng.uniform(-0.6, 0.6) if which == "barrel" else \
            rng.uniform(1.6, 2.3) * rng.choice([-1, 1])
        z0 = rng.normal(0, 5)
        for scale, expect in ((1.001, True), (0.999, False)):
            ev = E.simulate(geo, helix(p_edge * scale, eta, phi0, q, z0), None)
            mds = track_mds(geo, ev)
            for j in range(len(mds) - 4):
                _, out = orc.eval_t5([m[0] for m in mds[j:j + 5]], chain_hits(ev, mds[j:j + 5]))
                ok = [out[2 * i] <= out[2 * i + 1] for i in range(5)]
                assert ok[2] == expect, (scale, out[4], out[5])
                assert ok[0] and ok[1] and ok[3] and ok[4], (scale, out[:10])
                n += 1
    assert n > 40


# ---------------------------------------------------------------- FP64 decision margin
def test_cut_margin_is_the_relative_distance_of_the_deciding_cut(geo_b):
    """The margin that decides which GPU/oracle disagreements are allowed is
    the relative distance to threshold of the one cut that decides the
    candidate.  Segments of straight tracks from z0 = +-Z0MAX (1 -+ delta)
    are built with the coarse resolution removed, so the pointing cut S1
    (|z0| <= Z0MAX) sits at a known relative distance delta from its
    threshold and the other cuts are far from theirs:
      * S1 passing by delta, all else passing: margin = delta;
      * S1 failing by delta, all else passing: margin = delta;
      * S1 failing by delta and the outer MD turned by 0.3 rad (the
        relative-angle cut S3 fails as well): no single flip changes the
        decision, margin = infinity;
      * S1 passing by delta, S3 failing: margin = S3's distance, not delta."""
    orc = _sharp(geo_b, sigu=PR.DEFAULTS["sigu"], epsk=PR.DEFAULTS["epsk"],
                 epsa=PR.DEFAULTS["epsa"])
    rng = np.random.default_rng(55)
    n = {"pass": 0, "fail": 0, "inf": 0, "other": 0}
    for delta in (8e-6, 2e-5, 1e-4, 1e-3):
        for _ in range(8):
            phi0, q, s = rng.uniform(0, 2 * np.pi), rng.choice([-1, 1]), rng.choice([-1.0, 1.0])
            eta = rng.uniform(-0.5, 0.5)
            for side, expect in ((1, True), (-1, False)):
                ev, mds = _straight(geo_b, eta, phi0, q, s * Z0MAX * (1 - side * delta))
                for a, b in zip(mds[:-1], mds[1:]):
                    h = chain_hits(ev, [a, b])
                    p, _ = orc.eval_seg([a[0], b[0]], h)
                    assert p == expect
                    mg = orc.eval_margin(oracle.SEG, [a[0], b[0]], h)
                    # FP32 hit positions move the z0 estimate by ~1e-5 cm
                    assert abs(mg - delta) <= 3e-6 + delta * delta, (delta, mg)
                    n["pass" if expect else "fail"] += 1
                    t = h.copy()
                    dx, dy = t[9] - t[6], t[10] - t[7]
                    c, sn = math.cos(0.3), math.sin(0.3)
                    t[9], t[10] = t[6] + c * dx - sn * dy, t[7] + sn * dx + c * dy
                    p2, out2 = orc.eval_seg([a[0], b[0]], t)
                    assert not p2 and out2[8] > out2[9]
                    mg2 = orc.eval_margin(oracle.SEG, [a[0], b[0]], t)
                    if expect:
                        rel = (out2[8] - out2[9]) / out2[8]
                        assert abs(mg2 - rel) < 1e-5 and mg2 > 0.1, (mg2, rel)
                        n["other"] += 1
                    else:
                        assert math.isinf(mg2), mg2
                        n["inf"] += 1
    assert min(n.values()) > 50, n
