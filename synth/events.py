"""Seeded synthetic events: charged helices in a solenoid, crossing p_T modules.

Input generator shared by the HIP library tests, the benchmark and the CPU
oracle.  It simulates the detector response only (exact helix/sensor-plane
intersections, Gaussian smearing along the module axes, hit inefficiency and
uniform noise); it holds none of the Segment Linking arithmetic.

The paper measures on CMS Phase-2 t-tbar PU200 simulation and a muon gun
(Sec. 2.2, Sec. 3); neither is available, so these seeded events of the same
character stand in for them.  Every random number comes from one NumPy PCG64
stream per (config, event, purpose) built with ``SeedSequence``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

from . import geometry as G

K_B = 0.0029979245800    # GeV per (T cm): p_T = K_B * B * R
B_FIELD = 3.8             # T
SIGMA_U = 0.0030          # cm, precise-axis smearing (30 um)
SIGMA_V = 0.15            # cm, coarse-axis smearing (1.5 mm)

PURPOSE_EVAL, PURPOSE_TRAIN, PURPOSE_MAPCHECK = 0, 1, 2


@dataclass
class EventConfig:
    cid: int
    geometry: str
    n_events: int
    n_tracks: int            # fixed multiplicity (ignored when pileup_range set)
    spectrum: str            # "logu" (log-uniform pt_lo..pt_hi) or "pow3" (dN/dpT ~ pT^-3 above pt_lo)
    pt_lo: float
    pt_hi: float
    eta_max: float
    noise_frac: float = 0.0
    ineff: float = 0.0
    displaced_frac: float = 0.0
    d0_max: float = 10.0
    pileup_range: tuple | None = None   # (lo, hi): PU_e ~ Poisson(U(lo, hi)), tracks = 20 PU_e
    window: float = 1.0
    tracks_per_pu: int = 20
    z0_sigma: float = 5.0
    sigma_u: float = SIGMA_U
    sigma_v: float = SIGMA_V


CONFIGS = {
    1: EventConfig(1, "barrel_toy", 1, 200, "logu", 1.0, 10.0, 0.8),
    2: EventConfig(2, "full", 1, 4000, "pow3", 0.6, 1e9, 2.4, noise_frac=0.05, ineff=0.01),
    3: EventConfig(3, "barrel_toy", 64, 0, "logu", 1.0, 10.0, 0.8, pileup_range=(50, 250)),
    4: EventConfig(4, "barrel_toy", 16, 4000, "logu", 1.0, 10.0, 0.8),
    5: EventConfig(5, "barrel_toy", 16, 6000, "logu", 1.0, 10.0, 0.8, noise_frac=0.10,
                   displaced_frac=0.05, window=1.5),
}


def scorer_training_config(base: EventConfig) -> EventConfig:
    """Events of the learned scorer's training set: the base configuration's
    detector and spectra, pileup Poisson(U(50, 250)) x 20 helices, and cut
    windows widened 1.5x so that the chain keeps hard wrong candidates."""
    return replace(base, pileup_range=(50, 250), window=1.5)


@dataclass
class Event:
    x: np.ndarray            # float32 [n_hits]
    y: np.ndarray
    z: np.ndarray
    module: np.ndarray       # int32
    sensor: np.ndarray       # uint8 (0 lower, 1 upper)
    truth: np.ndarray        # int32 simulated-track id, -1 for noise
    tracks: dict = field(default_factory=dict)   # per-track truth: pt, eta, phi0, q, z0, d0, R

    @property
    def n_hits(self) -> int:
        return int(self.x.shape[0])


def rng_for(cid: int, event: int, purpose: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([cid, event, purpose])))


# ----------------------------------------------------------------------------
# helix model
# ----------------------------------------------------------------------------
class Helices:
    """Vectorised helices.  Transverse arc length s >= 0 from the point of
    closest approach P0 to the beam line; h = -q is the turning sense for a
    field along +z.  P(s) = P0 + R h (sin(phi0 + h s/R) - sin phi0,
    cos phi0 - cos(phi0 + h s/R)),  z(s) = z0 + s cot(theta)."""

    def __init__(self, pt, eta, phi0, q, z0, d0, bfield=B_FIELD):
        self.pt = np.asarray(pt, float)
        self.eta = np.asarray(eta, float)
        self.phi0 = np.asarray(phi0, float)
        self.q = np.asarray(q, float)
        self.z0 = np.asarray(z0, float)
        self.d0 = np.asarray(d0, float)
        self.R = self.pt / (K_B * bfield)
        self.h = -self.q
        self.cot = np.sinh(self.eta)
        self.x0 = -self.d0 * np.sin(self.phi0)
        self.y0 = self.d0 * np.cos(self.phi0)
        self.smax = math.pi * self.R          # outgoing half turn only

    def pos(self, s, idx=None):
        if idx is None:
            idx = slice(None)
        R, h, p0 = self.R[idx], self.h[idx], self.phi0[idx]
        th = p0 + h * s / R
        x = self.x0[idx] + R * h * (np.sin(th) - np.sin(p0))
        y = self.y0[idx] + R * h * (np.cos(p0) - np.cos(th))
        z = self.z0[idx] + s * self.cot[idx]
        return x, y, z

    def direction(self, s, idx=None):
        if idx is None:
            idx = slice(None)
        th = self.phi0[idx] + self.h[idx] * s / self.R[idx]
        return np.cos(th), np.sin(th)

    def s_at_radius(self, r, idx=None):
        """Smallest s in [0, smax] with |P_xy(s)| = r (NaN if never reached).
        |P_xy| grows monotonically on the outgoing half turn, so bisection is exact."""
        if idx is None:
            idx = np.arange(self.pt.shape[0])
        lo = np.zeros(idx.shape[0])
        hi = self.smax[idx].copy()
        xh, yh, _ = self.pos(hi, idx)
        ok = (np.hypot(xh, yh) >= r) & (np.abs(self.d0[idx]) <= r)
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            xm, ym, _ = self.pos(mid, idx)
            out = np.hypot(xm, ym) >= r
            hi = np.where(out, mid, hi)
            lo = np.where(out, lo, mid)
        s = 0.5 * (lo + hi)
        return np.where(ok, s, np.nan)


def _draw_tracks(cfg: EventConfig, rng: np.random.Generator, n: int) -> dict:
    if cfg.spectrum == "logu":
        pt = np.exp(rng.uniform(math.log(cfg.pt_lo), math.log(cfg.pt_hi), n))
    elif cfg.spectrum == "pow3":
        # dN/dpT ~ pT^-3 above pt_lo: inverse CDF pT = pt_lo (1-U)^(-1/2)
        pt = cfg.pt_lo * (1.0 - rng.uniform(0.0, 1.0, n)) ** -0.5
    else:
        raise ValueError(cfg.spectrum)
    eta = rng.uniform(-cfg.eta_max, cfg.eta_max, n)
    phi0 = rng.uniform(0.0, 2.0 * math.pi, n)
    q = np.where(rng.uniform(0.0, 1.0, n) < 0.5, -1.0, 1.0)
    z0 = rng.normal(0.0, cfg.z0_sigma, n)
    disp = rng.uniform(0.0, 1.0, n) < cfg.displaced_frac
    d0 = np.where(disp, rng.uniform(0.0, cfg.d0_max, n) * np.where(
        rng.uniform(0.0, 1.0, n) < 0.5, -1.0, 1.0), 0.0)
    return dict(pt=pt, eta=eta, phi0=phi0, q=q, z0=z0, d0=d0)


def _barrel_hits(geo: G.Geometry, hel: Helices, layer: int):
    """Exact helix crossings with both sensor planes of the barrel modules of one layer."""
    m = geo.meta[layer]
    n = hel.pt.shape[0]
    s_cyl = hel.s_at_radius(m["r"])
    tr_all = np.nonzero(np.isfinite(s_cyl))[0]
    if tr_all.size == 0:
        return []
    xc, yc, zc = hel.pos(s_cyl[tr_all], tr_all)
    dphi = 2.0 * math.pi / m["nphi"]
    k0 = np.rint((np.arctan2(yc, xc) - m["off"]) / dphi).astype(np.int64)
    j0 = np.floor(zc / (2.0 * m["hv"]) + m["nrow"] / 2).astype(np.int64)
    out = []
    f64 = geo.f64
    for dk in (-1, 0, 1):
        for dj in (-1, 0, 1):
            k = np.mod(k0 + dk, m["nphi"])
            j = j0 + dj
            sel = (j >= 0) & (j < m["nrow"])
            tr = tr_all[sel]
            mod = m["base"] + k[sel] * m["nrow"] + j[sel]
            wx, wy = f64[G.F_WX, mod], f64[G.F_WY, mod]
            ux, uy = f64[G.F_UX, mod], f64[G.F_UY, mod]
            cx, cy, czm = f64[G.F_CX, mod], f64[G.F_CY, mod], f64[G.F_CZ, mod]
            for sensor in (0, 1):
                d = m["r"] + (sensor - 0.5) * m["g"]
                s = s_cyl[tr].copy()
                for _ in range(8):
                    x, y, _ = hel.pos(s, tr)
                    tx, ty = hel.direction(s, tr)
                    f = x * wx + y * wy - d
                    fp = tx * wx + ty * wy
                    s = s - f / np.where(np.abs(fp) > 1e-12, fp, 1e-12)
                x, y, z = hel.pos(s, tr)
                f = x * wx + y * wy - d
                lu = (x - cx) * ux + (y - cy) * uy
                lv = z - czm
                ok = ((np.abs(f) < 1e-7) & (s >= 0.0) & (s <= hel.smax[tr]) &
                      (np.abs(lu) <= m["hu"]) & (np.abs(lv) <= m["hv"]))
                if np.any(ok):
                    out.append((tr[ok], mod[ok], np.full(ok.sum(), sensor), x[ok], y[ok], z[ok]))
    return out


def _disk_hits(geo: G.Geometry, hel: Helices, layer: int):
    m = geo.meta[layer]
    side = m["side"]
    zmid = side * m["z"]
    with np.errstate(divide="ignore", invalid="ignore"):
        s_mid = (zmid - hel.z0) / hel.cot
    tr_all = np.nonzero((s_mid > 0) & (s_mid <= hel.smax))[0]
    if tr_all.size == 0:
        return []
    x, y, _ = hel.pos(s_mid[tr_all], tr_all)
    r = np.hypot(x, y)
    ph = np.arctan2(y, x)
    f64 = geo.f64
    out = []
    for ring in m["rings"]:
        near = (r > ring["r_in"] - 2.0) & (r < ring["r_out"] + 6.0)
        if not np.any(near):
            continue
        trn = tr_all[near]
        dphi = 2.0 * math.pi / ring["nphi"]
        k0 = np.rint((ph[near] - ring["off"]) / dphi).astype(np.int64)
        for dk in (-1, 0, 1):
            k = np.mod(k0 + dk, ring["nphi"])
            mod = ring["base"] + k
            for sensor in (0, 1):
                zs = zmid + side * (sensor - 0.5) * ring["g"]
                s = (zs - hel.z0[trn]) / hel.cot[trn]
                xs, ys, zz = hel.pos(s, trn)
                lu = (xs - f64[G.F_CX, mod]) * f64[G.F_UX, mod] + (ys - f64[G.F_CY, mod]) * f64[G.F_UY, mod]
                lv = (xs - f64[G.F_CX, mod]) * f64[G.F_VX, mod] + (ys - f64[G.F_CY, mod]) * f64[G.F_VY, mod]
                ok = ((s > 0) & (s <= hel.smax[trn]) & (np.abs(lu) <= ring["hu"]) &
                      (np.abs(lv) <= ring["hv"]))
                if np.any(ok):
                    out.append((trn[ok], mod[ok], np.full(ok.sum(), sensor), xs[ok], ys[ok], zz[ok]))
    return out


def simulate(geo: G.Geometry, hel: Helices, rng: np.random.Generator | None,
             sigma_u=SIGMA_U, sigma_v=SIGMA_V, ineff=0.0, noise_frac=0.0, shuffle=True):
    """Hits of the helices in geometry ``geo``.  With ``rng=None`` nothing is
    smeared, dropped, added or shuffled (exact crossings, in generation order)."""
    parts = []
    layers = sorted(geo.meta.keys())
    for layer in layers:
        if geo.meta[layer]["kind"] == "barrel":
            parts += _barrel_hits(geo, hel, layer)
        else:
            parts += _disk_hits(geo, hel, layer)
    if parts:
        tr = np.concatenate([p[0] for p in parts])
        mod = np.concatenate([p[1] for p in parts])
        sen = np.concatenate([p[2] for p in parts])
        x = np.concatenate([p[3] for p in parts])
        y = np.concatenate([p[4] for p in parts])
        z = np.concatenate([p[5] for p in parts])
    else:
        tr = np.zeros(0, np.int64); mod = np.zeros(0, np.int64); sen = np.zeros(0, np.int64)
        x = y = z = np.zeros(0)
    f64 = geo.f64
    if rng is not None:
        du = rng.normal(0.0, sigma_u, x.shape[0])
        dv = rng.normal(0.0, sigma_v, x.shape[0])
        x = x + du * f64[G.F_UX, mod] + dv * f64[G.F_VX, mod]
        y = y + du * f64[G.F_UY, mod] + dv * f64[G.F_VY, mod]
        z = z + du * f64[G.F_UZ, mod] + dv * f64[G.F_VZ, mod]
        if ineff > 0.0:
            keep = rng.uniform(0.0, 1.0, x.shape[0]) >= ineff
            tr, mod, sen, x, y, z = tr[keep], mod[keep], sen[keep], x[keep], y[keep], z[keep]
        n_noise = int(round(noise_frac * x.shape[0]))
        if n_noise > 0:
            area = 4.0 * f64[G.F_HU] * f64[G.F_HV]
            nm = rng.choice(geo.n_mod, size=n_noise, p=area / area.sum())
            ns = rng.integers(0, 2, n_noise)
            lu = rng.uniform(-1.0, 1.0, n_noise) * f64[G.F_HU, nm]
            lv = rng.uniform(-1.0, 1.0, n_noise) * f64[G.F_HV, nm]
            off = (ns - 0.5) * f64[G.F_GAP, nm]
            nx = f64[G.F_CX, nm] + off * f64[G.F_WX, nm] + lu * f64[G.F_UX, nm] + lv * f64[G.F_VX, nm]
            ny = f64[G.F_CY, nm] + off * f64[G.F_WY, nm] + lu * f64[G.F_UY, nm] + lv * f64[G.F_VY, nm]
            nz = f64[G.F_CZ, nm] + off * f64[G.F_WZ, nm] + lu * f64[G.F_UZ, nm] + lv * f64[G.F_VZ, nm]
            tr = np.concatenate([tr, np.full(n_noise, -1)])
            mod = np.concatenate([mod, nm]); sen = np.concatenate([sen, ns])
            x = np.concatenate([x, nx]); y = np.concatenate([y, ny]); z = np.concatenate([z, nz])
        if shuffle:
            perm = rng.permutation(x.shape[0])
            tr, mod, sen, x, y, z = tr[perm], mod[perm], sen[perm], x[perm], y[perm], z[perm]
    return Event(x=x.astype(np.float32), y=y.astype(np.float32), z=z.astype(np.float32),
                 module=mod.astype(np.int32), sensor=sen.astype(np.uint8),
                 truth=tr.astype(np.int32))


def n_tracks_for(cfg: EventConfig, rng: np.random.Generator) -> int:
    if cfg.pileup_range is not None:
        lam = rng.uniform(*cfg.pileup_range)
        return cfg.tracks_per_pu * int(rng.poisson(lam))
    return cfg.n_tracks


def generate(cid: int, event: int = 0, purpose: int = PURPOSE_EVAL,
             n_tracks: int | None = None, cfg: EventConfig | None = None) -> Event:
    cfg = cfg or CONFIGS[cid]
    rng = rng_for(cfg.cid, event, purpose)
    n = n_tracks if n_tracks is not None else n_tracks_for(cfg, rng)
    trk = _draw_tracks(cfg, rng, n)
    hel = Helices(**trk)
    ev = simulate(G.get(cfg.geometry), hel, rng, sigma_u=cfg.sigma_u, sigma_v=cfg.sigma_v,
                  ineff=cfg.ineff, noise_frac=cfg.noise_frac)
    trk["R"] = hel.R
    ev.tracks = trk
    return ev


@dataclass
class Batch:
    events: list
    offsets: np.ndarray      # int32 [n_events + 1]
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    module: np.ndarray
    sensor: np.ndarray


def concat(events) -> Batch:
    offs = np.zeros(len(events) + 1, np.int32)
    offs[1:] = np.cumsum([e.n_hits for e in events])
    cat = lambda a: np.ascontiguousarray(np.concatenate([getattr(e, a) for e in events]))
    return Batch(events=list(events), offsets=offs, x=cat("x"), y=cat("y"), z=cat("z"),
                 module=cat("module"), sensor=cat("sensor"))


def generate_batch(cid: int, n_events: int | None = None, purpose: int = PURPOSE_EVAL,
                   first_event: int = 0) -> Batch:
    cfg = CONFIGS[cid]
    n = cfg.n_events if n_events is None else n_events
    return concat([generate(cid, first_event + e, purpose) for e in range(n)])


# ----------------------------------------------------------------------------
# pixel detector and pixel seeds (input of the pixel line segments, Sec. 2.1)
# ----------------------------------------------------------------------------
PURPOSE_PIXEL = 3
PIXEL_RADII = (3.0, 6.8, 10.9, 16.0)   # cm, four idealised barrel cylinders
SIGMA_PIX_RPHI = 0.0010                # cm (10 um)
SIGMA_PIX_Z = 0.0020                   # cm (20 um)
PIXEL_SEED_PT = 0.8                    # GeV: seeds of simulated tracks above it
PIXEL_FAKE_FRAC = 0.05                 # fake seeds per real seed


@dataclass
class PixelSeeds:
    """Pixel hits of one event and its seeds (four hit indices each, inner to
    outer).  Stand-in for the pixel tracking that feeds the method: every
    simulated track above PIXEL_SEED_PT crossing all four layers (each hit
    kept with probability 1 - ineff) gives a seed, and PIXEL_FAKE_FRAC fake
    seeds join the two inner hits of one track to the two outer hits of
    another track close to it in azimuth."""
    x: np.ndarray            # float32 [n_px]
    y: np.ndarray
    z: np.ndarray
    truth: np.ndarray        # int32 track id of each pixel hit
    seeds: np.ndarray        # int32 [n_seeds, 4] pixel hit indices

    @property
    def n_hits(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_seeds(self) -> int:
        return int(self.seeds.shape[0])


def pixel_seeds(ev: Event, cid: int, event: int, cfg: EventConfig | None = None) -> PixelSeeds:
    """Pixel hits and seeds of event `event` of configuration `cid` (its own
    random stream: the outer-tracker hits of the event are unchanged)."""
    cfg = cfg or CONFIGS[cid]
    rng = rng_for(cfg.cid, event, PURPOSE_PIXEL)
    trk = ev.tracks
    hel = Helices(trk["pt"], trk["eta"], trk["phi0"], trk["q"], trk["z0"], trk["d0"])
    n = hel.pt.shape[0]
    pos = np.full((n, 4, 3), np.nan)
    for j, r in enumerate(PIXEL_RADII):
        s = hel.s_at_radius(r)
        ok = np.isfinite(s)
        x, y, z = hel.pos(np.where(ok, s, 0.0))
        # smearing along the azimuthal direction and along z
        d = rng.normal(0.0, SIGMA_PIX_RPHI, n)
        dz = rng.normal(0.0, SIGMA_PIX_Z, n)
        rr = np.maximum(np.hypot(x, y), 1e-9)
        x, y, z = x - d * y / rr, y + d * x / rr, z + dz
        hit = ok & (rng.uniform(0.0, 1.0, n) >= cfg.ineff)
        pos[hit, j] = np.stack([x[hit], y[hit], z[hit]], axis=1)
    has = np.all(np.isfinite(pos[:, :, 0]), axis=1)
    # every pixel hit, track-major, then shuffled
    tr_of, lay_of = np.nonzero(np.isfinite(pos[:, :, 0]))
    px = pos[tr_of, lay_of]
    perm = rng.permutation(tr_of.shape[0])
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.shape[0])
    index = np.full((n, 4), -1, np.int64)
    index[tr_of, lay_of] = inv
    real = np.nonzero(has & (hel.pt >= PIXEL_SEED_PT))[0]
    seeds = [index[t] for t in real]
    n_fake = int(round(PIXEL_FAKE_FRAC * real.shape[0]))
    if n_fake and real.shape[0] > 1:
        phi = np.arctan2(pos[real, 3, 1], pos[real, 3, 0])
        order = np.argsort(phi)
        for _ in range(n_fake):
            i = int(rng.integers(0, real.shape[0]))
            k = int(np.searchsorted(phi[order], phi[i]))
            j = order[(k + int(rng.choice([-2, -1, 1, 2]))) % real.shape[0]]
            a, b = real[i], real[j]
            if a != b:
                seeds.append(np.r_[index[a, :2], index[b, 2:]])
    seeds = np.array(seeds, np.int64).reshape(-1, 4)
    seeds = seeds[rng.permutation(seeds.shape[0])]
    return PixelSeeds(x=px[perm, 0].astype(np.float32), y=px[perm, 1].astype(np.float32),
                      z=px[perm, 2].astype(np.float32), truth=tr_of[perm].astype(np.int32),
                      seeds=seeds.astype(np.int32))
