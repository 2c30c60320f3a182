"""Synthetic outer-tracker geometry made of p_T modules.

This module describes the detector only: where each two-sensor module sits,
its local frame and its extent.  It contains none of the Segment Linking
arithmetic (no windows, no cuts, no compatibility map); both the HIP library
and the CPU oracle receive the arrays built here as plain inputs.

Detector model (Sec. 2 of the paper): every layer (barrel) or disk (endcap) is
tiled by p_T modules, each a pair of closely spaced parallel sensors.  The
paper's CMS Phase-2 layout is not available, so two stand-ins are built:

* ``barrel_toy`` -- six cylindrical layers at r = 23, 36, 51, 68, 86, 110 cm,
  flat 10 x 5 cm modules with a 1.8 mm sensor gap, half a phi pitch offset on
  odd layers, rows of 5 cm covering |z| <= r sinh(0.8) + 15 cm.
* ``full`` -- the same radii with |z| <= 120 cm, PS modules (10 x 5 cm, 2.6 mm
  gap) below r = 60 cm and 2S modules (10 x 10 cm, 4 mm gap) above, plus five
  endcap disks per side at |z| = 131, 156, 185, 220, 262 cm tiled by rings from
  r = 23 cm outwards (5 cm radial rings while the inner radius is below 60 cm,
  10 cm above).

Local frame of a module: ``u`` is the precise (tangential) axis, ``v`` the
coarse axis (+z in the barrel, radially outwards in the endcap) and ``w`` the
sensor normal pointing away from the interaction point.  The centre is the
mid-plane between the sensors; sensor 0 (lower) sits at centre - g/2 w and
sensor 1 (upper) at centre + g/2 w.

Logical layers: barrel 1..6, +z disks 7..11, -z disks 12..16.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Field layout of the float32 module table (SoA, shape [N_F32, n_mod]).
F_CX, F_CY, F_CZ = 0, 1, 2
F_UX, F_UY, F_UZ = 3, 4, 5
F_VX, F_VY, F_VZ = 6, 7, 8
F_WX, F_WY, F_WZ = 9, 10, 11
F_HU, F_HV, F_GAP = 12, 13, 14
F_RMIN, F_RMAX, F_ZMIN, F_ZMAX = 15, 16, 17, 18
F_PHI, F_DPHI = 19, 20
N_F32 = 21

# Field layout of the int32 module table (SoA, shape [N_I32, n_mod]).
I_LAYER, I_SUBDET, I_SIDE, I_TYPE = 0, 1, 2, 3
N_I32 = 4

SUBDET_BARREL, SUBDET_ENDCAP = 0, 1
TYPE_PS, TYPE_2S = 0, 1

BARREL_RADII = (23.0, 36.0, 51.0, 68.0, 86.0, 110.0)
DISK_Z = (131.0, 156.0, 185.0, 220.0, 262.0)
N_LAYERS = 16


@dataclass
class Geometry:
    name: str
    f32: np.ndarray          # [N_F32, n_mod] float32
    i32: np.ndarray          # [N_I32, n_mod] int32
    f64: np.ndarray          # [N_F32, n_mod] float64 (exact placement, generator use only)
    meta: dict               # per-layer tiling description (generator use only)

    @property
    def n_mod(self) -> int:
        return int(self.f32.shape[1])

    def layer_modules(self, layer: int) -> np.ndarray:
        return np.nonzero(self.i32[I_LAYER] == layer)[0]


class _Builder:
    def __init__(self):
        self.rows_f = []
        self.rows_i = []

    def add(self, c, u, v, w, hu, hv, g, rmin, rmax, zmin, zmax, phi, dphi,
            layer, subdet, side, mtype):
        row = np.zeros(N_F32)
        row[F_CX:F_CZ + 1] = c
        row[F_UX:F_UZ + 1] = u
        row[F_VX:F_VZ + 1] = v
        row[F_WX:F_WZ + 1] = w
        row[F_HU], row[F_HV], row[F_GAP] = hu, hv, g
        row[F_RMIN], row[F_RMAX], row[F_ZMIN], row[F_ZMAX] = rmin, rmax, zmin, zmax
        row[F_PHI], row[F_DPHI] = phi, dphi
        self.rows_f.append(row)
        self.rows_i.append((layer, subdet, side, mtype))

        return len(self.rows_f) - 1

    def finish(self, name, meta):
        f64 = np.ascontiguousarray(np.array(self.rows_f).T)
        i32 = np.ascontiguousarray(np.array(self.rows_i, dtype=np.int32).T)
        return Geometry(name=name, f32=f64.astype(np.float32), i32=i32, f64=f64, meta=meta)


def _wrap(phi):
    return (phi + math.pi) % (2.0 * math.pi) - math.pi


def n_phi_barrel(r: float, hu: float = 5.0) -> int:
    """Number of flat modules of half-width hu needed to close a ring of apothem r."""
    return int(math.ceil(math.pi / math.atan(hu / r)))


def _barrel_layer(b: _Builder, li: int, r: float, hu: float, hv: float, g: float,
                  zhalf: float, mtype: int):
    nphi = n_phi_barrel(r, hu)
    nrow = 2 * int(math.ceil(zhalf / (2.0 * hv)))
    off = (math.pi / nphi) if (li % 2 == 1) else 0.0
    base = len(b.rows_f)
    for k in range(nphi):
        phi = _wrap(2.0 * math.pi * k / nphi + off)
        w = np.array([math.cos(phi), math.sin(phi), 0.0])
        u = np.array([-math.sin(phi), math.cos(phi), 0.0])
        v = np.array([0.0, 0.0, 1.0])
        for j in range(nrow):
            zc = (j - nrow / 2 + 0.5) * (2.0 * hv)
            c = r * w + zc * v
            b.add(c, u, v, w, hu, hv, g,
                  rmin=r, rmax=math.hypot(r, hu), zmin=zc - hv, zmax=zc + hv,
                  phi=phi, dphi=math.atan(hu / r),
                  layer=li, subdet=SUBDET_BARREL, side=0, mtype=mtype)
    return dict(kind="barrel", base=base, nphi=nphi, nrow=nrow, off=off, r=r,
                hu=hu, hv=hv, g=g)


def _disk_rings(r_lo=23.0, r_hi=110.0):
    rings = []
    r = r_lo
    while r < r_hi:
        length = 5.0 if r < 60.0 else 10.0
        rings.append((r, r + length))
        r += length
    return rings


def n_phi_ring(r_out: float, hu: float = 5.0) -> int:
    return int(math.ceil(math.pi / math.asin(hu / r_out)))


def _disk(b: _Builder, layer: int, zd: float, side: int):
    rings = []
    for (r_in, r_out) in _disk_rings():
        ps = r_in < 60.0
        g = 0.26 if ps else 0.40
        hu = 5.0
        hv = 0.5 * (r_out - r_in)
        rc = 0.5 * (r_in + r_out)
        nphi = n_phi_ring(r_out, hu)
        off = (math.pi / nphi) if (layer % 2 == 1) else 0.0
        rings.append(dict(base=len(b.rows_f), nphi=nphi, off=off, r_in=r_in,
                          r_out=r_out, hu=hu, hv=hv, g=g))
        for k in range(nphi):
            phi = _wrap(2.0 * math.pi * k / nphi + off)
            v = np.array([math.cos(phi), math.sin(phi), 0.0])
            u = np.array([-math.sin(phi), math.cos(phi), 0.0])
            w = np.array([0.0, 0.0, float(side)])
            c = rc * v + np.array([0.0, 0.0, side * zd])
            b.add(c, u, v, w, hu, hv, g,
                  rmin=r_in, rmax=math.hypot(r_out, hu),
                  zmin=side * zd, zmax=side * zd,
                  phi=phi, dphi=math.atan(hu / r_in),
                  layer=layer, subdet=SUBDET_ENDCAP, side=side,
                  mtype=TYPE_PS if ps else TYPE_2S)
    return dict(kind="disk", z=zd, side=side, rings=rings)


def barrel_toy() -> Geometry:
    """Six-layer barrel-only toy: 10 x 5 cm modules, 1.8 mm gap."""
    b = _Builder()
    meta = {}
    for li, r in enumerate(BARREL_RADII, start=1):
        zhalf = r * math.sinh(0.8) + 15.0
        meta[li] = _barrel_layer(b, li, r, hu=5.0, hv=2.5, g=0.18, zhalf=zhalf,
                                 mtype=TYPE_PS)
    return b.finish("barrel_toy", meta)


def full() -> Geometry:
    """Barrel (|z| <= 120 cm, PS below r = 60 cm, 2S above) plus 5 disks per side."""
    b = _Builder()
    meta = {}
    for li, r in enumerate(BARREL_RADII, start=1):
        if r < 60.0:
            meta[li] = _barrel_layer(b, li, r, hu=5.0, hv=2.5, g=0.26, zhalf=120.0,
                                     mtype=TYPE_PS)
        else:
            meta[li] = _barrel_layer(b, li, r, hu=5.0, hv=5.0, g=0.40, zhalf=120.0,
                                     mtype=TYPE_2S)
    for di, zd in enumerate(DISK_Z):
        meta[7 + di] = _disk(b, 7 + di, zd, +1)
    for di, zd in enumerate(DISK_Z):
        meta[12 + di] = _disk(b, 12 + di, zd, -1)
    return b.finish("full", meta)


_CACHE = {}


def get(name: str) -> Geometry:
    if name not in _CACHE:
        _CACHE[name] = {"barrel_toy": barrel_toy, "full": full}[name]()
    return _CACHE[name]
