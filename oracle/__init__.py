"""CPU oracle of the Segment Linking hot path -- TEST INFRASTRUCTURE.

Plain, slow C (``lst_oracle.c`` + ``cuts.inc``) loaded through ctypes.  Only the
test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the HIP library never does, and the two
share no code.  Inputs are the synthetic geometry, hits and the primary
parameter vector; every derived constant, the module map and every cut value
is computed here independently.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, f) for f in ("lst_oracle.c", "cuts.inc", "lst_oracle.h")]

# primary parameter vector (same order as ORC_P_* in lst_oracle.h)
PARAM_NAMES = ("bfield", "ptmin", "z0max", "sigu", "sigv", "nsig", "epsk", "epsa", "d0max",
               "xrphi", "xrz", "w", "map_dphi", "map_dl")
N_PARAMS = len(PARAM_NAMES)
MD, SEG, T3, T5, T5_KEPT = 0, 1, 2, 3, 4
WIDTH = {MD: 2, SEG: 4, T3: 6, T5: 10, T5_KEPT: 10}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (FP32 strict: no contraction, no fast-math)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", _SO, os.path.join(_HERE, "lst_oracle.c"), "-lm"]
        subprocess.run(cmd, check=True)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    P = ctypes.c_void_p
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P]
    lib.orc_destroy.argtypes = [P]
    lib.orc_map_edges.restype = ctypes.c_int64
    lib.orc_map_edges.argtypes = [P]
    lib.orc_map.argtypes = [P, P, P]
    lib.orc_run.restype = ctypes.c_int
    lib.orc_run.argtypes = [P, ctypes.c_int32, P, P, P, P, P]
    lib.orc_count.restype = ctypes.c_int64
    lib.orc_count.argtypes = [P, ctypes.c_int]
    lib.orc_tuples.argtypes = [P, ctypes.c_int, P]
    lib.orc_cands.argtypes = [P, P]
    lib.orc_t5_scores.argtypes = [P, P]
    lib.orc_t5_keep.argtypes = [P, P]
    lib.orc_t3_curv.argtypes = [P, P]
    lib.orc_t5_features.argtypes = [P, P]
    lib.orc_t3_features.argtypes = [P, P]
    lib.orc_rerun_t5.restype = ctypes.c_int
    lib.orc_rerun_t5.argtypes = [P, P]
    for f in ("orc_eval_t3_features", "orc_eval_t5_features"):
        getattr(lib, f).restype = ctypes.c_int
        getattr(lib, f).argtypes = [P, P, P, P]
    lib.orc_near_count.restype = ctypes.c_int64
    lib.orc_near_count.argtypes = [P, ctypes.c_int]
    lib.orc_near.argtypes = [P, ctypes.c_int, P, P, P]
    for f in ("orc_eval_md",):
        getattr(lib, f).restype = ctypes.c_int
        getattr(lib, f).argtypes = [P, ctypes.c_int, P, P, P]
    for f in ("orc_eval_seg", "orc_eval_t3", "orc_eval_t5"):
        getattr(lib, f).restype = ctypes.c_int
        getattr(lib, f).argtypes = [P, P, P, P]
    lib.orc_consts.argtypes = [P, P]
    lib.orc_run_pixel.restype = ctypes.c_int
    lib.orc_run_pixel.argtypes = [P, P, ctypes.c_int, ctypes.c_int32, P, P, P, ctypes.c_int32, P]
    lib.orc_px_count.restype = ctypes.c_int64
    lib.orc_px_count.argtypes = [P, ctypes.c_int]
    lib.orc_px_candidates.argtypes = [P, ctypes.c_int, P]
    lib.orc_tc.argtypes = [P, P]
    lib.orc_eval_link.restype = ctypes.c_int
    lib.orc_eval_link.argtypes = [P, P, P, ctypes.c_int, P, P, P]
    lib.orc_set_hit_storage.argtypes = [P, ctypes.c_int]
    lib.orc_set_margins.argtypes = [P, ctypes.c_int]
    lib.orc_f32_to_f16.restype = ctypes.c_uint16
    lib.orc_f32_to_f16.argtypes = [ctypes.c_float]
    lib.orc_f16_to_f32.restype = ctypes.c_float
    lib.orc_f16_to_f32.argtypes = [ctypes.c_uint16]
    lib.orc_set_truncation.restype = ctypes.c_int
    lib.orc_set_truncation.argtypes = [P, P]
    lib.orc_dropped.argtypes = [P, P]
    lib.orc_eval_margin.restype = ctypes.c_double
    lib.orc_eval_margin.argtypes = [P, ctypes.c_int, P, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Result:
    tuples: dict            # kind -> int32 [n, width]
    t5_scores: np.ndarray
    t5_keep: np.ndarray
    t3_curv: np.ndarray
    t5_features: np.ndarray  # float32 [n_t5, 40]
    t3_features: np.ndarray  # float32 [n_t3, 40]
    cands: np.ndarray       # int64 [4]
    near: dict              # kind -> (tuples, margins, decisions)


def f32_to_f16_bits(values) -> np.ndarray:
    """the oracle's binary32 -> binary16 conversion (nearest even), as bits"""
    lib = _load()
    return np.array([lib.orc_f32_to_f16(float(v)) for v in np.asarray(values, np.float32)],
                    np.uint16)


def f16_bits_to_f32(bits) -> np.ndarray:
    lib = _load()
    return np.array([lib.orc_f16_to_f32(int(b)) for b in np.asarray(bits, np.uint16)],
                    np.float32)


@dataclass
class PixelResult:
    pt5: np.ndarray         # int32 [n, 13]: seed, 10 hits, score bits, kept
    pt3: np.ndarray         # int32 [n, 13]: seed, 6 hits + 4 x -1, score bits, kept
    tc: np.ndarray          # int32 [n, 12]: type, seed, 10 hits (-1 padded)
    near: int               # pixel decisions within 1e-5 (relative) of a threshold


TC_PT5, TC_PT3, TC_T5, TC_PLS = 0, 1, 2, 3


class Oracle:
    """One geometry + parameter set; ``run(event)`` evaluates one event."""

    def __init__(self, params: np.ndarray, geo_f32: np.ndarray, geo_i32: np.ndarray):
        lib = _load()
        self._params = np.ascontiguousarray(params, dtype=np.float64)
        self._f32 = np.ascontiguousarray(geo_f32, dtype=np.float32)
        self._i32 = np.ascontiguousarray(geo_i32, dtype=np.int32)
        self.n_mod = int(self._f32.shape[1])
        h = lib.orc_create(_ptr(self._params), len(self._params), self.n_mod,
                           _ptr(self._f32), _ptr(self._i32))
        if not h:
            raise ValueError("oracle: bad geometry or parameters")
        self._h = ctypes.c_void_p(h)
        self._lib = lib

    def __del__(self):
        if getattr(self, "_h", None) is not None and self._lib is not None:
            self._lib.orc_destroy(self._h)
            self._h = None

    def module_map(self):
        n_e = self._lib.orc_map_edges(self._h)
        ptr = np.zeros(self.n_mod + 1, np.int32)
        col = np.zeros(max(n_e, 1), np.int32)
        self._lib.orc_map(self._h, _ptr(ptr), _ptr(col))
        return ptr, col[:n_e]

    def consts(self):
        out = np.zeros(7, np.float32)
        self._lib.orc_consts(self._h, _ptr(out))
        return dict(zip(("kmax", "klim", "kh", "tolu", "tolv", "tolkc", "epsak"), out))

    def set_hit_storage(self, fp16: bool):
        """hits stored as module-local FP16 (u, v) for later events"""
        self._lib.orc_set_hit_storage(self._h, int(bool(fp16)))

    def set_margins(self, on: bool):
        """FP64 margins on (default) or off (FP32 decisions only, no
        near-threshold records; objects unchanged)"""
        self._lib.orc_set_margins(self._h, int(bool(on)))

    def set_truncation(self, caps=None):
        """per-module capacities (MD, SEG, T3, T5; 0 = none) for later events"""
        if caps is None:
            rc = self._lib.orc_set_truncation(self._h, None)
        else:
            c = np.ascontiguousarray(caps, np.int32)
            assert c.shape == (4,)
            rc = self._lib.orc_set_truncation(self._h, _ptr(c))
        if rc != 0:
            raise ValueError("oracle: negative capacity")

    def dropped(self) -> np.ndarray:
        """objects removed by the capacities in the last event, per kind"""
        out = np.zeros(4, np.int64)
        self._lib.orc_dropped(self._h, _ptr(out))
        return out

    def run_pixel(self, pix_params, px):
        """Pixel objects and track candidates of the last event (run / run_event
        first): px has x, y, z (pixel hits) and seeds [n, 4].  Returns a
        PixelResult."""
        pp = np.ascontiguousarray(pix_params, np.float64)
        x = np.ascontiguousarray(px.x, np.float32); y = np.ascontiguousarray(px.y, np.float32)
        z = np.ascontiguousarray(px.z, np.float32)
        sd = np.ascontiguousarray(px.seeds, np.int32).reshape(-1, 4)
        rc = self._lib.orc_run_pixel(self._h, _ptr(pp), len(pp), int(x.shape[0]), _ptr(x),
                                     _ptr(y), _ptr(z), int(sd.shape[0]), _ptr(sd))
        if rc != 0:
            raise ValueError("oracle: bad pixel input or no event")
        lib, h = self._lib, self._h
        cand = {}
        for what in (0, 2):
            n = lib.orc_px_count(h, what)
            out = np.zeros((max(n, 1), 13), np.int32)
            lib.orc_px_candidates(h, what, _ptr(out))
            cand[what] = out[:n]
        n = lib.orc_px_count(h, 4)
        tc = np.zeros((max(n, 1), 12), np.int32)
        lib.orc_tc(h, _ptr(tc))
        return PixelResult(pt5=cand[0], pt3=cand[2], tc=tc[:n], near=int(lib.orc_px_count(h, 5)))

    def run(self, x, y, z, module, sensor) -> Result:
        x = np.ascontiguousarray(x, np.float32); y = np.ascontiguousarray(y, np.float32)
        z = np.ascontiguousarray(z, np.float32)
        module = np.ascontiguousarray(module, np.int32)
        sensor = np.ascontiguousarray(sensor, np.uint8)
        rc = self._lib.orc_run(self._h, int(x.shape[0]), _ptr(x), _ptr(y), _ptr(z),
                               _ptr(module), _ptr(sensor))
        if rc != 0:
            raise ValueError("oracle: invalid hits")
        return self._collect()

    def run_event(self, ev) -> Result:
        return self.run(ev.x, ev.y, ev.z, ev.module, ev.sensor)

    def rerun_t5(self, t3_veto=None) -> Result:
        """Quintuplets and duplicate removal again on the last event's
        triplets, those with t3_veto set (order of the T3 tuples) left out."""
        if t3_veto is None:
            rc = self._lib.orc_rerun_t5(self._h, None)
        else:
            v = np.ascontiguousarray(t3_veto, np.uint8)
            assert v.shape[0] == self._lib.orc_count(self._h, T3)
            rc = self._lib.orc_rerun_t5(self._h, _ptr(v))
        if rc != 0:
            raise ValueError("oracle: no event to rerun")
        return self._collect()

    def _collect(self) -> Result:
        lib, h = self._lib, self._h
        tuples = {}
        for kind in (MD, SEG, T3, T5, T5_KEPT):
            n = lib.orc_count(h, kind)
            out = np.zeros((max(n, 1), WIDTH[kind]), np.int32)
            lib.orc_tuples(h, kind, _ptr(out))
            tuples[kind] = out[:n]
        n5 = lib.orc_count(h, T5)
        sc = np.zeros(max(n5, 1), np.float32); lib.orc_t5_scores(h, _ptr(sc))
        kp = np.zeros(max(n5, 1), np.uint8); lib.orc_t5_keep(h, _ptr(kp))
        n3 = lib.orc_count(h, T3)
        k3 = np.zeros(max(n3, 1), np.float32); lib.orc_t3_curv(h, _ptr(k3))
        cands = np.zeros(4, np.int64); lib.orc_cands(h, _ptr(cands))
        ft = np.zeros((max(n5, 1), 40), np.float32); lib.orc_t5_features(h, _ptr(ft))
        f3 = np.zeros((max(n3, 1), 40), np.float32); lib.orc_t3_features(h, _ptr(f3))
        near = {}
        for kind in (MD, SEG, T3, T5):
            nn = lib.orc_near_count(h, kind)
            tt = np.zeros((max(nn, 1), WIDTH[kind]), np.int32)
            mg = np.zeros(max(nn, 1), np.float64)
            dc = np.zeros(max(nn, 1), np.uint8)
            lib.orc_near(h, kind, _ptr(tt), _ptr(mg), _ptr(dc))
            near[kind] = (tt[:nn], mg[:nn], dc[:nn])
        return Result(tuples=tuples, t5_scores=sc[:n5], t5_keep=kp[:n5].astype(bool),
                      t3_curv=k3[:n3], t5_features=ft[:n5], t3_features=f3[:n3], cands=cands,
                      near=near)

    # -- single-candidate evaluation (closed-form checks) -------------------
    def eval_md(self, module: int, lo3, up3):
        lo = np.ascontiguousarray(lo3, np.float32); up = np.ascontiguousarray(up3, np.float32)
        out = np.zeros(8)
        p = self._lib.orc_eval_md(self._h, int(module), _ptr(lo), _ptr(up), _ptr(out))
        return bool(p), out

    def _eval(self, fn, n, mods, hits, nout):
        mods = np.ascontiguousarray(mods, np.int32)
        hits = np.ascontiguousarray(hits, np.float32).reshape(-1)
        assert mods.shape[0] == n and hits.shape[0] == 6 * n
        out = np.zeros(nout)
        p = fn(self._h, _ptr(mods), _ptr(hits), _ptr(out))
        return bool(p), out

    def eval_seg(self, mods, hits):
        return self._eval(self._lib.orc_eval_seg, 2, mods, hits, 13)

    def eval_t3(self, mods, hits):
        return self._eval(self._lib.orc_eval_t3, 3, mods, hits, 7)

    def eval_t5(self, mods, hits):
        return self._eval(self._lib.orc_eval_t5, 5, mods, hits, 18)

    def _eval_f(self, fn, n, mods, hits):
        mods = np.ascontiguousarray(mods, np.int32)
        hits = np.ascontiguousarray(hits, np.float32).reshape(-1)
        assert mods.shape[0] == n and hits.shape[0] == 6 * n
        out = np.zeros(40, np.float32)
        p = fn(self._h, _ptr(mods), _ptr(hits), _ptr(out))
        return bool(p), out

    def eval_t3_features(self, mods, hits):
        return self._eval_f(self._lib.orc_eval_t3_features, 3, mods, hits)

    def eval_t5_features(self, mods, hits):
        return self._eval_f(self._lib.orc_eval_t5_features, 5, mods, hits)

    def eval_link(self, pix_params, pix12, mods, hits):
        """one pixel link: four pixel hits (12 floats) with a quintuplet (5 MDs)
        or a triplet (3 MDs); returns (decision, out[12]): pLS tx, ty, cot,
        object tx, ty, cot, window cos-term, sin^2, polar term, chi2_rphi,
        chi2_rz, score"""
        pp = np.ascontiguousarray(pix_params, np.float64)
        p12 = np.ascontiguousarray(pix12, np.float32).reshape(-1)
        mods = np.ascontiguousarray(mods, np.int32)
        hits = np.ascontiguousarray(hits, np.float32).reshape(-1)
        assert p12.shape[0] == 12 and hits.shape[0] == 6 * mods.shape[0]
        out = np.zeros(12)
        d = self._lib.orc_eval_link(self._h, _ptr(pp), _ptr(p12), int(mods.shape[0]), _ptr(mods),
                                    _ptr(hits), _ptr(out))
        if d < 0:
            raise ValueError("oracle: 3 or 5 MDs")
        return bool(d), out

    def eval_margin(self, kind: int, mods, hits) -> float:
        """FP64 margin the chain records for one candidate of ``kind`` (MD,
        SEG, T3, T5) built from the given MDs: the relative distance to
        threshold of the cut that decides it (infinite when two cuts fail)."""
        n = {MD: 1, SEG: 2, T3: 3, T5: 5}[kind]
        mods = np.ascontiguousarray(np.atleast_1d(mods), np.int32)
        hits = np.ascontiguousarray(hits, np.float32).reshape(-1)
        assert mods.shape[0] == n and hits.shape[0] == 6 * n
        return float(self._lib.orc_eval_margin(self._h, int(kind), _ptr(mods), _ptr(hits)))
