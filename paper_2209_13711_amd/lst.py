"""ctypes binding of liblst (include/lst.h): same function names, argument
marshalling only.  PyTorch provides the device arena and the HIP stream; every
step of the chain runs in the library's kernels.

``import torch`` happens first so that the library binds to the HIP runtime
torch has already loaded (one runtime per process).  A missing or unloadable
library raises immediately: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblst.so")

LST_OK, LST_E_INVALID, LST_E_STATE, LST_E_CAPACITY, LST_E_HIP, LST_E_NOMEM = 0, -1, -2, -3, -4, -5
LST_E_FAULT = -6
LST_MD, LST_SEG, LST_T3, LST_T5, LST_T5_KEPT = 0, 1, 2, 3, 4
WIDTH = {LST_MD: 2, LST_SEG: 4, LST_T3: 6, LST_T5: 10, LST_T5_KEPT: 10}
LST_N_PARAMS = 14
LST_MOD_NF, LST_MOD_NI = 21, 4
LST_MODE_CUTS, LST_MODE_MLP = 0, 1
LST_MLP_NFEAT, LST_MLP_NPARAM = 40, 6849
LST_PX_N_PARAMS = 8
LST_TC_PT5, LST_TC_PT3, LST_TC_T5, LST_TC_PLS = 0, 1, 2, 3


class lst_caps(ctypes.Structure):
    _fields_ = [("events", ctypes.c_int32), ("hits", ctypes.c_int64), ("md", ctypes.c_int64),
                ("seg", ctypes.c_int64), ("t3", ctypes.c_int64), ("t5", ctypes.c_int64),
                ("features", ctypes.c_int32), ("px_hits", ctypes.c_int64),
                ("seeds", ctypes.c_int64), ("px_cand", ctypes.c_int64)]


class lst_counts(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("n_hits", "n_md", "n_seg", "n_t3", "n_t5",
                                               "n_t5_kept", "cand_md", "cand_seg", "cand_t3",
                                               "cand_t5")] + \
               [("overflow_mask", ctypes.c_int32), ("error_flags", ctypes.c_int32),
                ("dropped", ctypes.c_int64 * 4)] + \
               [(n, ctypes.c_int64) for n in ("n_pls", "cand_pt5", "n_pt5", "cand_pt3", "n_pt3",
                                               "n_tc")] + \
               [("mlp_fallback", ctypes.c_int32)]

    def as_dict(self):
        d = {n: getattr(self, n) for n, _ in self._fields_}
        d["dropped"] = list(self.dropped)
        return d


class LSTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblst error {code}: {msg}")
        self.code = code


_lib = None
_P = ctypes.c_void_p
_SIGS = {
    "lst_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _P, ctypes.c_int32]),
    "lst_destroy": (None, [_P]),
    "lst_last_error": (ctypes.c_char_p, [_P]),
    "lst_load_geometry": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    "lst_build_map": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P,
                                     ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "lst_get_map": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "lst_arena_bytes": (ctypes.c_int, [_P, ctypes.POINTER(lst_caps), ctypes.POINTER(ctypes.c_size_t)]),
    "lst_attach_arena": (ctypes.c_int, [_P, _P, ctypes.c_size_t, ctypes.POINTER(lst_caps)]),
    "lst_load_hits": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P, _P, _P, ctypes.c_int, _P]),
    "lst_run_sort": (ctypes.c_int, [_P, _P]),
    "lst_run_md": (ctypes.c_int, [_P, _P]),
    "lst_run_segments": (ctypes.c_int, [_P, _P]),
    "lst_run_triplets": (ctypes.c_int, [_P, _P]),
    "lst_run_quintuplets": (ctypes.c_int, [_P, _P]),
    "lst_run_dedup": (ctypes.c_int, [_P, _P]),
    "lst_run_chain": (ctypes.c_int, [_P, _P]),
    "lst_run_chain_graph": (ctypes.c_int, [_P, _P]),
    "lst_get_counts": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(lst_counts), _P]),
    "lst_raise_error_flags": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "lst_set_capacities": (ctypes.c_int, [_P, _P]),
    "lst_set_hit_storage": (ctypes.c_int, [_P, ctypes.c_int32]),
    "lst_load_pixel": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P,
                                      ctypes.c_int32, _P]),
    "lst_run_pixel": (ctypes.c_int, [_P, _P]),
    "lst_get_track_candidates": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int64,
                                                ctypes.POINTER(ctypes.c_int64), _P]),
    "lst_get_pixel_candidates": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P,
                                                ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), _P]),
    "lst_get_objects": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int64,
                                       ctypes.POINTER(ctypes.c_int64), _P]),
    "lst_get_t5_scores": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int64,
                                         ctypes.POINTER(ctypes.c_int64), _P]),
    "lst_stream_copy": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P]),
    "lst_run_chain_persistent": (ctypes.c_int, [_P, _P]),
    "lst_run_t5_features": (ctypes.c_int, [_P, _P]),
    "lst_get_t5_features": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int64,
                                           ctypes.POINTER(ctypes.c_int64), _P]),
    "lst_set_tuning": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32]),
    "lst_get_tuning": (ctypes.c_int, [_P, _P]),
    "lst_tune": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.c_int32, _P, _P]),
    "lst_mlp_load": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32, _P, _P, ctypes.c_float]),
    "lst_set_mode": (ctypes.c_int, [_P, ctypes.c_int32]),
    "lst_run_t5_score": (ctypes.c_int, [_P, _P]),
    "lst_run_t3_score": (ctypes.c_int, [_P, _P]),
    "lst_get_t3_logits": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.c_int64,
                                         ctypes.POINTER(ctypes.c_int64), _P]),
    "lst_run_t3_features": (ctypes.c_int, [_P, _P]),
    "lst_get_t3_features": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int64,
                                           ctypes.POINTER(ctypes.c_int64), _P]),
    "lst_get_t5_logits": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.c_int64,
                                         ctypes.POINTER(ctypes.c_int64), _P]),
    "lst_mlp_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64]),
    "lst_mlp_prepare": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int64, _P, _P]),
    "lst_mlp_forward": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, _P, _P, _P, _P]),
    "lst_mlp_backward": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int64, _P, _P, _P, _P,
                                        ctypes.c_size_t, _P, _P, _P]),
    "lst_mlp_backward_noalloc": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int64, _P, _P, _P, _P,
                                                _P, _P]),
    "lst_mlp_adam": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int32, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_float, ctypes.c_float, _P]),
    "lst_mlp_train_steps": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_int64, _P,
                                           ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P,
                                           ctypes.c_size_t, _P, _P, _P, _P, ctypes.c_float,
                                           ctypes.c_float, ctypes.c_float, ctypes.c_float, _P]),
}
EXPORTS = tuple(_SIGS)


def load_library():
    """Load liblst.so (built by paper_2209_13711_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"liblst.so not built ({LIB_PATH}); run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def lst_build_map(params, geo_f32, geo_i32):
    """Module map as (row_ptr, col) through the library's host-only entry point."""
    lib = load_library()
    params = np.ascontiguousarray(params, np.float64)
    f32 = np.ascontiguousarray(geo_f32, np.float32)
    i32 = np.ascontiguousarray(geo_i32, np.int32)
    n = f32.shape[1]
    ptr = np.zeros(n + 1, np.int32)
    ne = ctypes.c_int64(0)
    rc = lib.lst_build_map(_np_ptr(params), len(params), n, _np_ptr(f32), _np_ptr(i32),
                           _np_ptr(ptr), None, 0, ctypes.byref(ne))
    col = np.zeros(max(ne.value, 1), np.int32)
    rc = lib.lst_build_map(_np_ptr(params), len(params), n, _np_ptr(f32), _np_ptr(i32),
                           _np_ptr(ptr), _np_ptr(col), ne.value, ctypes.byref(ne))
    if rc != LST_OK:
        raise LSTError(rc, "lst_build_map")
    return ptr, col[:ne.value]


def lst_stream_copy(dst: "torch.Tensor", src: "torch.Tensor", stream=None):
    """Device copy dst <- src through the library's STREAM-like kernel."""
    lib = load_library()
    assert dst.is_cuda and src.is_cuda and dst.numel() * dst.element_size() == src.numel() * src.element_size()
    s = ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
    rc = lib.lst_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                             src.numel() * src.element_size(), s)
    if rc != LST_OK:
        raise LSTError(rc, "lst_stream_copy")


def default_caps(n_events: int, n_hits: int) -> dict:
    md = max(4096, int(1.5 * n_hits))
    return dict(events=n_events, hits=max(n_hits, 1), md=md, seg=6 * md, t3=4 * md, t5=4 * md,
                features=0, px_hits=0, seeds=0, px_cand=0)


class Context:
    """One detector geometry + parameter set on one GPU."""

    def __init__(self, params, geo_f32, geo_i32, device: int = 0):
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("liblst needs a HIP device")
        self.device = device
        self._params = np.ascontiguousarray(params, np.float64)
        h = _P()
        rc = self.lib.lst_create(ctypes.byref(h), device, _np_ptr(self._params), len(self._params))
        if rc != LST_OK:
            raise LSTError(rc, "lst_create")
        self.h = h
        f32 = np.ascontiguousarray(geo_f32, np.float32)
        i32 = np.ascontiguousarray(geo_i32, np.int32)
        self.n_mod = f32.shape[1]
        self._check(self.lib.lst_load_geometry(self.h, self.n_mod, _np_ptr(f32), _np_ptr(i32)))
        self.arena = None
        self.caps = None
        self.n_events = 0
        self._keep = []

    def __del__(self):
        if getattr(self, "h", None) is not None and self.lib is not None:
            self.lib.lst_destroy(self.h)
            self.h = None

    def _check(self, rc):
        if rc != LST_OK:
            raise LSTError(rc, self.lib.lst_last_error(self.h).decode())
        return rc

    @staticmethod
    def _stream(stream):
        if stream is None:
            stream = torch.cuda.current_stream()
        return ctypes.c_void_p(stream.cuda_stream)

    # -- memory -------------------------------------------------------------
    def arena_bytes(self, caps: dict) -> int:
        """bytes of the arena the library needs for `caps` (lst_arena_bytes)"""
        caps = dict(caps)
        for k in ("features", "px_hits", "seeds", "px_cand"):
            caps.setdefault(k, 0)
        c = lst_caps(**caps)
        nbytes = ctypes.c_size_t(0)
        self._check(self.lib.lst_arena_bytes(self.h, ctypes.byref(c), ctypes.byref(nbytes)))
        return int(nbytes.value)

    def reserve(self, caps: dict):
        caps = dict(caps)
        for k in ("features", "px_hits", "seeds", "px_cand"):
            caps.setdefault(k, 0)
        c = lst_caps(**caps)
        nbytes = ctypes.c_size_t(0)
        self._check(self.lib.lst_arena_bytes(self.h, ctypes.byref(c), ctypes.byref(nbytes)))
        if self.arena is None or self.arena.numel() < nbytes.value:
            self.arena = None
            torch.cuda.synchronize(self.device)
            self.arena = torch.empty(nbytes.value, dtype=torch.uint8, device=f"cuda:{self.device}")
        self._check(self.lib.lst_attach_arena(self.h, ctypes.c_void_p(self.arena.data_ptr()),
                                              self.arena.numel(), ctypes.byref(c)))
        self.caps = dict(caps)

    def module_map(self):
        ptr = np.zeros(self.n_mod + 1, np.int32)
        ne = ctypes.c_int64(0)
        self.lib.lst_get_map(self.h, _np_ptr(ptr), None, 0, ctypes.byref(ne))
        col = np.zeros(max(ne.value, 1), np.int32)
        self._check(self.lib.lst_get_map(self.h, _np_ptr(ptr), _np_ptr(col), ne.value, ctypes.byref(ne)))
        return ptr, col[:ne.value]

    # -- inputs -------------------------------------------------------------
    def load_hits(self, offsets, x, y, z, module, sensor, stream=None):
        """Host numpy arrays or device torch tensors (one batch)."""
        offsets = np.ascontiguousarray(offsets, np.int32)
        n_ev = len(offsets) - 1
        n = int(offsets[-1])
        if self.caps is None or self.caps["events"] < n_ev or self.caps["hits"] < n:
            caps = default_caps(n_ev, n)
            if self.caps is not None:
                for k in ("features", "px_hits", "seeds", "px_cand"):
                    caps[k] = self.caps.get(k, 0)
            self.reserve(caps)
        if isinstance(x, torch.Tensor):
            arrs = [x, y, z, module, sensor]
            for a in arrs:
                assert a.is_cuda and a.is_contiguous()
            ptrs = [ctypes.c_void_p(a.data_ptr()) for a in arrs]
            on_dev = 1
        else:
            arrs = [np.ascontiguousarray(x, np.float32), np.ascontiguousarray(y, np.float32),
                    np.ascontiguousarray(z, np.float32), np.ascontiguousarray(module, np.int32),
                    np.ascontiguousarray(sensor, np.uint8)]
            ptrs = [_np_ptr(a) for a in arrs]
            on_dev = 0
        self._keep = [offsets] + arrs       # host buffers must outlive the async copies
        self._check(self.lib.lst_load_hits(self.h, n_ev, _np_ptr(offsets), *ptrs, on_dev,
                                           self._stream(stream)))
        self.n_events = n_ev

    # -- stages -------------------------------------------------------------
    def run_sort(self, stream=None):
        self._check(self.lib.lst_run_sort(self.h, self._stream(stream)))

    def run_md(self, stream=None):
        self._check(self.lib.lst_run_md(self.h, self._stream(stream)))

    def run_segments(self, stream=None):
        self._check(self.lib.lst_run_segments(self.h, self._stream(stream)))

    def run_triplets(self, stream=None):
        self._check(self.lib.lst_run_triplets(self.h, self._stream(stream)))

    def run_quintuplets(self, stream=None):
        self._check(self.lib.lst_run_quintuplets(self.h, self._stream(stream)))

    def run_dedup(self, stream=None):
        self._check(self.lib.lst_run_dedup(self.h, self._stream(stream)))

    def run_chain(self, stream=None):
        self._check(self.lib.lst_run_chain(self.h, self._stream(stream)))

    def run_chain_graph(self, stream=None):
        self._check(self.lib.lst_run_chain_graph(self.h, self._stream(stream)))

    def run_chain_persistent(self, stream=None):
        self._check(self.lib.lst_run_chain_persistent(self.h, self._stream(stream)))

    def tuning(self) -> dict:
        out = np.zeros(15, np.int32)
        self._check(self.lib.lst_get_tuning(self.h, _np_ptr(out)))
        return dict(grid=out[:6].tolist(), lanes=out[6:12].tolist(), persistent=int(out[12]),
                    blocks_per_cu=int(out[13]), n_cu=int(out[14]))

    def set_tuning(self, grid, persistent=0, blocks_per_cu=1, lanes=None):
        g = np.ascontiguousarray(grid, np.int32)
        ln = None if lanes is None else np.ascontiguousarray(lanes, np.int32)
        self._check(self.lib.lst_set_tuning(self.h, _np_ptr(g), None if ln is None else _np_ptr(ln),
                                            int(persistent), int(blocks_per_cu)))

    def tune(self, cache_path=None, reps=5, stream=None) -> dict:
        """Autotune the launch shape on the loaded batch (see lst_tune)."""
        rep = np.zeros(8, np.float64)
        cp = cache_path.encode() if cache_path else None
        self._check(self.lib.lst_tune(self.h, cp, int(reps), _np_ptr(rep), self._stream(stream)))
        out = self.tuning()
        out["report_us"] = rep.tolist()
        return out

    # -- outputs ------------------------------------------------------------
    def counts(self, event=0, stream=None, check=True) -> dict:
        c = lst_counts()
        rc = self.lib.lst_get_counts(self.h, event, ctypes.byref(c), self._stream(stream))
        if check:
            self._check(rc)
        d = c.as_dict()
        d["rc"] = rc
        return d

    def set_hit_storage(self, fp16: bool):
        """hits grouped as module-local FP16 (u, v) (lst_set_hit_storage)"""
        self._check(self.lib.lst_set_hit_storage(self.h, int(bool(fp16))))

    def set_capacities(self, caps=None):
        """per-module capacities of MD, SEG, T3, T5 (0 = none; None = off)"""
        if caps is None:
            self._check(self.lib.lst_set_capacities(self.h, None))
        else:
            c = np.ascontiguousarray(caps, np.int32)
            assert c.shape == (4,)
            self._keep_caps = c
            self._check(self.lib.lst_set_capacities(self.h, _np_ptr(c)))

    # -- pixel objects and track candidates ----------------------------------
    def load_pixel(self, px_offsets, x, y, z, seed_offsets, seeds, pix_params, stream=None):
        """pixel hits and seeds of the loaded batch (host arrays); grows the
        arena's pixel capacities when needed (which needs the hits loaded
        again: call before the chain)"""
        px_offsets = np.ascontiguousarray(px_offsets, np.int32)
        seed_offsets = np.ascontiguousarray(seed_offsets, np.int32)
        n_px, n_sd = int(px_offsets[-1]), int(seed_offsets[-1])
        need = dict(px_hits=max(n_px, 1), seeds=max(n_sd, 1), px_cand=max(4096, 8 * n_sd))
        if any(self.caps.get(k, 0) < v for k, v in need.items()):
            raise LSTError(LST_E_CAPACITY, f"reserve pixel capacities first: {need}")
        arrs = [np.ascontiguousarray(a, np.float32) for a in (x, y, z)]
        sd = np.ascontiguousarray(seeds, np.int32).reshape(-1)
        pp = np.ascontiguousarray(pix_params, np.float64)
        self._keep_px = [px_offsets, seed_offsets, sd, pp] + arrs
        self._check(self.lib.lst_load_pixel(self.h, len(px_offsets) - 1, _np_ptr(px_offsets),
                                            *[_np_ptr(a) for a in arrs], _np_ptr(seed_offsets),
                                            _np_ptr(sd), _np_ptr(pp), len(pp), self._stream(stream)))

    def pixel_caps(self, n_px, n_seeds):
        """reserve an arena that also holds n_px pixel hits and n_seeds seeds"""
        caps = dict(self.caps)
        caps.update(px_hits=max(n_px, 1, caps.get("px_hits", 0)),
                    seeds=max(n_seeds, 1, caps.get("seeds", 0)),
                    px_cand=max(4096, 8 * n_seeds, caps.get("px_cand", 0)))
        if caps != self.caps:
            self.reserve(caps)

    def run_pixel(self, stream=None):
        self._check(self.lib.lst_run_pixel(self.h, self._stream(stream)))

    def _rows(self, fn, width, *args, stream=None):
        n = ctypes.c_int64(0)
        rc = fn(self.h, *args, None, 0, ctypes.byref(n), self._stream(stream))
        if rc not in (LST_OK, LST_E_CAPACITY):
            self._check(rc)
        out = np.zeros((max(n.value, 1), width), np.int32)
        self._check(fn(self.h, *args, _np_ptr(out), n.value, ctypes.byref(n), self._stream(stream)))
        return out[:n.value]

    def track_candidates(self, event, stream=None) -> np.ndarray:
        """[n, 12]: type, seed (-1 for T5), outer hits (-1 padded)"""
        return self._rows(self.lib.lst_get_track_candidates, 12, event, stream=stream)

    def pixel_candidates(self, event, what, stream=None) -> np.ndarray:
        """[n, 13]: seed, outer hits (-1 padded), score bits, kept (what 0 pT5, 1 pT3)"""
        return self._rows(self.lib.lst_get_pixel_candidates, 13, event, int(what), stream=stream)

    def run_event_pixel(self, ev, px, pix_params, stream=None, graph=False):
        """one event through the chain and the pixel stage"""
        offs = np.array([0, ev.n_hits], np.int32)
        if self.caps is None:
            self.reserve(default_caps(1, ev.n_hits))
        self.pixel_caps(px.n_hits, px.n_seeds)
        self.run_batch(offs, ev.x, ev.y, ev.z, ev.module, ev.sensor, stream, graph=graph)
        self.load_pixel(np.array([0, px.n_hits], np.int32), px.x, px.y, px.z,
                        np.array([0, px.n_seeds], np.int32), px.seeds, pix_params, stream)
        self.run_pixel(stream)
        return self.track_candidates(0, stream)

    def raise_error_flags(self, bits, stream=None):
        """test hook: OR error bits 1/2 into the device error word (lst_raise_error_flags)"""
        self._check(self.lib.lst_raise_error_flags(self.h, int(bits), self._stream(stream)))

    def _hint(self, kind):
        """rows an output of `kind` can hold at most: the arena's capacity"""
        key = {LST_MD: "md", LST_SEG: "seg", LST_T3: "t3", LST_T5: "t5", LST_T5_KEPT: "t5"}[kind]
        return int(self.caps.get(key, 0)) if self.caps else 0

    def _fetch(self, call, shape, dtype, hint):
        """One getter call into a buffer of `hint` rows (the getters copy the
        device arrays on every call); a second call only when they do not
        fit.  `call(out_ptr, cap, n)` returns the status."""
        n = ctypes.c_int64(0)
        out = np.empty((max(hint, 1),) + shape, dtype)
        rc = call(_np_ptr(out), hint, n)
        if rc == LST_E_CAPACITY and n.value > hint:
            out = np.empty((n.value,) + shape, dtype)
            rc = call(_np_ptr(out), n.value, n)
        self._check(rc)
        return out[:n.value]

    def objects(self, event, kind, stream=None) -> np.ndarray:
        st = self._stream(stream)
        return self._fetch(lambda o, cap, n: self.lib.lst_get_objects(
            self.h, event, kind, o, cap, ctypes.byref(n), st), (WIDTH[kind],), np.int32,
            self._hint(kind))

    def run_t5_features(self, stream=None):
        self._check(self.lib.lst_run_t5_features(self.h, self._stream(stream)))

    def _features(self, fn, event, stream, kind):
        st = self._stream(stream)
        return self._fetch(lambda o, cap, n: fn(self.h, event, o, cap, ctypes.byref(n), st),
                           (40,), np.float32, self._hint(kind))

    def t5_features(self, event, stream=None) -> np.ndarray:
        return self._features(self.lib.lst_get_t5_features, event, stream, LST_T5)

    def run_t3_features(self, stream=None):
        self._check(self.lib.lst_run_t3_features(self.h, self._stream(stream)))

    def t3_features(self, event, stream=None) -> np.ndarray:
        return self._features(self.lib.lst_get_t3_features, event, stream, LST_T3)

    def t5_scores(self, event, stream=None) -> np.ndarray:
        n = ctypes.c_int64(0)
        rc = self.lib.lst_get_t5_scores(self.h, event, None, 0, ctypes.byref(n), self._stream(stream))
        if rc not in (LST_OK, LST_E_CAPACITY):
            self._check(rc)
        out = np.zeros(max(n.value, 1), np.float32)
        self._check(self.lib.lst_get_t5_scores(self.h, event, _np_ptr(out), n.value,
                                               ctypes.byref(n), self._stream(stream)))
        return out[:n.value]

    # -- learned scorer -----------------------------------------------------
    def mlp_load(self, params, mean, istd, threshold=0.0, kind=LST_T5):
        """load the scorer of `kind` (LST_T3 or LST_T5)"""
        p = np.ascontiguousarray(params, np.float32)
        m = np.ascontiguousarray(mean, np.float32)
        s = np.ascontiguousarray(istd, np.float32)
        self._check(self.lib.lst_mlp_load(self.h, int(kind), _np_ptr(p), len(p), _np_ptr(m),
                                          _np_ptr(s), float(threshold)))

    def set_mode(self, mode):
        self._check(self.lib.lst_set_mode(self.h, int(mode)))

    def run_t5_score(self, stream=None):
        self._check(self.lib.lst_run_t5_score(self.h, self._stream(stream)))

    def run_t3_score(self, stream=None):
        self._check(self.lib.lst_run_t3_score(self.h, self._stream(stream)))

    def _logits(self, fn, event, stream):
        n = ctypes.c_int64(0)
        rc = fn(self.h, event, None, None, 0, ctypes.byref(n), self._stream(stream))
        if rc not in (LST_OK, LST_E_CAPACITY):
            self._check(rc)
        lg = np.zeros(max(n.value, 1), np.float32)
        vt = np.zeros(max(n.value, 1), np.uint8)
        self._check(fn(self.h, event, _np_ptr(lg), _np_ptr(vt), n.value, ctypes.byref(n),
                       self._stream(stream)))
        return lg[:n.value], vt[:n.value].astype(bool)

    def t5_logits(self, event, stream=None):
        """(logits float32, veto bool) in lst_get_objects(LST_T5) order"""
        return self._logits(self.lib.lst_get_t5_logits, event, stream)

    def t3_logits(self, event, stream=None):
        """(logits float32, veto bool) in lst_get_objects(LST_T3) order"""
        return self._logits(self.lib.lst_get_t3_logits, event, stream)

    # training calls: device tensors, asynchronous on the stream
    @staticmethod
    def _dev(t, dtype):
        assert t.is_cuda and t.is_contiguous() and t.dtype == dtype, (t.dtype, dtype)
        return ctypes.c_void_p(t.data_ptr())

    def mlp_workspace_bytes(self, n):
        return int(self.lib.lst_mlp_workspace_bytes(int(n)))

    def mlp_prepare(self, feat, mean, istd, x, stream=None):
        d = self._dev
        self._check(self.lib.lst_mlp_prepare(self.h, d(feat, torch.float32), d(mean, torch.float32),
                                             d(istd, torch.float32), feat.shape[0],
                                             d(x, torch.int16), self._stream(stream)))

    def mlp_forward(self, params, x, logits, h1=None, h2=None, stream=None):
        d = self._dev
        self._check(self.lib.lst_mlp_forward(
            self.h, d(params, torch.float32), d(x, torch.int16), x.shape[0],
            d(logits, torch.float32), None if h1 is None else d(h1, torch.int16),
            None if h2 is None else d(h2, torch.float32), self._stream(stream)))

    def mlp_backward(self, params, x, y, logits, h1, h2, work, grad, loss, stream=None):
        d = self._dev
        self._check(self.lib.lst_mlp_backward(
            self.h, d(params, torch.float32), d(x, torch.int16), d(y, torch.uint8), x.shape[0],
            d(logits, torch.float32), d(h1, torch.int16), d(h2, torch.float32),
            d(work, torch.uint8), work.numel(), d(grad, torch.float32), d(loss, torch.float32),
            self._stream(stream)))

    def mlp_backward_noalloc(self, params, x, y, logits, h1, h2, grad, loss, stream=None):
        """lst_mlp_backward with the library's fixed workspace (no allocation)"""
        d = self._dev
        self._check(self.lib.lst_mlp_backward_noalloc(
            self.h, d(params, torch.float32), d(x, torch.int16), d(y, torch.uint8), x.shape[0],
            d(logits, torch.float32), d(h1, torch.int16), d(h2, torch.float32),
            d(grad, torch.float32), d(loss, torch.float32), self._stream(stream)))

    def mlp_adam(self, params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        d = self._dev
        self._check(self.lib.lst_mlp_adam(self.h, d(params, torch.float32), d(grad, torch.float32),
                                          d(m, torch.float32), d(v, torch.float32), int(step),
                                          float(lr), float(beta1), float(beta2), float(eps),
                                          self._stream(stream)))

    def mlp_train_steps(self, params, x, y, batch, order, first_step, logits, h1, h2, work, grad,
                        m, v, losses, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        """len(order) Adam steps on the batches order[i] of x, y (see lst_mlp_train_steps)"""
        d = self._dev
        order = np.ascontiguousarray(order, np.int32)
        self._check(self.lib.lst_mlp_train_steps(
            self.h, d(params, torch.float32), d(x, torch.int16), d(y, torch.uint8), x.shape[0],
            int(batch), _np_ptr(order) if len(order) else None, len(order), int(first_step),
            d(logits, torch.float32), d(h1, torch.int16), d(h2, torch.float32),
            d(work, torch.uint8), work.numel(), d(grad, torch.float32), d(m, torch.float32),
            d(v, torch.float32), d(losses, torch.float32), float(lr), float(beta1), float(beta2),
            float(eps), self._stream(stream)))

    def run_batch(self, offsets, x, y, z, module, sensor, stream=None, max_retry=8, graph=False):
        """Load, run the chain and grow the arena to the reported need on overflow
        (a stage's need is known once its upstream fits: one retry per stage)."""
        for _ in range(max_retry):
            self.load_hits(offsets, x, y, z, module, sensor, stream)
            if graph:
                self.run_chain_graph(stream)
            else:
                self.run_chain(stream)
            c = lst_counts()
            ovf = False
            for e in range(self.n_events):
                rc = self.lib.lst_get_counts(self.h, e, ctypes.byref(c), self._stream(stream))
                if rc == LST_E_CAPACITY:
                    ovf = True
                elif rc != LST_OK:
                    self._check(rc)
            if not ovf:
                return
            # on overflow every event reports the batch-wide requirement
            self.lib.lst_get_counts(self.h, 0, ctypes.byref(c), self._stream(stream))
            tot = {"md": c.n_md, "seg": c.n_seg, "t3": c.n_t3, "t5": c.n_t5}
            caps = dict(self.caps)
            for k in tot:
                caps[k] = max(caps[k], int(tot[k] * 1.25) + 1024)
            self.reserve(caps)
        raise LSTError(LST_E_CAPACITY, "capacity still exceeded after growing the arena")

    def run_event(self, ev, stream=None, graph=False):
        offs = np.array([0, ev.n_hits], np.int32)
        self.run_batch(offs, ev.x, ev.y, ev.z, ev.module, ev.sensor, stream, graph=graph)
        return {k: self.objects(0, k, stream) for k in WIDTH}
