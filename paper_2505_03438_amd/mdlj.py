"""Thin ctypes binding of libmdlj (include/mdlj.h): the same names, argument
marshalling only.  Device arrays are torch tensors on the GPU; every call runs
on torch's current HIP stream unless a stream is given.  Raises RuntimeError
when the library is missing or a call fails; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

MD_MAX_TYPES = 2
MD_OK = 0
MD_ERR_INVALID_ARG = -1
MD_ERR_BOX_TOO_SMALL = -2
MD_ERR_LIST_OVERFLOW = -3
MD_ERR_NONFINITE = -4
MD_ERR_HIP = -5
MD_ERR_NOT_BUILT = -6
MD_ERR_NO_DEVICE = -7

MD_FP32 = 0
MD_FP64 = 1
MD_CONTAINER_LC = 0
MD_CONTAINER_VL = 1
MD_CONTAINER_CL = 2
MD_CONTAINER_PVL = 3
MD_CONTAINER_VLC = 4
MD_N3L_OFF = 0
MD_N3L_ON = 1
MD_N3L_C08 = 2
MD_LAYOUT_PACKED = 0
MD_LAYOUT_ALIGNED = 1
MD_LAYOUT_SOA = 2
MD_TUNE_OFF = 0
MD_TUNE_FULL = 1
MD_TUNE_PREDICTIVE = 2
MD_TUNE_EXPERT = 3
MD_TUNE_RF = 4
MD_SUIT_BAD = 0
MD_SUIT_OKAY = 1
MD_SUIT_GOOD = 2
MD_FLAG_LIST_OVERFLOW = 1
MD_FLAG_SKIN_EXCEEDED = 2
MD_FLAG_NONFINITE = 4
MD_FLAG_WINDOW_FALLBACK = 8

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmdlj.so")


class md_config(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("n_types", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("box", ctypes.c_double * 3),
        ("rc2", ctypes.c_double * (MD_MAX_TYPES * MD_MAX_TYPES)),
        ("skin", ctypes.c_double),
        ("csf", ctypes.c_double),
        ("container", ctypes.c_int32),
        ("newton3", ctypes.c_int32),
        ("rebuild_interval", ctypes.c_int32),
        ("max_neighbors", ctypes.c_int32),
        ("autotune", ctypes.c_int32),
        ("tune_interval", ctypes.c_int32),
        ("tune_trial_steps", ctypes.c_int32),
        ("total_steps_hint", ctypes.c_int32),
        ("tune_skin", ctypes.c_int32),
        ("tune_first", ctypes.c_int32),
        ("layout", ctypes.c_int32),
    ]


class md_fuzzy_rule(ctypes.Structure):
    """IF stats[input[0]] IS trap[0] (AND stats[input[1]] IS trap[1]) THEN
    suitability(config) IS then; input[1] = -1 for one antecedent."""
    _fields_ = [("input", ctypes.c_int32 * 2), ("trap", (ctypes.c_double * 4) * 2),
                ("config", ctypes.c_int32), ("then", ctypes.c_int32)]


def fuzzy_rules(rules):
    """ctypes array of md_fuzzy_rule from dicts {"if": [(stat index,
    (a, b, c, d)), ...] (one or two), "config": c, "then": MD_SUIT_*}."""
    arr = (md_fuzzy_rule * max(len(rules), 1))()
    for k, r in enumerate(rules):
        ants = list(r["if"])
        if not 1 <= len(ants) <= 2:
            raise ValueError("a rule has one or two antecedents")
        arr[k].input[0] = int(ants[0][0])
        arr[k].input[1] = int(ants[1][0]) if len(ants) == 2 else -1
        for j, (_, trap) in enumerate(ants):
            for q in range(4):
                arr[k].trap[j][q] = float(trap[q])
        arr[k].config = int(r["config"])
        arr[k].then = int(r["then"])
    return arr


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_d = ctypes.c_double

# name -> (restype, argtypes)
_SIGS = {
    "md_config_default": (_i32, [ctypes.POINTER(md_config), _i64, _d]),
    "md_create": (_i32, [ctypes.POINTER(md_config), ctypes.POINTER(_vp)]),
    "md_destroy": (None, [_vp]),
    "md_build_cells": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "md_build_neighbors": (_i32, [_vp, _vp, _vp, _vp]),
    "md_compute_forces": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "md_step": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _d, _i32, _i32, _vp, _vp]),
    "md_forces_backward": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "md_live_stats": (_i32, [_vp, _vp, _vp, _vp]),
    "md_get_neighbors": (_i32, [_vp, _vp, _vp, _i32, _vp]),
    "md_status": (_i32, [_vp, ctypes.POINTER(ctypes.c_uint32)]),
    "md_get_config": (_i32, [_vp, ctypes.POINTER(md_config)]),
    "md_get_counters": (_i32, [_vp, _vp]),
    "md_timing": (_i32, [_vp, _i32, _vp]),
    "md_get_phase_choices": (_i32, [_vp, _vp, _i32]),
    "md_get_trial_scores": (_i32, [_vp, _vp, _vp, _i32]),
    "md_set_expert_rules": (_i32, [_vp, _vp, _i32]),
    "md_expert_suitability": (_i32, [_vp, _i32, _i32, _vp, _vp]),
    "md_rf_predict": (_i32, [_vp, _i32]),
    "md_last_error": (ctypes.c_char_p, []),
    "md_compute_forces_noalloc": (_i32, [ctypes.POINTER(md_config), _vp, _vp, _vp, _vp, _vp, _vp]),
    "md_noalloc_max_particles": (_i64, []),
    "md_batch_create": (_i32, [ctypes.POINTER(md_config), _i32, _vp, _vp, ctypes.POINTER(_vp)]),
    "md_batch_destroy": (None, [_vp]),
    "md_batch_build_cells": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "md_batch_compute_forces": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "md_batch_step": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _d, _i32, _i32, _vp]),
    "md_batch_get_counters": (_i32, [_vp, _vp]),
    "md_tuner_create": (_i32, [_i32, _i32, _i32, _d, _d, ctypes.POINTER(_vp)]),
    "md_tuner_destroy": (None, [_vp]),
    "md_tuner_begin_phase": (_i32, [_vp, _vp]),
    "md_tuner_set_suitability": (_i32, [_vp, _vp]),
    "md_tuner_report": (_i32, [_vp, _i32, _d]),
    "md_tuner_end_phase": (_i32, [_vp]),
    "md_tuner_blacklist": (_i32, [_vp, _vp]),
}

_lib = None


def lib():
    """Load libmdlj.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmdlj.so is missing: build it with "
                               "`python -m paper_2505_03438_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def md_last_error() -> str:
    return lib().md_last_error().decode()


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise RuntimeError("%s failed (%d): %s" % (what, rc, md_last_error()))
    return rc


def _stream(stream):
    if stream is None:
        return _vp(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return _vp(stream.cuda_stream)
    return _vp(int(stream))


def _ptr(t, dtype=None, numel=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must have %d elements, got %d" % (name, numel, t.numel()))
    return _vp(t.data_ptr())


def config_default(n: int, L: float) -> md_config:
    c = md_config()
    _check(lib().md_config_default(ctypes.byref(c), int(n), float(L)), "md_config_default")
    return c


class Handle:
    """Owns an md_handle; remembers n, the real dtype and the type count."""

    def __init__(self, cfg: md_config):
        self._h = _vp()
        _check(lib().md_create(ctypes.byref(cfg), ctypes.byref(self._h)), "md_create")
        self.n = int(cfg.n)
        self.n_types = int(cfg.n_types)
        self.real = torch.float64 if cfg.precision == MD_FP64 else torch.float32

    @property
    def ptr(self):
        return self._h

    def close(self):
        if self._h and self._h.value:
            lib().md_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def md_create(cfg: md_config) -> Handle:
    return Handle(cfg)


def md_destroy(h: Handle) -> None:
    h.close()


def _particles(h, pos, vel=None, force=None, type=None, ids=None):
    n = h.n
    return (_ptr(pos, torch.float64, 3 * n, "pos"), _ptr(vel, h.real, 3 * n, "vel"),
            _ptr(force, h.real, 3 * n, "force"), _ptr(type, torch.int32, n, "type"),
            _ptr(ids, torch.int32, n, "ids"))


def md_build_cells(h: Handle, pos, vel, force, type, ids, stream=None):
    p, v, f, t, i = _particles(h, pos, vel, force, type, ids)
    _check(lib().md_build_cells(h.ptr, p, v, f, t, i, _stream(stream)), "md_build_cells")


def md_build_neighbors(h: Handle, pos, type, stream=None):
    p, _, _, t, _ = _particles(h, pos, type=type)
    _check(lib().md_build_neighbors(h.ptr, p, t, _stream(stream)), "md_build_neighbors")


def md_compute_forces(h: Handle, pos, type, lj, force, out=None, stream=None):
    p, _, f, t, _ = _particles(h, pos, force=force, type=type)
    _check(lib().md_compute_forces(h.ptr, p, t, _ptr(lj, torch.float64, 2 * h.n_types, "lj"), f,
                                   _ptr(out, torch.float64, 4, "out"), _stream(stream)),
           "md_compute_forces")


def md_compute_forces_noalloc(cfg: md_config, pos, type, lj, force, out=None, stream=None):
    """Allocation-free forces without a handle (linked cells, gather-only),
    arrays in the caller's order."""
    n = int(cfg.n)
    real = torch.float64 if cfg.precision == MD_FP64 else torch.float32
    _check(lib().md_compute_forces_noalloc(ctypes.byref(cfg), _ptr(pos, torch.float64, 3 * n, "pos"),
                                           _ptr(type, torch.int32, n, "type"),
                                           _ptr(lj, torch.float64, 2 * int(cfg.n_types), "lj"),
                                           _ptr(force, real, 3 * n, "force"), _ptr(out, torch.float64, 4, "out"),
                                           _stream(stream)),
           "md_compute_forces_noalloc")


def md_noalloc_max_particles() -> int:
    return int(lib().md_noalloc_max_particles())


def md_step(h: Handle, pos, vel, force, type, ids, inv_mass, lj, dt, nsteps, energy_every=0,
            log=None, stream=None):
    p, v, f, t, i = _particles(h, pos, vel, force, type, ids)
    nlog = (nsteps // energy_every) * 4 if (log is not None and energy_every > 0) else None
    _check(lib().md_step(h.ptr, p, v, f, t, i, _ptr(inv_mass, torch.float64, h.n_types, "inv_mass"),
                         _ptr(lj, torch.float64, 2 * h.n_types, "lj"), float(dt), int(nsteps),
                         int(energy_every), _ptr(log, torch.float64, nlog, "log"), _stream(stream)),
           "md_step")


def md_forces_backward(h: Handle, pos, type, lj, grad_force, grad_pos, grad_lj, stream=None):
    p, _, g, t, _ = _particles(h, pos, force=grad_force, type=type)
    _check(lib().md_forces_backward(h.ptr, p, t, _ptr(lj, torch.float64, 2 * h.n_types, "lj"), g,
                                    _ptr(grad_pos, torch.float64, 3 * h.n, "grad_pos"),
                                    _ptr(grad_lj, torch.float64, 2 * h.n_types, "grad_lj"),
                                    _stream(stream)),
           "md_forces_backward")


def md_live_stats(h: Handle, pos, stream=None):
    out = (ctypes.c_double * 8)()
    _check(lib().md_live_stats(h.ptr, _ptr(pos, torch.float64, 3 * h.n, "pos"), out, _stream(stream)),
           "md_live_stats")
    return list(out)


def md_get_neighbors(h: Handle, max_per_row: int = 256, stream=None):
    """(counts int32[n], rows int32[n, max_per_row]) device tensors, cell order."""
    counts = torch.zeros(h.n, dtype=torch.int32, device="cuda")
    rows = torch.full((h.n, max_per_row), -1, dtype=torch.int32, device="cuda")
    _check(lib().md_get_neighbors(h.ptr, _ptr(counts), _ptr(rows), int(max_per_row), _stream(stream)),
           "md_get_neighbors")
    return counts, rows


def md_status(h: Handle) -> int:
    f = ctypes.c_uint32()
    _check(lib().md_status(h.ptr, ctypes.byref(f)), "md_status")
    return int(f.value)


def md_get_config(h: Handle) -> md_config:
    c = md_config()
    _check(lib().md_get_config(h.ptr, ctypes.byref(c)), "md_get_config")
    return c


def md_get_counters(h: Handle):
    out = (ctypes.c_int64 * 7)()
    _check(lib().md_get_counters(h.ptr, out), "md_get_counters")
    keys = ("rebuilds", "forced_rebuilds", "tuning_phases", "trials", "config_index", "list_entries",
            "force_family")
    return dict(zip(keys, list(out)))


def md_get_phase_choices(h: Handle):
    """Tuning-space index chosen by every tuning phase so far."""
    m = lib().md_get_phase_choices(h.ptr, None, 0)
    _check(m if m < 0 else 0, "md_get_phase_choices")
    out = (ctypes.c_int32 * max(m, 1))()
    lib().md_get_phase_choices(h.ptr, out, m)
    return list(out[:m])


def md_get_trial_scores(h: Handle, n_max: int = 64):
    """Last trial score (ms per step, NaN if never trialled) and the
    configuration of every entry of the handle's tuning space."""
    scores = (ctypes.c_double * n_max)()
    cfgs = (md_config * n_max)()
    m = lib().md_get_trial_scores(h.ptr, scores, cfgs, n_max)
    _check(m if m < 0 else 0, "md_get_trial_scores")
    return list(scores[:m]), [cfgs[k] for k in range(m)]


def md_set_expert_rules(h: Handle, rules=None):
    """Rules of the Expert strategy (dicts as in fuzzy_rules); None restores
    the built-in rules."""
    if not rules:
        _check(lib().md_set_expert_rules(h.ptr, None, 0), "md_set_expert_rules")
    else:
        _check(lib().md_set_expert_rules(h.ptr, fuzzy_rules(rules), len(rules)), "md_set_expert_rules")


def md_expert_suitability(stats, n_configs: int = 7, rules=None):
    """Crisp suitability per configuration (host only); rules None: the
    built-in rules."""
    st = (ctypes.c_double * 8)(*[float(v) for v in stats])
    out = (ctypes.c_double * n_configs)()
    arr = fuzzy_rules(rules) if rules is not None else None
    _check(lib().md_expert_suitability(arr, len(rules) if rules is not None else 0, n_configs, st, out),
           "md_expert_suitability")
    return list(out)


def md_rf_predict(stats, n_configs: int = 7) -> int:
    """Configuration the built-in Random Forest predicts (host only)."""
    st = (ctypes.c_double * 8)(*[float(v) for v in stats])
    return _check(lib().md_rf_predict(st, n_configs), "md_rf_predict")


def md_timing(h: Handle, enable: bool, want: bool = True):
    """Start (True) / stop (False) kernel-class timing of md_step; returns
    {force_ms, force_passes, build_ms, builds} accumulated so far."""
    out = (ctypes.c_double * 4)()
    _check(lib().md_timing(h.ptr, 1 if enable else 0, out if want else None), "md_timing")
    return dict(zip(("force_ms", "force_passes", "build_ms", "builds"), list(out)))


# ---------------------------------------------------------------- batched systems

class Batch:
    def __init__(self, cfg: md_config, offsets, boxes):
        import numpy as np
        offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        bx = np.ascontiguousarray(np.asarray(boxes, dtype=np.float64).reshape(-1))
        self.n_sys = offs.size - 1
        self.n = int(offs[-1])
        self.n_types = int(cfg.n_types)
        self.real = torch.float64 if cfg.precision == MD_FP64 else torch.float32
        self._b = _vp()
        _check(lib().md_batch_create(ctypes.byref(cfg), self.n_sys, _vp(offs.ctypes.data),
                                     _vp(bx.ctypes.data), ctypes.byref(self._b)), "md_batch_create")

    @property
    def ptr(self):
        return self._b

    def close(self):
        if self._b and self._b.value:
            lib().md_batch_destroy(self._b)
            self._b = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def md_batch_create(cfg, offsets, boxes) -> Batch:
    return Batch(cfg, offsets, boxes)


def md_batch_destroy(b: Batch) -> None:
    b.close()


def md_batch_build_cells(b: Batch, pos, vel, force, type, ids, stream=None):
    p, v, f, t, i = _particles(b, pos, vel, force, type, ids)
    _check(lib().md_batch_build_cells(b.ptr, p, v, f, t, i, _stream(stream)), "md_batch_build_cells")


def md_batch_compute_forces(b: Batch, pos, type, lj, force, out=None, stream=None):
    p, _, f, t, _ = _particles(b, pos, force=force, type=type)
    _check(lib().md_batch_compute_forces(b.ptr, p, t, _ptr(lj, torch.float64, 2 * b.n_types, "lj"), f,
                                         _ptr(out, torch.float64, 4 * b.n_sys, "out"), _stream(stream)),
           "md_batch_compute_forces")


def md_batch_step(b: Batch, pos, vel, force, type, ids, inv_mass, lj, dt, nsteps, use_graph=True,
                  stream=None):
    p, v, f, t, i = _particles(b, pos, vel, force, type, ids)
    _check(lib().md_batch_step(b.ptr, p, v, f, t, i, _ptr(inv_mass, torch.float64, b.n_types, "inv_mass"),
                               _ptr(lj, torch.float64, 2 * b.n_types, "lj"), float(dt), int(nsteps),
                               1 if use_graph else 0, _stream(stream)),
           "md_batch_step")


def md_batch_get_counters(b: Batch) -> dict:
    out = (ctypes.c_int64 * 4)()
    _check(lib().md_batch_get_counters(b.ptr, out), "md_batch_get_counters")
    return dict(zip(("rebuilds", "forced_rebuilds", "steps", "rebuild_interval"), (int(x) for x in out)))


# ---------------------------------------------------------------- tuner engine (host only)

class Tuner:
    def __init__(self, strategy: int, n_configs: int, total_phases: int, rel_threshold: float = 2.0,
                 blacklist_factor: float = 10.0):
        self.n = n_configs
        self._t = _vp()
        _check(lib().md_tuner_create(strategy, n_configs, total_phases, rel_threshold, blacklist_factor,
                                     ctypes.byref(self._t)), "md_tuner_create")

    def begin_phase(self):
        arr = (ctypes.c_int32 * self.n)()
        _check(lib().md_tuner_begin_phase(self._t, arr), "md_tuner_begin_phase")
        return [c for c in range(self.n) if arr[c]]

    def set_suitability(self, suit):
        arr = (ctypes.c_double * self.n)(*[float(v) for v in suit])
        _check(lib().md_tuner_set_suitability(self._t, arr), "md_tuner_set_suitability")

    def report(self, c: int, score: float):
        _check(lib().md_tuner_report(self._t, int(c), float(score)), "md_tuner_report")

    def end_phase(self) -> int:
        return _check(lib().md_tuner_end_phase(self._t), "md_tuner_end_phase")

    def blacklisted(self):
        arr = (ctypes.c_int32 * self.n)()
        _check(lib().md_tuner_blacklist(self._t, arr), "md_tuner_blacklist")
        return [c for c in range(self.n) if arr[c]]

    def __del__(self):
        try:
            if self._t and self._t.value:
                lib().md_tuner_destroy(self._t)
        except Exception:
            pass
