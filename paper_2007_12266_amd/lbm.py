"""Thin ctypes binding of the colour-LBM C-ABI (include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels of liblbm.so. The
library must have been built (``python -m paper_2007_12266_amd.build``); loading fails loudly
otherwise. PyTorch, when present, provides the device memory (through the caching allocator) and
the stream; it never computes anything here.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_ERR_ARG, LBM_ERR_OOM, LBM_ERR_DEVICE, LBM_ERR_UNSTABLE, LBM_ERR_STATE = range(6)
FP64, FP32_DEV, FP32_MIXED = 0, 1, 2
NBR_AUTO, NBR_TABLE, NBR_RANK, NBR_COMPACT = 0, 1, 2, 3
FIELDS = {"Na": 0, "Nb": 1, "phi": 2, "rho": 3, "p": 4, "ux": 5, "uy": 6, "uz": 7}

# Every symbol include/lbm.h declares.
EXPORTS = ("lbm_domain_create", "lbm_step", "lbm_step_timed", "lbm_read_field",
           "lbm_read_pore_field", "lbm_pore_index", "lbm_reduce", "lbm_read_history",
           "lbm_state_save", "lbm_state_load", "lbm_domain_get_info", "lbm_domain_destroy",
           "lbm_prepass_query", "lbm_domain_footprint", "lbm_autotune", "lbm_set_tuning", "lbm_get_tuning",
           "lbm_pool_create", "lbm_pool_admit", "lbm_pool_retire", "lbm_pool_step",
           "lbm_pool_reduce", "lbm_pool_reduce_all", "lbm_pool_get_info", "lbm_pool_set_grid", "lbm_pool_autotune",
           "lbm_pool_destroy", "lbm_pool_set_order", "lbm_pool_set_group_bytes",
           "lbm_set_force", "lbm_run_steady",
           "lbm_morph", "lbm_phase_volume", "lbm_shell_aggregate",
           "lbm_prep_distance", "lbm_prep_distance_noalloc", "lbm_prep_drain", "lbm_prep_relabel", "lbm_prep_mixing_layer",
           "lbm_last_error", "lbm_version")


class LbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("lbm status %d: %s" % (status, msg))
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("periodic", ctypes.c_int32 * 3),
                ("tau_a", ctypes.c_double), ("tau_b", ctypes.c_double),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("force", ctypes.c_double * 3), ("wall_affinity", ctypes.c_double),
                ("bc_z", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("rho_in", ctypes.c_double), ("rho_out", ctypes.c_double),
                ("reduce_every", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("neighbour_mode", ctypes.c_int32), ("inlet_mode", ctypes.c_int32),
                ("flux_in", ctypes.c_double), ("order_rows", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("rho_a", ctypes.c_double),
                ("rho_b", ctypes.c_double)]


class Reduction(ctypes.Structure):
    _fields_ = [("mass_a", ctypes.c_double), ("mass_b", ctypes.c_double),
                ("sw", ctypes.c_double), ("sw_count", ctypes.c_double),
                ("flux", ctypes.c_double * 3), ("flux_a", ctypes.c_double * 3),
                ("flux_b", ctypes.c_double * 3), ("p_a", ctypes.c_double),
                ("p_b", ctypes.c_double), ("ca", ctypes.c_double),
                ("n_pore", ctypes.c_int64), ("step", ctypes.c_int64),
                ("unstable", ctypes.c_int32), ("pad_", ctypes.c_int32)]

    def as_dict(self) -> dict:
        d = {"mass_a": self.mass_a, "mass_b": self.mass_b, "sw": self.sw,
             "sw_count": self.sw_count, "p_a": self.p_a, "p_b": self.p_b, "ca": self.ca,
             "n_pore": self.n_pore, "step": self.step, "unstable": self.unstable}
        for name, arr in (("q", self.flux), ("qa", self.flux_a), ("qb", self.flux_b)):
            for c, ax in enumerate("xyz"):
                d[name + ax] = arr[c]
        return d


class SteadyParams(ctypes.Structure):
    _fields_ = [("ca_target", ctypes.c_double), ("max_factor", ctypes.c_double),
                ("tol", ctypes.c_double), ("relax_steps", ctypes.c_int64),
                ("interval", ctypes.c_int64), ("max_steps", ctypes.c_int64)]


class SteadyResult(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("converged", ctypes.c_int32),
                ("rescales", ctypes.c_int32), ("ca", ctypes.c_double),
                ("delta_ca", ctypes.c_double), ("factor", ctypes.c_double),
                ("force", ctypes.c_double * 3), ("last", Reduction)]

    def as_dict(self) -> dict:
        return {"steps": self.steps, "converged": bool(self.converged),
                "rescales": self.rescales, "ca": self.ca, "delta_ca": self.delta_ca,
                "factor": self.factor, "force": tuple(self.force), "last": self.last.as_dict()}


class MorphParams(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("target_ratio", ctypes.c_double),
                ("band", ctypes.c_double), ("radius", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class MorphResult(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("volume_before", ctypes.c_int64),
                ("volume_unit", ctypes.c_int64), ("volume_after", ctypes.c_int64)]


SHELL_MAX_DELTAS = 32


class ShellParams(ctypes.Structure):
    _fields_ = [("target_ratio", ctypes.c_double), ("band", ctypes.c_double),
                ("radius", ctypes.c_int32), ("max_rounds", ctypes.c_int32),
                ("relax_steps", ctypes.c_int64)]


class ShellResult(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("reached", ctypes.c_int32),
                ("steps", ctypes.c_int64), ("volume_start", ctypes.c_int64),
                ("volume_end", ctypes.c_int64), ("deltas", ctypes.c_double * SHELL_MAX_DELTAS)]


class DrainParams(ctypes.Structure):
    _fields_ = [("target_sw", ctypes.c_double), ("inlet", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


class DrainResult(ctypes.Structure):
    _fields_ = [("radius_sq", ctypes.c_int32), ("max_radius_sq", ctypes.c_int32),
                ("evaluations", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("n_pore", ctypes.c_int64), ("n_nw", ctypes.c_int64), ("sw", ctypes.c_double)]


class Timing(ctypes.Structure):
    _fields_ = [("phase_ms", ctypes.c_double), ("collide_ms", ctypes.c_double),
                ("bc_ms", ctypes.c_double), ("step_ms", ctypes.c_double),
                ("phase_launches", ctypes.c_int64), ("collide_launches", ctypes.c_int64),
                ("bc_launches", ctypes.c_int64), ("collide_parity_ms", ctypes.c_double * 2)]


class Tuning(ctypes.Structure):
    _fields_ = [("phase_block", ctypes.c_int32), ("phase_schedule", ctypes.c_int32),
                ("collide_block", ctypes.c_int32), ("collide_schedule", ctypes.c_int32),
                ("phase_stream", ctypes.c_int32), ("collide_stream", ctypes.c_int32),
                ("phase_wg", ctypes.c_int32), ("collide_wg", ctypes.c_int32),
                ("phase_run", ctypes.c_int32 * 2), ("collide_run", ctypes.c_int32 * 2),
                ("phase_ms", ctypes.c_double), ("collide_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        """Field values; the run lengths as [even, odd] lists."""
        out = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            out[k] = list(v) if isinstance(v, ctypes.Array) else v
        return out


class Info(ctypes.Structure):
    _fields_ = [("n_pore", ctypes.c_int64), ("n_solid_tail", ctypes.c_int64),
                ("ld", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("step", ctypes.c_int64), ("precision", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("neighbour_mode", ctypes.c_int32),
                ("compact_ex_waves", ctypes.c_int32)]


class PoolInfo(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("members", ctypes.c_int32),
                ("chunk_steps", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("step", ctypes.c_int64), ("used_bytes", ctypes.c_int64),
                ("budget_bytes", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("graph_replays", ctypes.c_int64), ("eager_steps", ctypes.c_int64),
                ("order", ctypes.c_int32), ("groups", ctypes.c_int32)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("liblbm.so is not built (%s); run "
                           "`python -m paper_2007_12266_amd.build`" % path)
    L = ctypes.CDLL(path)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    L.lbm_domain_create.argtypes = [ctypes.POINTER(Params), vp, i32, vp, vp, vp, vp,
                                    ctypes.POINTER(Allocator), vp, ctypes.POINTER(vp)]
    L.lbm_step.argtypes = [vp, i64]
    L.lbm_set_force.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.lbm_morph.argtypes = [vp, ctypes.POINTER(MorphParams), ctypes.POINTER(MorphResult)]
    L.lbm_phase_volume.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.lbm_shell_aggregate.argtypes = [vp, ctypes.POINTER(ShellParams),
                                      ctypes.POINTER(ShellResult)]
    L.lbm_run_steady.argtypes = [vp, ctypes.POINTER(SteadyParams), ctypes.POINTER(SteadyResult)]
    L.lbm_step_timed.argtypes = [vp, i64, ctypes.POINTER(Timing)]
    L.lbm_read_field.argtypes = [vp, i32, dp]
    L.lbm_read_pore_field.argtypes = [vp, i32, dp]
    L.lbm_pore_index.argtypes = [vp, vp]
    L.lbm_reduce.argtypes = [vp, ctypes.POINTER(Reduction)]
    L.lbm_read_history.argtypes = [vp, ctypes.POINTER(Reduction), i32, ctypes.POINTER(i32)]
    L.lbm_state_save.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_size_t)]
    L.lbm_state_load.argtypes = [vp, vp, ctypes.c_size_t]
    L.lbm_domain_get_info.argtypes = [vp, ctypes.POINTER(Info)]
    L.lbm_domain_destroy.argtypes = [vp]
    L.lbm_prepass_query.argtypes = [ctypes.POINTER(Params), vp, i32, vp, vp, vp, vp,
                                    ctypes.POINTER(i64), ctypes.POINTER(i64), vp, vp, vp]
    L.lbm_autotune.argtypes = [vp, i32, ctypes.POINTER(Tuning)]
    L.lbm_domain_footprint.argtypes = [ctypes.POINTER(Params), vp, i32, vp, vp, vp, vp,
                                       ctypes.POINTER(i64)]
    L.lbm_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.lbm_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.lbm_pool_create.argtypes = [i64, i32, i32, i32, ctypes.POINTER(Allocator), vp,
                                  ctypes.POINTER(vp)]
    L.lbm_pool_admit.argtypes = [vp, vp, ctypes.POINTER(i32)]
    L.lbm_pool_retire.argtypes = [vp, i32, ctypes.POINTER(vp)]
    L.lbm_pool_step.argtypes = [vp, i64]
    L.lbm_pool_reduce.argtypes = [vp, i32, ctypes.POINTER(Reduction)]
    L.lbm_pool_reduce_all.argtypes = [vp, ctypes.POINTER(Reduction), i32, ctypes.POINTER(i32)]
    L.lbm_pool_get_info.argtypes = [vp, ctypes.POINTER(PoolInfo)]
    L.lbm_pool_set_grid.argtypes = [vp, i32]
    L.lbm_pool_set_order.argtypes = [vp, i32]
    L.lbm_pool_set_group_bytes.argtypes = [vp, i64]
    L.lbm_pool_destroy.argtypes = [vp]
    L.lbm_pool_autotune.argtypes = [vp, i32, ctypes.POINTER(i32)]
    i32p = ctypes.POINTER(i32)
    L.lbm_prep_distance.argtypes = [i32, i32, i32, i32p, i32, vp, vp, vp]
    L.lbm_prep_distance_noalloc.argtypes = [i32, i32, i32, i32p, i32, vp, vp, vp]
    L.lbm_prep_drain.argtypes = [i32, i32, i32, i32p, vp, ctypes.POINTER(DrainParams), vp,
                                 ctypes.POINTER(DrainResult), vp]
    L.lbm_prep_relabel.argtypes = [i32, i32, i32, i32p, vp, i32, vp, vp, ctypes.c_double, i32,
                                   vp, vp]
    L.lbm_prep_mixing_layer.argtypes = [i32, i32, i32, vp, i32, vp, i32, i32, vp, vp]
    L.lbm_last_error.restype = ctypes.c_char_p
    L.lbm_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("lbm_last_error", "lbm_version"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != LBM_OK:
        raise LbmError(status, load_library().lbm_last_error().decode())


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def make_params(problem, precision: int = FP64, reduce_every: int = 0,
                block_size: int = 0, neighbour_mode: int = NBR_AUTO,
                order_rows: int = 0) -> Params:
    """lbm_params of an ``inputs.Problem``."""
    p = Params()
    p.nz, p.ny, p.nx = problem.shape
    for a in range(3):
        p.periodic[a] = 1 if problem.periodic[a] else 0
        p.force[a] = float(problem.force[a])
    p.tau_a, p.tau_b = problem.tau_a, problem.tau_b
    p.alpha, p.beta = problem.alpha, problem.beta
    p.wall_affinity = problem.wall_affinity
    p.bc_z = problem.bc_z
    p.inlet_mode = getattr(problem, "inlet_mode", 0)
    p.flux_in = float(getattr(problem, "flux_in", 0.0))
    p.precision = precision
    p.rho_in, p.rho_out = problem.rho_in, problem.rho_out
    p.rho_a = p.rho_b = 1.0                 # unit density of both fluids (the model's rho0)
    p.reduce_every = reduce_every
    p.block_size = block_size
    p.neighbour_mode = neighbour_mode
    p.order_rows = order_rows
    return p


def _problem_arrays(problem):
    labels = np.ascontiguousarray(problem.labels, dtype=np.int32)
    kind = np.ascontiguousarray(problem.label_kind, dtype=np.int8)
    aff = np.ascontiguousarray(problem.label_affinity, dtype=np.float64)
    vaff = None if problem.voxel_affinity is None else np.ascontiguousarray(
        problem.voxel_affinity, dtype=np.float64)
    iphi = None if problem.init_phi is None else np.ascontiguousarray(
        problem.init_phi, dtype=np.float64)
    return labels, kind, aff, vaff, iphi


def prepass_query(problem, order_rows: int = 0) -> dict:
    """Host-only pre-pass of a problem: pore list, neighbour table [18, N] and phi tail."""
    L = load_library()
    p = make_params(problem, order_rows=order_rows)
    labels, kind, aff, vaff, iphi = _problem_arrays(problem)
    n, t = ctypes.c_int64(), ctypes.c_int64()
    args = (ctypes.byref(p), _ptr(labels), int(aff.size), _ptr(kind), _ptr(aff), _ptr(vaff),
            _ptr(iphi), ctypes.byref(n), ctypes.byref(t))
    _check(L.lbm_prepass_query(*args, None, None, None))
    pv = np.empty(n.value, dtype=np.int64)
    nbr = np.empty((18, n.value), dtype=np.int32)
    tail = np.empty(t.value, dtype=np.float64)
    _check(L.lbm_prepass_query(*args, _ptr(pv), _ptr(nbr), _ptr(tail)))
    return {"n_pore": n.value, "n_tail": t.value, "pore_voxel": pv, "nbr": nbr,
            "tail_phi": tail}


def footprint(problem, precision: int = FP64, neighbour_mode: int = NBR_AUTO,
              order_rows: int = 0) -> int:
    """Device bytes a Domain of this problem would allocate (host-only pre-pass)."""
    L = load_library()
    p = make_params(problem, precision, neighbour_mode=neighbour_mode, order_rows=order_rows)
    labels, kind, aff, vaff, iphi = _problem_arrays(problem)
    b = ctypes.c_int64()
    _check(L.lbm_domain_footprint(ctypes.byref(p), _ptr(labels), int(aff.size), _ptr(kind),
                                  _ptr(aff), _ptr(vaff), _ptr(iphi), ctypes.byref(b)))
    return b.value


class _TorchAllocator:
    """Device memory from PyTorch's caching allocator on a given stream."""

    def __init__(self, stream):
        import torch
        self.torch = torch
        self.device = torch.cuda.current_device()
        self.stream = stream
        self._alloc = ALLOC_FN(self._do_alloc)
        self._free = FREE_FN(self._do_free)
        self.struct = Allocator(self._alloc, self._free, None)

    def _do_alloc(self, nbytes, ctx):
        try:
            return int(self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                               self.stream))
        except Exception:
            return None

    def _do_free(self, ptr, ctx):
        self.torch.cuda.caching_allocator_delete(ptr)


class Domain:
    """One colour-LBM domain on the GPU (wraps lbm_domain*)."""

    def __init__(self, problem, precision: int = FP64, reduce_every: int = 0,
                 block_size: int = 0, allocator: str = "torch", stream=None,
                 neighbour_mode: int = NBR_AUTO, order_rows: int = 0):
        L = load_library()
        self.problem = problem
        self.shape = problem.shape
        p = make_params(problem, precision, reduce_every, block_size, neighbour_mode, order_rows)
        self.params = p
        labels, kind, aff, vaff, iphi = _problem_arrays(problem)
        self._torch_alloc = None
        stream_handle = None
        if stream is not None:
            stream_handle = ctypes.c_void_p(stream)
        if allocator == "torch":
            import torch
            s = torch.cuda.current_stream() if stream is None else None
            handle = stream if stream is not None else s.cuda_stream
            self._torch_alloc = _TorchAllocator(handle)
            stream_handle = ctypes.c_void_p(handle)
        h = ctypes.c_void_p()
        _check(L.lbm_domain_create(ctypes.byref(p), _ptr(labels), int(aff.size), _ptr(kind),
                                   _ptr(aff), _ptr(vaff), _ptr(iphi),
                                   ctypes.byref(self._torch_alloc.struct)
                                   if self._torch_alloc else None,
                                   stream_handle, ctypes.byref(h)))
        self.handle = h
        info = self.info()
        self.n_pore = info["n_pore"]

    def close(self):
        if getattr(self, "handle", None):
            _check(load_library().lbm_domain_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int):
        _check(load_library().lbm_step(self.handle, int(n)))
        return self

    def step_timed(self, n: int) -> dict:
        t = Timing()
        _check(load_library().lbm_step_timed(self.handle, int(n), ctypes.byref(t)))
        out = {k: getattr(t, k) for k, _ in Timing._fields_}
        out["collide_parity_ms"] = list(out["collide_parity_ms"])   # [even, odd]
        return out

    def field(self, name: str) -> np.ndarray:
        out = np.empty(self.shape, dtype=np.float64)
        _check(load_library().lbm_read_field(self.handle, FIELDS[name], _ptr(out)))
        return out

    def pore_field(self, name: str) -> np.ndarray:
        out = np.empty(self.n_pore, dtype=np.float64)
        _check(load_library().lbm_read_pore_field(self.handle, FIELDS[name], _ptr(out)))
        return out

    def pore_index(self) -> np.ndarray:
        out = np.empty(self.n_pore, dtype=np.int64)
        _check(load_library().lbm_pore_index(self.handle, _ptr(out)))
        return out

    def fields(self) -> dict:
        return {k: self.field(k) for k in FIELDS}

    def reduce(self) -> dict:
        r = Reduction()
        _check(load_library().lbm_reduce(self.handle, ctypes.byref(r)))
        return r.as_dict()

    def history(self, max_count: int = 4096) -> list:
        arr = (Reduction * max_count)()
        n = ctypes.c_int32()
        _check(load_library().lbm_read_history(self.handle, arr, max_count, ctypes.byref(n)))
        return [arr[k].as_dict() for k in range(n.value)]

    def save(self) -> bytes:
        L = load_library()
        n = ctypes.c_size_t()
        _check(L.lbm_state_save(self.handle, None, ctypes.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)        # no zero fill before the library writes
        _check(L.lbm_state_save(self.handle, _ptr(buf), ctypes.byref(n)))
        return buf.tobytes()

    def load(self, blob):
        """Restore a state from lbm_state_save's bytes (bytes, bytearray or a uint8 array); the
        library reads the caller's buffer in place."""
        if isinstance(blob, bytes):
            ptr = ctypes.cast(ctypes.c_char_p(blob), ctypes.c_void_p)
        else:
            arr = np.frombuffer(blob, dtype=np.uint8)
            ptr = ctypes.c_void_p(arr.ctypes.data)
        _check(load_library().lbm_state_load(self.handle, ptr, len(blob)))
        return self

    def autotune(self, trial_steps: int = 10) -> dict:
        t = Tuning()
        _check(load_library().lbm_autotune(self.handle, int(trial_steps), ctypes.byref(t)))
        return t.as_dict()

    def set_force(self, force):
        """Replace the body force from the next step on."""
        f = (ctypes.c_double * 3)(*[float(x) for x in force])
        _check(load_library().lbm_set_force(self.handle, f))

    def run_steady(self, ca_target: float = 0.0, relax_steps: int = 0, interval: int = 1000,
                   tol: float = 1e-3, max_steps: int = 100000, max_factor: float = 2.0) -> dict:
        """One steady-state point: relax, rescale F towards Ca* (capped), then step in blocks of
        `interval` until |dCa|/Ca < tol or max_steps (lbm_run_steady)."""
        sp = SteadyParams(float(ca_target), float(max_factor), float(tol), int(relax_steps),
                          int(interval), int(max_steps))
        out = SteadyResult()
        _check(load_library().lbm_run_steady(self.handle, ctypes.byref(sp), ctypes.byref(out)))
        return out.as_dict()

    def morph(self, delta: float = 0.0, target_ratio: float = 0.0, radius: int = 6,
              band: float = 2.5) -> dict:
        """One morphological change of fluid a by delta voxels (or towards a volume ratio)."""
        mp = MorphParams(float(delta), float(target_ratio), float(band), int(radius), 0)
        r = MorphResult()
        _check(load_library().lbm_morph(self.handle, ctypes.byref(mp), ctypes.byref(r)))
        return {"delta": r.delta, "volume_before": r.volume_before,
                "volume_unit": r.volume_unit, "volume_after": r.volume_after}

    def phase_volume(self) -> int:
        """Pore voxels with phi > 0 (the volume of fluid a)."""
        v = ctypes.c_int64()
        _check(load_library().lbm_phase_volume(self.handle, ctypes.byref(v)))
        return v.value

    def shell_aggregate(self, target_ratio: float, relax_steps: int = 1000,
                        max_rounds: int = 8, radius: int = 6, band: float = 2.5) -> dict:
        """The shell aggregation protocol: morph and relax until the volume of fluid a has
        changed by target_ratio (lbm_shell_aggregate)."""
        sp = ShellParams(float(target_ratio), float(band), int(radius), int(max_rounds),
                         int(relax_steps))
        r = ShellResult()
        _check(load_library().lbm_shell_aggregate(self.handle, ctypes.byref(sp),
                                                  ctypes.byref(r)))
        return {"rounds": r.rounds, "reached": bool(r.reached), "steps": r.steps,
                "volume_start": r.volume_start, "volume_end": r.volume_end,
                "deltas": [r.deltas[k] for k in range(min(r.rounds, SHELL_MAX_DELTAS))]}

    def tuning(self) -> dict:
        t = Tuning()
        _check(load_library().lbm_get_tuning(self.handle, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        """Change fields of the current launch configuration (phase_run and collide_run take an
        [even, odd] pair)."""
        t = Tuning()
        _check(load_library().lbm_get_tuning(self.handle, ctypes.byref(t)))
        for k, v in kw.items():
            if k in ("phase_run", "collide_run"):
                v = (ctypes.c_int32 * 2)(*(int(x) for x in v))
            setattr(t, k, v)
        _check(load_library().lbm_set_tuning(self.handle, ctypes.byref(t)))
        return self

    def info(self) -> dict:
        i = Info()
        _check(load_library().lbm_domain_get_info(self.handle, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in Info._fields_}


class Pool:
    """Many domains stepped together by one launch per kernel per step (wraps lbm_pool*)."""

    def __init__(self, budget_bytes: int, precision: int = FP32_DEV, max_slots: int = 64,
                 chunk_steps: int = 100, stream=None, allocator: str = "torch"):
        L = load_library()
        h = ctypes.c_void_p()
        # The pool's own tables come from PyTorch's caching allocator (or hipMalloc).
        self._torch_alloc = None
        if allocator == "torch":
            import torch
            self._torch_alloc = _TorchAllocator(stream if stream is not None
                                                else torch.cuda.current_stream().cuda_stream)
        _check(L.lbm_pool_create(int(budget_bytes), int(precision), int(max_slots),
                                 int(chunk_steps),
                                 ctypes.byref(self._torch_alloc.struct) if self._torch_alloc
                                 else None,
                                 None if stream is None else ctypes.c_void_p(stream),
                                 ctypes.byref(h)))
        self.handle = h
        self.max_slots = max_slots
        self.members = {}

    def admit(self, dom: Domain) -> int:
        slot = ctypes.c_int32()
        _check(load_library().lbm_pool_admit(self.handle, dom.handle, ctypes.byref(slot)))
        self.members[slot.value] = dom
        return slot.value

    def retire(self, slot: int) -> Domain:
        h = ctypes.c_void_p()
        _check(load_library().lbm_pool_retire(self.handle, int(slot), ctypes.byref(h)))
        dom = self.members.pop(slot)
        assert h.value == dom.handle.value, "pool returned another domain"
        return dom

    def step(self, n: int):
        _check(load_library().lbm_pool_step(self.handle, int(n)))
        return self

    def reduce_slot(self, slot: int) -> dict:
        """Reduction of the member of one slot."""
        r = Reduction()
        _check(load_library().lbm_pool_reduce(self.handle, int(slot), ctypes.byref(r)))
        return r.as_dict()

    def reduce(self) -> dict:
        """Reductions of every member (one batched launch), keyed by slot."""
        arr = (Reduction * self.max_slots)()
        n = ctypes.c_int32()
        _check(load_library().lbm_pool_reduce_all(self.handle, arr, self.max_slots,
                                                  ctypes.byref(n)))
        return {s: arr[s].as_dict() for s in range(n.value) if s in self.members}

    def info(self) -> dict:
        i = PoolInfo()
        _check(load_library().lbm_pool_get_info(self.handle, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in PoolInfo._fields_}

    def autotune(self, trial_steps: int = 10) -> int:
        g = ctypes.c_int32()
        _check(load_library().lbm_pool_autotune(self.handle, int(trial_steps), ctypes.byref(g)))
        return g.value

    def set_grid(self, grid: int):
        _check(load_library().lbm_pool_set_grid(self.handle, int(grid)))
        return self

    def set_order(self, order: int):
        """0: tiles in launch order; 1: XCD-aware runs of tiles."""
        _check(load_library().lbm_pool_set_order(self.handle, int(order)))
        return self

    def set_group_bytes(self, group_bytes: int):
        """Captured chunks run the members in cache groups of at most group_bytes of device
        memory each, one group after the other (0: all members together)."""
        _check(load_library().lbm_pool_set_group_bytes(self.handle, int(group_bytes)))
        return self

    def close(self):
        if getattr(self, "handle", None):
            load_library().lbm_pool_destroy(self.handle)
            self.handle = None
            self.members = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- Image pre-processing (lbm_prep_*): dense [z, y, x] host arrays in and out. -------------

def _periodic3(periodic):
    return (ctypes.c_int32 * 3)(*[1 if p else 0 for p in periodic])


def _stream_handle(stream):
    return None if stream is None else ctypes.c_void_p(stream)


def prep_distance(feature: np.ndarray, periodic=(False, False, False), wall_axes: int = 0,
                  stream=None) -> np.ndarray:
    """Squared Euclidean distance to the nearest nonzero voxel of feature (int32, -1 where
    there is none); wall_axes bit a adds wall planes outside non-periodic axis a."""
    f = np.ascontiguousarray(feature, dtype=np.uint8)
    nz, ny, nx = f.shape
    out = np.empty(f.shape, dtype=np.int32)
    _check(load_library().lbm_prep_distance(nx, ny, nz, _periodic3(periodic), int(wall_axes),
                                            _ptr(f), _ptr(out), _stream_handle(stream)))
    return out


def prep_distance_noalloc(feature, out, periodic=(False, False, False), wall_axes: int = 0,
                          stream=None):
    """The allocation-free transform on device tensors: feature (uint8, [nz, ny, nx], on the
    GPU) in, out (int32, same shape, on the GPU) written asynchronously on `stream` (a
    hipStream_t handle; None: the null stream)."""
    nz, ny, nx = feature.shape
    assert tuple(out.shape) == (nz, ny, nx) and feature.is_contiguous() and out.is_contiguous()
    _check(load_library().lbm_prep_distance_noalloc(
        nx, ny, nz, _periodic3(periodic), int(wall_axes), ctypes.c_void_p(feature.data_ptr()),
        ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def prep_drain(pore: np.ndarray, periodic=(False, False, False), target_sw: float = 0.5,
               inlet: bool = False, stream=None):
    """Morphological drainage to a target water saturation; returns (nw mask, result dict)."""
    m = np.ascontiguousarray(pore, dtype=np.uint8)
    nz, ny, nx = m.shape
    nw = np.empty(m.shape, dtype=np.uint8)
    dp = DrainParams(float(target_sw), 1 if inlet else 0, 0)
    r = DrainResult()
    _check(load_library().lbm_prep_drain(nx, ny, nz, _periodic3(periodic), _ptr(m),
                                         ctypes.byref(dp), _ptr(nw), ctypes.byref(r),
                                         _stream_handle(stream)))
    return nw.astype(bool), {"k": r.radius_sq, "kmax": r.max_radius_sq,
                             "evaluations": r.evaluations, "n_pore": r.n_pore,
                             "n_nw": r.n_nw, "sw": r.sw}


def prep_relabel(labels: np.ndarray, label_kind: np.ndarray, nw: np.ndarray,
                 periodic=(False, False, False), dist: float = 2.0, new_label: int = 0,
                 stream=None) -> np.ndarray:
    """Solid voxels within dist of the non-wetting mask take new_label."""
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    kind = np.ascontiguousarray(label_kind, dtype=np.int8)
    m = np.ascontiguousarray(nw, dtype=np.uint8)
    if m.shape != lab.shape:
        raise ValueError("nw and labels differ in shape")
    nz, ny, nx = lab.shape
    out = np.empty(lab.shape, dtype=np.int32)
    _check(load_library().lbm_prep_relabel(nx, ny, nz, _periodic3(periodic), _ptr(lab),
                                           len(kind), _ptr(kind), _ptr(m), float(dist),
                                           int(new_label), _ptr(out), _stream_handle(stream)))
    return out


def prep_mixing_layer(labels: np.ndarray, label_kind: np.ndarray, nmix: int, pore_label: int,
                      stream=None) -> np.ndarray:
    """Open the first and last nmix z planes where the opposite face is pore."""
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    kind = np.ascontiguousarray(label_kind, dtype=np.int8)
    nz, ny, nx = lab.shape
    out = np.empty(lab.shape, dtype=np.int32)
    _check(load_library().lbm_prep_mixing_layer(nx, ny, nz, _ptr(lab), len(kind), _ptr(kind),
                                                int(nmix), int(pore_label), _ptr(out),
                                                _stream_handle(stream)))
    return out
