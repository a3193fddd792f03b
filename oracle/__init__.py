"""Plain FP64 CPU oracle of the colour-LBM time step (arXiv 2007.12266, Color Lattice-Boltzmann
Model and Modeling Wetting sections).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU-baseline leg are the
only callers. The product path never imports this package; it shares no code with it.

The arithmetic lives in ``colorlbm_oracle.c`` (dense grid, explicit 19x19 moment matrix, push
streaming into a second buffer, OpenMP over z). This module only marshals numpy arrays.
``brute.py`` is a second, independent per-voxel NumPy implementation used to pin the C code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "colorlbm_oracle.c")
_LIB = os.path.join(_HERE, "libcolorlbm_oracle.so")

# Field order of ora_reduce's output vector.
REDUCE_KEYS = ("mass_a", "mass_b", "sw", "sw_count", "qx", "qy", "qz", "qax", "qay", "qaz",
               "qbx", "qby", "qbz", "p_a", "p_b", "ca", "n_pore", "unstable")


class OraParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("periodic", ctypes.c_int32 * 3),
                ("tau_a", ctypes.c_double), ("tau_b", ctypes.c_double),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("force", ctypes.c_double * 3), ("wall_affinity", ctypes.c_double),
                ("bc_z", ctypes.c_int32), ("inlet_mode", ctypes.c_int32),
                ("rho_in", ctypes.c_double), ("rho_out", ctypes.c_double),
                ("flux_in", ctypes.c_double), ("c_min", ctypes.c_double)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c99",
                               "-D_DEFAULT_SOURCE", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        up = ctypes.POINTER(ctypes.c_uint8)
        pp = ctypes.POINTER(OraParams)
        L.ora_moment_basis.argtypes = [dp, dp, dp]
        L.ora_velocity_set.argtypes = [ctypes.POINTER(ctypes.c_int32), dp, dp,
                                       ctypes.POINTER(ctypes.c_int32)]
        L.ora_collide.argtypes = [pp, dp, ctypes.c_double, ctypes.c_double, dp, dp, dp, dp, dp]
        L.ora_init.argtypes = [pp, up, dp, dp, dp, dp]
        L.ora_run.argtypes = [pp, up, dp, dp, dp, dp, ctypes.c_int]
        L.ora_run.restype = ctypes.c_int
        L.ora_fields.argtypes = [pp, up, dp, dp, dp] + [dp] * 8
        L.ora_reduce.argtypes = [pp, up, dp, dp, dp, dp]
        L.ora_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().ora_threads())


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(shape, periodic=(True, True, True), tau_a=0.7, tau_b=0.7, alpha=0.005,
                beta=0.95, force=(0.0, 0.0, 0.0), wall_affinity=0.0, bc_z=0, rho_in=1.0,
                rho_out=1.0, inlet_mode=0, flux_in=0.0, c_min=1e-10) -> OraParams:
    nz, ny, nx = shape
    p = OraParams()
    p.nx, p.ny, p.nz = nx, ny, nz
    for a in range(3):
        p.periodic[a] = 1 if periodic[a] else 0
        p.force[a] = float(force[a])
    p.tau_a, p.tau_b, p.alpha, p.beta = tau_a, tau_b, alpha, beta
    p.wall_affinity = wall_affinity
    p.bc_z = bc_z
    p.rho_in, p.rho_out = rho_in, rho_out
    p.inlet_mode, p.flux_in = inlet_mode, float(flux_in)
    p.c_min = float(c_min)
    return p


def params_of(problem) -> OraParams:
    """Oracle parameters of an ``inputs.Problem``."""
    return make_params(problem.shape, problem.periodic, problem.tau_a, problem.tau_b,
                       problem.alpha, problem.beta, problem.force, problem.wall_affinity,
                       problem.bc_z, problem.rho_in, problem.rho_out, problem.inlet_mode,
                       problem.flux_in)


def moment_basis():
    M = np.zeros(19 * 19)
    Minv = np.zeros(19 * 19)
    D = np.zeros(19)
    lib().ora_moment_basis(_d(M), _d(Minv), _d(D))
    return M.reshape(19, 19), Minv.reshape(19, 19), D


def velocity_set():
    xi = np.zeros(57, dtype=np.int32)
    t = np.zeros(19)
    w = np.zeros(7)
    opp = np.zeros(19, dtype=np.int32)
    lib().ora_velocity_set(xi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _d(t), _d(w),
                           opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return xi.reshape(19, 3), t, w, opp


def collide(params: OraParams, f, Na, Nb, C):
    """One voxel's collision + recolouring: returns (f*, A*, B*, u)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    C = np.ascontiguousarray(C, dtype=np.float64)
    fs = np.zeros(19)
    As = np.zeros(7)
    Bs = np.zeros(7)
    u = np.zeros(3)
    lib().ora_collide(ctypes.byref(params), _d(f), float(Na), float(Nb), _d(C), _d(fs), _d(As),
                      _d(Bs), _d(u))
    return fs, As, Bs, u


class State:
    """Dense oracle state: f [19, nz, ny, nx], A and B [7, nz, ny, nx]."""

    def __init__(self, params: OraParams, solid, phi_s):
        self.params = params
        self.shape = (params.nz, params.ny, params.nx)
        self.solid = np.ascontiguousarray(solid, dtype=np.uint8)
        self.phi_s = np.ascontiguousarray(phi_s, dtype=np.float64)
        self.f = np.zeros((19,) + self.shape)
        self.A = np.zeros((7,) + self.shape)
        self.B = np.zeros((7,) + self.shape)
        self.steps = 0

    def _u8(self):
        return self.solid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))

    def init(self, phi0):
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64)
        lib().ora_init(ctypes.byref(self.params), self._u8(), _d(phi0), _d(self.f), _d(self.A),
                       _d(self.B))
        self.steps = 0
        return self

    def run(self, nsteps: int):
        rc = lib().ora_run(ctypes.byref(self.params), self._u8(), _d(self.phi_s), _d(self.f),
                           _d(self.A), _d(self.B), int(nsteps))
        if rc != 0:
            raise MemoryError("oracle: allocation failed")
        self.steps += nsteps
        return self

    def fields(self) -> dict:
        out = {k: np.zeros(self.shape) for k in ("Na", "Nb", "phi", "rho", "p", "ux", "uy", "uz")}
        lib().ora_fields(ctypes.byref(self.params), self._u8(), _d(self.f), _d(self.A),
                         _d(self.B), *[_d(out[k]) for k in
                                       ("Na", "Nb", "phi", "rho", "p", "ux", "uy", "uz")])
        return out

    def reduce(self) -> dict:
        out = np.zeros(len(REDUCE_KEYS))
        lib().ora_reduce(ctypes.byref(self.params), self._u8(), _d(self.f), _d(self.A),
                         _d(self.B), _d(out))
        return dict(zip(REDUCE_KEYS, out.tolist()))


def state_for(problem) -> State:
    """Oracle state initialised from an ``inputs.Problem``."""
    return State(params_of(problem), problem.solid_mask(), problem.solid_affinity()).init(
        problem.phase0())
