"""FP64 CPU oracle for the 3D FD-LB update -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check (``__graft_entry__.smoke``) and
the CPU-baseline leg of ``bench.py`` may import this package.  The product
library never calls it, and it never calls the product library: the two share
no code.  What the C file computes, and which passage of the paper each part
follows, is documented in ``lbm3d_oracle.c``.

Pins: every function here is checked in ``tests/test_oracle_*.py`` against
facts the paper and the mathematics fix (closed-form equilibrium moments,
conservation on periodic boxes, uniform states, cubic symmetry, quasi-1D
reduction, exact Riemann solutions, Rankine-Hugoniot numbers printed in the
paper, the acoustic speed).  No function is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm3d_oracle.c")
_LIB = os.path.join(_HERE, "liblbm3d_oracle.so")

NV = 15
PERIODIC, OUTFLOW, INFLOW, REFLECT = 0, 1, 2, 3
NO_DISSIPATION = 1
UPWIND2 = 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
               "-std=c11", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("c1", ctypes.c_double), ("c2", ctypes.c_double), ("eta0", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("tau", ctypes.c_double), ("dt", ctypes.c_double), ("dx", ctypes.c_double),
        ("bc", ctypes.c_int32 * 6),
        ("inflow", (ctypes.c_double * 5) * 6),
        ("flags", ctypes.c_uint32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        D = ctypes.POINTER(ctypes.c_double)
        lib.orc_create.restype = P
        lib.orc_create.argtypes = [ctypes.POINTER(_Params)]
        lib.orc_destroy.argtypes = [P]
        lib.orc_init.argtypes = [P, D, D, D, D, D]
        lib.orc_step.argtypes = [P, ctypes.c_int64]
        lib.orc_moments.argtypes = [P, D, D, D, D, D]
        lib.orc_conserved.argtypes = [P, D]
        lib.orc_get_f.argtypes = [P, D]
        lib.orc_set_f.argtypes = [P, D]
        lib.orc_get_f_padded.argtypes = [P, D]
        lib.orc_steps_done.restype = ctypes.c_int64
        lib.orc_steps_done.argtypes = [P]
        lib.orc_nonphysical.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
        lib.orc_velocities.argtypes = [ctypes.c_double] * 3 + [D, D]
        lib.orc_equilibrium.argtypes = [ctypes.c_double] * 9 + [D]
        lib.orc_moments_of.argtypes = [ctypes.c_double] * 4 + [D, D]
        lib.orc_minmod.restype = ctypes.c_double
        lib.orc_minmod.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.orc_set_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> int:
    """Set the OpenMP thread count of the step loop; returns the count in use."""
    return int(_load().orc_set_threads(int(n)))


def velocities(c1: float, c2: float, eta0: float):
    v = np.zeros((NV, 3))
    eta = np.zeros(NV)
    _load().orc_velocities(c1, c2, eta0, _dp(v), _dp(eta))
    return v, eta


def equilibrium(c1, c2, eta0, gamma, rho, ux, uy, uz, T) -> np.ndarray:
    out = np.zeros(NV)
    _load().orc_equilibrium(c1, c2, eta0, gamma, rho, ux, uy, uz, T, _dp(out))
    return out


def moments_of(c1, c2, eta0, gamma, f) -> np.ndarray:
    """(rho, ux, uy, uz, T) of one node's 15 distributions."""
    f = _c64(f)
    q = np.zeros(5)
    _load().orc_moments_of(c1, c2, eta0, gamma, _dp(f), _dp(q))
    return q


def minmod(x: float, y: float) -> float:
    return float(_load().orc_minmod(x, y))


class Oracle:
    """One FP64 solve.  ``params`` is the plain dict produced by
    ``paper_1010_4135_amd.inputs`` (grid, model constants, boundary kinds)."""

    def __init__(self, params: dict):
        lib = _load()
        p = _Params()
        p.nx, p.ny, p.nz = (int(v) for v in params["grid"])
        p.c1, p.c2, p.eta0 = params["c1"], params["c2"], params["eta0"]
        p.gamma = params["gamma"]
        p.tau, p.dt, p.dx = params["tau"], params["dt"], params["dx"]
        for k in range(6):
            p.bc[k] = int(params["bc"][k])
        infl = params.get("inflow")
        if infl is not None:
            for k in range(6):
                for m in range(5):
                    p.inflow[k][m] = float(infl[k][m])
        p.flags = int(params.get("flags", 0))
        self.shape = (p.nz, p.ny, p.nx)
        self._lib = lib
        self._h = lib.orc_create(ctypes.byref(p))
        if not self._h:
            raise MemoryError("oracle: create failed")

    def close(self):
        if self._h:
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, rho, ux, uy, uz, p):
        arrs = [_c64(a).reshape(self.shape) for a in (rho, ux, uy, uz, p)]
        self._lib.orc_init(self._h, *[_dp(a) for a in arrs])

    def step(self, n: int = 1):
        self._lib.orc_step(self._h, int(n))

    @property
    def steps_done(self) -> int:
        return int(self._lib.orc_steps_done(self._h))

    def nonphysical(self):
        """(node-steps with rho <= 0, node-steps with T <= 0) since init,
        counted at the state each step starts from."""
        out = (ctypes.c_int64 * 2)()
        self._lib.orc_nonphysical(self._h, out)
        return int(out[0]), int(out[1])

    def moments(self):
        """(rho, ux, uy, uz, p) arrays of shape (nz, ny, nx)."""
        out = [np.zeros(self.shape) for _ in range(5)]
        self._lib.orc_moments(self._h, *[_dp(a) for a in out])
        return tuple(out)

    def conserved(self) -> np.ndarray:
        out = np.zeros(5)
        self._lib.orc_conserved(self._h, _dp(out))
        return out

    def get_f(self) -> np.ndarray:
        out = np.zeros((NV,) + self.shape)
        self._lib.orc_get_f(self._h, _dp(out))
        return out

    def get_f_padded(self) -> np.ndarray:
        nz, ny, nx = self.shape
        out = np.zeros((NV, nz + 4, ny + 4, nx + 4))
        self._lib.orc_get_f_padded(self._h, _dp(out))
        return out

    def set_f(self, f):
        f = _c64(f).reshape((NV,) + self.shape)
        self._lib.orc_set_f(self._h, _dp(f))
