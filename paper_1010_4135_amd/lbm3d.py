"""ctypes binding of the lbm3d C ABI (include/lbm3d.h).

Argument marshalling only: every step of the solver runs in the HIP library
``liblbm3d.so`` built in-tree by ``paper_1010_4135_amd.build``.  Importing
this module fails loudly if that library is missing; there is no CPU or
PyTorch fallback.  Function names match the C entry points; ``Solver`` and
``Server`` are small convenience wrappers over them.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm3d.so")

OK, E_INVAL, E_UNSTABLE, E_NOMEM, E_DEVICE, E_STATE, E_NONFINITE, E_NOTFOUND, E_CANCELLED = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
FP64, FP32, FP32_T64 = 0, 1, 2
PERIODIC, OUTFLOW, INFLOW, REFLECT = 0, 1, 2, 3
NO_DISSIPATION, UPWIND2, CHECK_STABILITY, VELOCITY_MAJOR = 1, 2, 4, 8
HEALTH_NONFINITE, HEALTH_RHO_NONPOS, HEALTH_T_NONPOS = 1, 2, 4
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp32_t64": FP32_T64}
NV = 15


class LbmError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {lbm3d_strerror(code)} ({code})")


class lbm3d_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("c1", ctypes.c_double), ("c2", ctypes.c_double), ("eta0", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("tau", ctypes.c_double), ("dt", ctypes.c_double), ("dx", ctypes.c_double),
        ("bc", ctypes.c_int32 * 6),
        ("inflow", (ctypes.c_double * 5) * 6),
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
    ]


class lbm3d_timing(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("steps", ctypes.c_int64),
                ("health", ctypes.c_uint32)]


class lbm3d_server_counters(ctypes.Structure):
    _fields_ = [("ticks", ctypes.c_int64), ("rebuilds", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("evicted", ctypes.c_int64), ("wall_s", ctypes.c_double),
                ("busy_s", ctypes.c_double), ("admit_s", ctypes.c_double), ("plan_s", ctypes.c_double),
                ("finish_s", ctypes.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"lbm3d HIP library not built: {LIB_PATH} is missing "
                          "(run __graft_entry__.build() or python -m paper_1010_4135_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
    D = ctypes.POINTER(ctypes.c_double)
    PP = ctypes.POINTER(lbm3d_params)
    sig = {
        "lbm3d_version": (ctypes.c_char_p, []),
        "lbm3d_strerror": (ctypes.c_char_p, [I32]),
        "lbm3d_device_count": (I32, [ctypes.POINTER(I32)]),
        "lbm3d_footprint": (I32, [PP, ctypes.POINTER(SZ)]),
        "lbm3d_create": (I32, [PP, ctypes.POINTER(P)]),
        "lbm3d_destroy": (I32, [P]),
        "lbm3d_set_stream": (I32, [P, P]),
        "lbm3d_init": (I32, [P, D, D, D, D, D]),
        "lbm3d_step": (I32, [P, I64]),
        "lbm3d_step_timed": (I32, [P, I64, D]),
        "lbm3d_step_profiled": (I32, [P, I64, D, D]),
        "lbm3d_set_tile": (I32, [P, I32, I32]),
        "lbm3d_tune": (I32, [P, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "lbm3d_tune_save": (I32, [ctypes.c_char_p]),
        "lbm3d_tune_load": (I32, [ctypes.c_char_p]),
        "lbm3d_batch_tune": (I32, [ctypes.POINTER(P), I32, I32, ctypes.POINTER(I32)]),
        "lbm3d_batch_set_depth": (I32, [I32, I32]),
        "lbm3d_get_tile": (I32, [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "lbm3d_set_streaming": (I32, [P, I32]),
        "lbm3d_get_streaming": (I32, [P, ctypes.POINTER(I32)]),
        "lbm3d_sync": (I32, [P]),
        "lbm3d_stream_copy_rate": (I32, [I64, I32, D]),
        "lbm3d_admit": (I32, [PP, D, D, D, D, D, D]),
        "lbm3d_stability": (I32, [PP, D, I32, ctypes.c_double, ctypes.c_double, I32, ctypes.c_double, D, D]),
        "lbm3d_moments": (I32, [P, D, D, D, D, D]),
        "lbm3d_conserved": (I32, [P, D]),
        "lbm3d_status": (I32, [P, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(I64)]),
        "lbm3d_get_f": (I32, [P, P, SZ]),
        "lbm3d_poison_next": (I32, [P]),
        "lbm3d_set_f": (I32, [P, P, SZ]),
        "lbm3d_batch_step": (I32, [ctypes.POINTER(P), I32, ctypes.POINTER(I64)]),
        "lbm3d_batch_step_noalloc": (I32, [ctypes.POINTER(P), I32, ctypes.POINTER(I64)]),
        "lbm3d_batch_plan": (I32, [PP, I32, I32, I32, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32),
                                   ctypes.POINTER(I32), I64, ctypes.POINTER(I32)]),
        "lbm3d_server_create": (I32, [SZ, I32, ctypes.POINTER(P)]),
        "lbm3d_server_set_tick": (I32, [P, I64]),
        "lbm3d_server_submit": (I32, [P, PP, D, D, D, D, D, I64, ctypes.POINTER(U64)]),
        "lbm3d_server_poll": (I32, [P, U64, ctypes.POINTER(I32)]),
        "lbm3d_server_wait": (I32, [P, U64, D, D, D, D, D, ctypes.POINTER(lbm3d_timing)]),
        "lbm3d_server_cancel": (I32, [P, U64]),
        "lbm3d_server_stats": (I32, [P, ctypes.POINTER(lbm3d_server_counters)]),
        "lbm3d_server_destroy": (I32, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, where: str):
    if rc != OK:
        raise LbmError(rc, where)


def make_params(d: dict) -> lbm3d_params:
    """lbm3d_params from the plain dict used by paper_1010_4135_amd.inputs."""
    p = lbm3d_params()
    p.nx, p.ny, p.nz = (int(v) for v in d["grid"])
    p.c1, p.c2, p.eta0 = float(d["c1"]), float(d["c2"]), float(d["eta0"])
    p.gamma = float(d["gamma"])
    p.tau, p.dt, p.dx = float(d["tau"]), float(d["dt"]), float(d["dx"])
    for k in range(6):
        p.bc[k] = int(d["bc"][k])
    infl = d.get("inflow")
    if infl is not None:
        for k in range(6):
            for m in range(5):
                p.inflow[k][m] = float(infl[k][m])
    prec = d.get("precision", "fp64")
    p.precision = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    p.flags = int(d.get("flags", 0))
    return p


def _params(p):
    return p if isinstance(p, lbm3d_params) else make_params(p)


# ---------------------------------------------------------------- C names --
def lbm3d_version() -> str:
    return _lib.lbm3d_version().decode()


def lbm3d_strerror(code: int) -> str:
    return _lib.lbm3d_strerror(int(code)).decode()


def lbm3d_device_count() -> int:
    c = ctypes.c_int32(0)
    _check(_lib.lbm3d_device_count(ctypes.byref(c)), "lbm3d_device_count")
    return c.value


def lbm3d_footprint(params) -> int:
    b = ctypes.c_size_t(0)
    _check(_lib.lbm3d_footprint(ctypes.byref(_params(params)), ctypes.byref(b)), "lbm3d_footprint")
    return b.value


def lbm3d_create(params):
    h = ctypes.c_void_p()
    _check(_lib.lbm3d_create(ctypes.byref(_params(params)), ctypes.byref(h)), "lbm3d_create")
    return h


def lbm3d_destroy(h):
    _check(_lib.lbm3d_destroy(h), "lbm3d_destroy")


def lbm3d_set_stream(h, stream_ptr):
    _check(_lib.lbm3d_set_stream(h, ctypes.c_void_p(stream_ptr) if stream_ptr else None), "lbm3d_set_stream")


def _fields5(fields, n):
    out = []
    for a in fields:
        a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
        if a.size != n:
            raise ValueError(f"field has {a.size} values, expected {n}")
        out.append(a)
    return out


def lbm3d_init(h, shape, rho, ux, uy, uz, p):
    n = int(np.prod(shape))
    arrs = _fields5((rho, ux, uy, uz, p), n)
    _check(_lib.lbm3d_init(h, *[_dp(a) for a in arrs]), "lbm3d_init")


def lbm3d_step(h, nsteps: int):
    _check(_lib.lbm3d_step(h, int(nsteps)), "lbm3d_step")


def lbm3d_step_timed(h, nsteps: int) -> float:
    ms = ctypes.c_double(0.0)
    _check(_lib.lbm3d_step_timed(h, int(nsteps), ctypes.byref(ms)), "lbm3d_step_timed")
    return ms.value


def lbm3d_step_profiled(h, nsteps: int):
    """(total_ms, mean fused-step kernel ms) over nsteps single launches."""
    tot = ctypes.c_double(0.0)
    ker = ctypes.c_double(0.0)
    _check(_lib.lbm3d_step_profiled(h, int(nsteps), ctypes.byref(tot), ctypes.byref(ker)),
           "lbm3d_step_profiled")
    return tot.value, ker.value


def lbm3d_set_tile(h, by: int, tz: int):
    _check(_lib.lbm3d_set_tile(h, int(by), int(tz)), "lbm3d_set_tile")


def lbm3d_get_tile(h):
    by = ctypes.c_int32(0)
    tz = ctypes.c_int32(0)
    _check(_lib.lbm3d_get_tile(h, ctypes.byref(by), ctypes.byref(tz)), "lbm3d_get_tile")
    return by.value, tz.value


def lbm3d_set_streaming(h, streaming: bool):
    _check(_lib.lbm3d_set_streaming(h, 1 if streaming else 0), "lbm3d_set_streaming")


def lbm3d_get_streaming(h) -> bool:
    v = ctypes.c_int32(0)
    _check(_lib.lbm3d_get_streaming(h, ctypes.byref(v)), "lbm3d_get_streaming")
    return bool(v.value)


def lbm3d_tune(h, launches: int = 10):
    by = ctypes.c_int32(0)
    tz = ctypes.c_int32(0)
    _check(_lib.lbm3d_tune(h, int(launches), ctypes.byref(by), ctypes.byref(tz)), "lbm3d_tune")
    return by.value, tz.value


def lbm3d_tune_save(path: str):
    _check(_lib.lbm3d_tune_save(os.fsencode(path)), "lbm3d_tune_save")


def lbm3d_tune_load(path: str):
    _check(_lib.lbm3d_tune_load(os.fsencode(path)), "lbm3d_tune_load")


def lbm3d_sync(h):
    _check(_lib.lbm3d_sync(h), "lbm3d_sync")


def lbm3d_stability(params: dict, q, axis: int = 0, kdx=(0.0, np.pi), nk: int = 64, alpha_t: float = 0.0):
    """Von Neumann analysis of the scheme about the uniform state
    q = (rho, ux, uy, uz, T): (max |omega|, k dx where it occurs) over nk
    wave numbers in [kdx[0], kdx[1]] along `axis` (3: all axes)."""
    p = make_params(params)
    qa = np.ascontiguousarray(q, dtype=np.float64)
    if qa.shape != (5,):
        raise ValueError("q must hold (rho, ux, uy, uz, T)")
    om = ctypes.c_double(0.0)
    kk = ctypes.c_double(0.0)
    _check(_lib.lbm3d_stability(ctypes.byref(p), _dp(qa), int(axis), float(kdx[0]), float(kdx[1]), int(nk),
                                float(alpha_t), ctypes.byref(om), ctypes.byref(kk)), "lbm3d_stability")
    return om.value, kk.value


def lbm3d_admit(params, fields):
    """Stability admission of an initial state: (status, max |omega|) with
    status OK or E_UNSTABLE (other errors raise)."""
    p = _params(params)
    n = p.nx * p.ny * p.nz
    arrs = _fields5(fields, n)
    om = ctypes.c_double(0.0)
    rc = _lib.lbm3d_admit(ctypes.byref(p), *[_dp(a) for a in arrs], ctypes.byref(om))
    if rc not in (OK, E_UNSTABLE):
        _check(rc, "lbm3d_admit")
    return rc, om.value


def lbm3d_stream_copy_rate(nbytes: int, launches: int = 10) -> float:
    """GB/s (read + written) of a plain copy alternating between two device
    buffers of nbytes each: the practical ceiling of an HBM-bound kernel."""
    gbs = ctypes.c_double(0.0)
    _check(_lib.lbm3d_stream_copy_rate(int(nbytes), int(launches), ctypes.byref(gbs)), "lbm3d_stream_copy_rate")
    return gbs.value


def lbm3d_moments(h, shape, allow_nonfinite: bool = False):
    out = [np.empty(shape, dtype=np.float64) for _ in range(5)]
    rc = _lib.lbm3d_moments(h, *[_dp(a) for a in out])
    if not (rc == E_NONFINITE and allow_nonfinite):
        _check(rc, "lbm3d_moments")
    return tuple(out)


def lbm3d_conserved(h) -> np.ndarray:
    out = np.zeros(5)
    _check(_lib.lbm3d_conserved(h, _dp(out)), "lbm3d_conserved")
    return out


def lbm3d_status(h):
    hw = ctypes.c_uint32(0)
    st = ctypes.c_int64(0)
    _check(_lib.lbm3d_status(h, ctypes.byref(hw), ctypes.byref(st)), "lbm3d_status")
    return hw.value, st.value


def lbm3d_get_f(h, shape, precision: int) -> np.ndarray:
    dt = np.float64 if precision == FP64 else np.float32
    out = np.empty((NV,) + tuple(shape), dtype=dt)
    _check(_lib.lbm3d_get_f(h, out.ctypes.data_as(ctypes.c_void_p), out.nbytes), "lbm3d_get_f")
    return out


def lbm3d_poison_next(h):
    _check(_lib.lbm3d_poison_next(h), "lbm3d_poison_next")


def lbm3d_set_f(h, f: np.ndarray):
    f = np.ascontiguousarray(f)
    _check(_lib.lbm3d_set_f(h, f.ctypes.data_as(ctypes.c_void_p), f.nbytes), "lbm3d_set_f")


def lbm3d_batch_step(handles, nsteps):
    arr = (ctypes.c_void_p * len(handles))(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])
    ns = (ctypes.c_int64 * len(handles))(*[int(n) for n in nsteps])
    _check(_lib.lbm3d_batch_step(arr, len(handles), ns), "lbm3d_batch_step")


def lbm3d_batch_step_noalloc(handles, nsteps):
    arr = (ctypes.c_void_p * len(handles))(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])
    ns = (ctypes.c_int64 * len(handles))(*[int(n) for n in nsteps])
    _check(_lib.lbm3d_batch_step_noalloc(arr, len(handles), ns), "lbm3d_batch_step_noalloc")


def lbm3d_batch_set_depth(precision, tz: int):
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(_lib.lbm3d_batch_set_depth(prec, int(tz)), "lbm3d_batch_set_depth")


def lbm3d_batch_plan(params_list, tz: int = 0, cus: int = 256):
    """Host-side work plan of the batched step: (tiles, list_first, nblocks)
    with tiles an (n, 7) int32 array of (solve, x0, x1, y0, y1, z0, z1)."""
    arr = (lbm3d_params * len(params_list))(*[_params(p) for p in params_list])
    nt, nl, nb = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    _check(_lib.lbm3d_batch_plan(arr, len(params_list), int(tz), int(cus), ctypes.byref(nt), ctypes.byref(nl),
                                 ctypes.byref(nb), None, 0, None), "lbm3d_batch_plan")
    tiles = np.zeros((max(nt.value, 1), 7), dtype=np.int32)
    first = np.zeros(9, dtype=np.int32)
    I32P = ctypes.POINTER(ctypes.c_int32)
    _check(_lib.lbm3d_batch_plan(arr, len(params_list), int(tz), int(cus), None, None, None,
                                 tiles.ctypes.data_as(I32P), tiles.shape[0], first.ctypes.data_as(I32P)),
           "lbm3d_batch_plan")
    return tiles[:nt.value], first[:nl.value + 1], nb.value


def lbm3d_batch_tune(handles, launches: int = 5) -> int:
    arr = (ctypes.c_void_p * len(handles))(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])
    tz = ctypes.c_int32(0)
    _check(_lib.lbm3d_batch_tune(arr, len(handles), int(launches), ctypes.byref(tz)), "lbm3d_batch_tune")
    return tz.value


def lbm3d_server_create(hbm_budget_bytes: int, max_active: int):
    s = ctypes.c_void_p()
    _check(_lib.lbm3d_server_create(int(hbm_budget_bytes), int(max_active), ctypes.byref(s)),
           "lbm3d_server_create")
    return s


def lbm3d_server_set_tick(s, steps: int):
    _check(_lib.lbm3d_server_set_tick(s, int(steps)), "lbm3d_server_set_tick")


def lbm3d_server_submit(s, params, fields, nsteps: int) -> int:
    p = _params(params)
    n = p.nx * p.ny * p.nz
    arrs = _fields5(fields, n)
    t = ctypes.c_uint64(0)
    _check(_lib.lbm3d_server_submit(s, ctypes.byref(p), *[_dp(a) for a in arrs], int(nsteps),
                                    ctypes.byref(t)), "lbm3d_server_submit")
    return t.value


def lbm3d_server_poll(s, ticket: int) -> bool:
    d = ctypes.c_int32(0)
    _check(_lib.lbm3d_server_poll(s, ctypes.c_uint64(ticket), ctypes.byref(d)), "lbm3d_server_poll")
    return bool(d.value)


def lbm3d_server_wait(s, ticket: int, shape):
    """Returns (status, (rho, ux, uy, uz, p), timing dict)."""
    out = [np.empty(shape, dtype=np.float64) for _ in range(5)]
    t = lbm3d_timing()
    rc = _lib.lbm3d_server_wait(s, ctypes.c_uint64(ticket), *[_dp(a) for a in out], ctypes.byref(t))
    if rc not in (OK, E_NONFINITE, E_CANCELLED, E_UNSTABLE):
        raise LbmError(rc, "lbm3d_server_wait")
    timing = dict(t_submit=t.t_submit, t_admit=t.t_admit, t_done=t.t_done, steps=t.steps, health=t.health)
    return rc, tuple(out), timing


def lbm3d_server_stats(s) -> dict:
    st = lbm3d_server_counters()
    _check(_lib.lbm3d_server_stats(s, ctypes.byref(st)), "lbm3d_server_stats")
    return {name: getattr(st, name) for name, _ in lbm3d_server_counters._fields_}


def lbm3d_server_cancel(s, ticket: int):
    _check(_lib.lbm3d_server_cancel(s, ctypes.c_uint64(ticket)), "lbm3d_server_cancel")


def lbm3d_server_destroy(s):
    _check(_lib.lbm3d_server_destroy(s), "lbm3d_server_destroy")


# ----------------------------------------------------------- conveniences --
class Solver:
    """One solve on the GPU: ``Solver(params_dict)``; fields are (nz, ny, nx)."""

    def __init__(self, params):
        self.params = _params(params)
        self.shape = (self.params.nz, self.params.ny, self.params.nx)
        self.precision = self.params.precision
        self.h = lbm3d_create(self.params)

    def close(self):
        if self.h is not None and self.h.value:
            lbm3d_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def init(self, rho, ux, uy, uz, p):
        lbm3d_init(self.h, self.shape, rho, ux, uy, uz, p)

    def step(self, n: int = 1):
        lbm3d_step(self.h, n)

    def step_timed(self, n: int) -> float:
        return lbm3d_step_timed(self.h, n)

    def step_profiled(self, n: int):
        return lbm3d_step_profiled(self.h, n)

    def sync(self):
        lbm3d_sync(self.h)

    def set_tile(self, by: int, tz: int):
        lbm3d_set_tile(self.h, by, tz)

    def get_tile(self):
        return lbm3d_get_tile(self.h)

    def set_streaming(self, streaming: bool):
        lbm3d_set_streaming(self.h, streaming)

    def streaming(self) -> bool:
        return lbm3d_get_streaming(self.h)

    def tune(self, launches: int = 10):
        return lbm3d_tune(self.h, launches)

    def moments(self, allow_nonfinite: bool = False):
        return lbm3d_moments(self.h, self.shape, allow_nonfinite)

    def conserved(self):
        return lbm3d_conserved(self.h)

    def status(self):
        return lbm3d_status(self.h)

    def get_f(self):
        return lbm3d_get_f(self.h, self.shape, self.precision)

    def set_f(self, f):
        lbm3d_set_f(self.h, f)

    def poison_next(self):
        lbm3d_poison_next(self.h)


class Server:
    """Continuous-batching server: ``Server(budget_bytes, max_active)``;
    ``submit(params, fields, nsteps) -> ticket``; ``wait(ticket, shape)``."""

    def __init__(self, hbm_budget_bytes: int, max_active: int, tick_steps: int = None):
        self.s = lbm3d_server_create(hbm_budget_bytes, max_active)
        if tick_steps is not None:
            lbm3d_server_set_tick(self.s, tick_steps)

    def submit(self, params, fields, nsteps: int) -> int:
        return lbm3d_server_submit(self.s, params, fields, nsteps)

    def poll(self, ticket: int) -> bool:
        return lbm3d_server_poll(self.s, ticket)

    def wait(self, ticket: int, shape):
        return lbm3d_server_wait(self.s, ticket, shape)

    def cancel(self, ticket: int):
        lbm3d_server_cancel(self.s, ticket)

    def stats(self) -> dict:
        return lbm3d_server_stats(self.s)

    def close(self):
        if self.s is not None and self.s.value:
            lbm3d_server_destroy(self.s)
        self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
