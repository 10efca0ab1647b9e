"""ctypes binding of ``libcavity.so`` (the C ABI in ``include/cavity.h``).

Argument marshalling only: every step of the time stepper runs in the HIP
library.  PyTorch supplies device memory (the workspace and field tensors)
and the stream.  The functions carry the C names; :class:`Cavity` wraps them.

There is no fallback: if the library is missing this module raises on import.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
# torch first: the library then binds to the HIP runtime torch has loaded.
# Loaded before torch, the library binds to the system's HIP runtime and torch
# loads its own, two runtimes in one process, and the library's pinned host
# allocations fail.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcavity.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_0809_3098_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

# ----------------------------------------------------------------- status
CAVITY_OK = 0
CAVITY_EINVAL = -1
CAVITY_ENOMEM = -2
CAVITY_EHIP = -3
CAVITY_ENOCONV = -4
CAVITY_ENONFINITE = -5
CAVITY_ESTATE = -6
CAVITY_FP64 = 0
CAVITY_MIXED = 1
CAVITY_EXEC_STREAM = 0
CAVITY_EXEC_PERSISTENT = 1
CAVITY_EXEC_GRAPH = 2
CAVITY_EXEC_RESIDENT = 3
CAVITY_SOLVER_SOR = 0
CAVITY_SOLVER_MG = 1
CAVITY_WARM_DEFAULT = 0
CAVITY_WARM_PREVIOUS = 1
CAVITY_WARM_LEVELS_FP64 = 6
CAVITY_WARM_LEVELS_MIXED = 8
CAVITY_WARM_DEGREE_MIXED = 5
CAVITY_WARM_LEVELS_MAX = 8

_STATUS_NAMES = {0: "CAVITY_OK", -1: "CAVITY_EINVAL", -2: "CAVITY_ENOMEM", -3: "CAVITY_EHIP",
                 -4: "CAVITY_ENOCONV", -5: "CAVITY_ENONFINITE", -6: "CAVITY_ESTATE"}


class CavityError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(code, code)}: {message}")
        self.code = code
        self.message = message


# ------------------------------------------------------------------ structs
class cavity_params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("re", ctypes.c_double), ("u_lid", ctypes.c_double), ("nu", ctypes.c_double),
        ("dt", ctypes.c_double), ("cfl", ctypes.c_double), ("poisson_tol", ctypes.c_double),
        ("poisson_max_sweeps", ctypes.c_int32), ("resume", ctypes.c_int32),
        ("sor_omega", ctypes.c_double),
        ("omega0", ctypes.c_void_p), ("psi0", ctypes.c_void_p),
        ("fixed_sweeps", ctypes.c_int32), ("warm_start", ctypes.c_int32),
    ]


class cavity_stats(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("t", ctypes.c_double), ("dt", ctypes.c_double),
        ("res_psi", ctypes.c_double), ("res_omega", ctypes.c_double),
        ("domega_inf_over_dt", ctypes.c_double), ("ke", ctypes.c_double),
        ("last_resid_inf", ctypes.c_double), ("sweeps_total", ctypes.c_int64),
        ("sweeps_last_step", ctypes.c_int64), ("floor_limited", ctypes.c_int32),
        ("status", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class cavity_poisson_info(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("resid_inf", ctypes.c_double),
                ("floor_limited", ctypes.c_int32), ("status", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class cavity_tuning(ctypes.Structure):
    _fields_ = [
        ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
        ("sweeps_per_launch", ctypes.c_int32), ("threads", ctypes.c_int32),
        ("tile_x32", ctypes.c_int32), ("tile_y32", ctypes.c_int32),
        ("sweeps_per_launch32", ctypes.c_int32), ("threads32", ctypes.c_int32),
        ("check_every", ctypes.c_int32), ("inner_sweeps", ctypes.c_int32),
        ("xcd_bands", ctypes.c_int32), ("solver", ctypes.c_int32),
        ("sor_omega", ctypes.c_double), ("warm_degree", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.POINTER
_lib.cavity_workspace_bytes.argtypes = [_P(cavity_params), ctypes.c_int32, _P(ctypes.c_size_t)]
_lib.cavity_create.argtypes = [_P(cavity_params), ctypes.c_int32, ctypes.c_void_p,
                               ctypes.c_size_t, ctypes.c_void_p, _P(ctypes.c_void_p)]
_lib.cavity_step.argtypes = [ctypes.c_void_p, ctypes.c_int32, _P(cavity_stats)]
_lib.cavity_run_steady.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                   _P(ctypes.c_double), _P(ctypes.c_double), _P(ctypes.c_int64),
                                   _P(cavity_stats)]
_lib.cavity_poisson.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                ctypes.c_void_p, _P(cavity_poisson_info)]
_lib.cavity_poisson_noalloc.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, _P(cavity_poisson_info)]
_lib.cavity_fields.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_void_p]
_lib.cavity_relax.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                              ctypes.c_void_p, _P(ctypes.c_int64)]
_lib.cavity_get_tuning.argtypes = [ctypes.c_void_p, ctypes.c_int32, _P(cavity_tuning)]
_lib.cavity_set_tuning.argtypes = [ctypes.c_void_p, ctypes.c_int32, _P(cavity_tuning)]
_lib.cavity_autotune.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_char_p,
                                 _P(cavity_tuning)]
_lib.cavity_set_exec.argtypes = [ctypes.c_void_p, ctypes.c_int32]
_lib.cavity_get_exec.argtypes = [ctypes.c_void_p, _P(ctypes.c_int32)]
_lib.cavity_destroy.argtypes = [ctypes.c_void_p]
_lib.cavity_warm_weights.argtypes = [ctypes.c_int32, ctypes.c_int32, _P(ctypes.c_double)]
_lib.cavity_last_error.restype = ctypes.c_char_p
for _f in ("cavity_workspace_bytes", "cavity_create", "cavity_step", "cavity_run_steady",
           "cavity_poisson", "cavity_poisson_noalloc",
           "cavity_fields", "cavity_relax", "cavity_get_tuning", "cavity_set_tuning",
           "cavity_set_exec", "cavity_get_exec", "cavity_autotune", "cavity_destroy",
           "cavity_warm_weights"):
    getattr(_lib, _f).restype = ctypes.c_int

EXPORTED = ("cavity_workspace_bytes", "cavity_create", "cavity_step", "cavity_run_steady",
            "cavity_poisson", "cavity_poisson_noalloc",
            "cavity_fields", "cavity_relax", "cavity_get_tuning", "cavity_set_tuning",
            "cavity_set_exec", "cavity_get_exec", "cavity_autotune", "cavity_destroy",
            "cavity_warm_weights", "cavity_last_error")


def cavity_warm_weights(levels: int, degree: int) -> np.ndarray:
    """Warm-start weights w[q-1] of psi(step - q), q = 1 ... levels (host only)."""
    w = (ctypes.c_double * max(levels, 1))()
    _check(_lib.cavity_warm_weights(levels, degree, w))
    return np.array(w[:levels], dtype=np.float64)


def cavity_last_error() -> str:
    return (_lib.cavity_last_error() or b"").decode()


def _check(rc: int, allow=()):
    if rc != CAVITY_OK and rc not in allow:
        raise CavityError(rc, cavity_last_error())
    return rc


# ------------------------------------------------------------------ params
@dataclass
class Params:
    """Python mirror of ``cavity_params`` (device pointers set by the caller)."""
    n: int
    re: float = 1000.0
    u_lid: float = 1.0
    nu: float = 0.0
    dt: float = 0.0
    cfl: float = 0.5
    poisson_tol: float = 1e-10
    poisson_max_sweeps: int = 0
    precision: int = CAVITY_FP64
    sor_omega: float = 0.0
    resume: int = 0
    fixed_sweeps: int = 0
    warm_start: int = CAVITY_WARM_DEFAULT

    def to_c(self, omega0_ptr: int = 0, psi0_ptr: int = 0) -> cavity_params:
        return cavity_params(n=self.n, precision=self.precision, re=self.re, u_lid=self.u_lid,
                             nu=self.nu, dt=self.dt, cfl=self.cfl, poisson_tol=self.poisson_tol,
                             poisson_max_sweeps=self.poisson_max_sweeps, resume=self.resume,
                             sor_omega=self.sor_omega, omega0=omega0_ptr or None,
                             psi0=psi0_ptr or None, fixed_sweeps=self.fixed_sweeps,
                             warm_start=self.warm_start)


def _param_array(params: Sequence[cavity_params]):
    arr = (cavity_params * len(params))()
    for k, p in enumerate(params):
        arr[k] = p
    return arr


# --------------------------------------------------------------- functions
def cavity_workspace_bytes(params: Sequence[cavity_params]) -> int:
    arr = _param_array(params)
    out = ctypes.c_size_t(0)
    _check(_lib.cavity_workspace_bytes(arr, len(params), ctypes.byref(out)))
    return int(out.value)


def cavity_create(params: Sequence[cavity_params], ws_ptr: int, ws_bytes: int,
                  stream_ptr: int, allow_noconv: bool = False) -> int:
    arr = _param_array(params)
    h = ctypes.c_void_p(0)
    rc = _lib.cavity_create(arr, len(params), ctypes.c_void_p(ws_ptr), ws_bytes,
                            ctypes.c_void_p(stream_ptr), ctypes.byref(h))
    _check(rc, allow=(CAVITY_ENOCONV,) if allow_noconv else ())
    return int(h.value)


def cavity_step(h: int, nsteps: int, count: int = 1, want_stats: bool = True,
                allow_noconv: bool = False):
    stats = (cavity_stats * count)() if want_stats else None
    rc = _lib.cavity_step(ctypes.c_void_p(h), nsteps, stats)
    _check(rc, allow=(CAVITY_ENOCONV,) if allow_noconv else ())
    return [s.as_dict() for s in stats] if want_stats else None


def cavity_run_steady(h: int, max_steps: int, check_every: int, count: int = 1,
                      res_psi_tol: Optional[Sequence[float]] = None,
                      res_omega_tol: Optional[Sequence[float]] = None,
                      allow_noconv: bool = False):
    """Returns (steady_step per cavity, stats of the last step per cavity)."""
    def arr(v):
        return None if v is None else (ctypes.c_double * count)(*[float(x) for x in v])
    steady = (ctypes.c_int64 * count)()
    stats = (cavity_stats * count)()
    rc = _lib.cavity_run_steady(ctypes.c_void_p(h), max_steps, check_every, arr(res_psi_tol),
                                arr(res_omega_tol), steady, stats)
    _check(rc, allow=(CAVITY_ENOCONV,) if allow_noconv else ())
    return [int(x) for x in steady], [s.as_dict() for s in stats]


def cavity_poisson(h: int, idx: int, omega_ptr: int = 0, psi_ptr: int = 0,
                   want_info: bool = True, allow_noconv: bool = False):
    info = cavity_poisson_info() if want_info else None
    rc = _lib.cavity_poisson(ctypes.c_void_p(h), idx, ctypes.c_void_p(omega_ptr or None),
                             ctypes.c_void_p(psi_ptr or None),
                             ctypes.byref(info) if want_info else None)
    _check(rc, allow=(CAVITY_ENOCONV,) if allow_noconv else ())
    return info.as_dict() if want_info else None


def cavity_poisson_noalloc(n: int, omega_ptr: int, psi_ptr: int, stream_ptr: int,
                           poisson_tol: float = 0.0, sor_omega: float = 0.0,
                           poisson_max_sweeps: int = 0, allow_noconv: bool = False) -> dict:
    """Handle-free Poisson solve whose scratch is the library's device array."""
    info = cavity_poisson_info()
    rc = _lib.cavity_poisson_noalloc(n, poisson_tol, sor_omega, poisson_max_sweeps,
                                     ctypes.c_void_p(omega_ptr or None),
                                     ctypes.c_void_p(psi_ptr or None),
                                     ctypes.c_void_p(stream_ptr or None), ctypes.byref(info))
    _check(rc, allow=(CAVITY_ENOCONV,) if allow_noconv else ())
    return info.as_dict()


def cavity_fields(h: int, idx: int, psi_ptr: int = 0, omega_ptr: int = 0, u_ptr: int = 0,
                  v_ptr: int = 0) -> None:
    _check(_lib.cavity_fields(ctypes.c_void_p(h), idx, ctypes.c_void_p(psi_ptr or None),
                              ctypes.c_void_p(omega_ptr or None), ctypes.c_void_p(u_ptr or None),
                              ctypes.c_void_p(v_ptr or None)))


def cavity_relax(h: int, idx: int, sweeps: int, arith: int = 0, psi_out_ptr: int = 0) -> int:
    done = ctypes.c_int64(0)
    _check(_lib.cavity_relax(ctypes.c_void_p(h), idx, sweeps, arith,
                             ctypes.c_void_p(psi_out_ptr or None), ctypes.byref(done)))
    return int(done.value)


def cavity_get_tuning(h: int, idx: int) -> dict:
    t = cavity_tuning()
    _check(_lib.cavity_get_tuning(ctypes.c_void_p(h), idx, ctypes.byref(t)))
    return t.as_dict()


def cavity_set_tuning(h: int, idx: int, **kw) -> dict:
    t = cavity_tuning()
    _check(_lib.cavity_get_tuning(ctypes.c_void_p(h), idx, ctypes.byref(t)))
    for k, v in kw.items():
        if k not in t.as_dict():
            raise KeyError(k)
        setattr(t, k, v)
    _check(_lib.cavity_set_tuning(ctypes.c_void_p(h), idx, ctypes.byref(t)))
    return cavity_get_tuning(h, idx)


def cavity_autotune(h: int, idx: int, cache_path: Optional[str] = None) -> dict:
    t = cavity_tuning()
    path = cache_path.encode() if cache_path else None
    _check(_lib.cavity_autotune(ctypes.c_void_p(h), idx, path, ctypes.byref(t)))
    return t.as_dict()


def cavity_set_exec(h: int, mode: int) -> None:
    _check(_lib.cavity_set_exec(ctypes.c_void_p(h), mode))


def cavity_get_exec(h: int) -> int:
    out = ctypes.c_int32(0)
    _check(_lib.cavity_get_exec(ctypes.c_void_p(h), ctypes.byref(out)))
    return int(out.value)


def cavity_destroy(h: int) -> None:
    _check(_lib.cavity_destroy(ctypes.c_void_p(h)))


# ------------------------------------------------------------ convenience
class Cavity:
    """One or more cavities on one GPU; torch supplies memory and the stream.

    ``omega0`` / ``psi0`` are optional lists (per cavity) of n x n float64
    numpy arrays or CUDA tensors.
    """

    def __init__(self, params: Sequence[Params] | Params, device: str = "cuda:0",
                 omega0: Optional[Sequence] = None, psi0: Optional[Sequence] = None,
                 stream=None, allow_noconv: bool = False):
        import torch
        self._torch = torch
        if isinstance(params, Params):
            params = [params]
        self.params = list(params)
        self.count = len(self.params)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        keep = []

        def dev(a):
            if a is None:
                return 0
            t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
            t = t.to(device=self.device, dtype=torch.float64).contiguous()
            keep.append(t)
            return t.data_ptr()

        cps = []
        for k, p in enumerate(self.params):
            w = dev(omega0[k]) if omega0 is not None else 0
            s = dev(psi0[k]) if psi0 is not None else 0
            cps.append(p.to_c(w, s))
        nbytes = cavity_workspace_bytes(cps)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        self.handle = cavity_create(cps, self.workspace.data_ptr(), nbytes,
                                    self.stream.cuda_stream, allow_noconv=allow_noconv)
        del keep

    def step(self, nsteps: int = 1, want_stats: bool = True, allow_noconv: bool = False):
        return cavity_step(self.handle, nsteps, self.count, want_stats, allow_noconv)

    def run_steady(self, max_steps: int, check_every: int = 10, res_psi_tol=None,
                   res_omega_tol=None, allow_noconv: bool = False):
        return cavity_run_steady(self.handle, max_steps, check_every, self.count, res_psi_tol,
                                 res_omega_tol, allow_noconv)

    def poisson(self, idx: int = 0, omega=None, want_psi: bool = True, allow_noconv=False):
        torch = self._torch
        n = self.params[idx].n
        w = None
        if omega is not None:
            w = omega if isinstance(omega, torch.Tensor) else torch.from_numpy(
                np.ascontiguousarray(omega))
            w = w.to(device=self.device, dtype=torch.float64).contiguous()
        out = torch.empty((n, n), dtype=torch.float64, device=self.device) if want_psi else None
        info = cavity_poisson(self.handle, idx, w.data_ptr() if w is not None else 0,
                              out.data_ptr() if out is not None else 0, True, allow_noconv)
        self.stream.synchronize()
        return (out.cpu().numpy() if out is not None else None), info

    def fields_tensors(self, idx: int = 0):
        torch = self._torch
        n = self.params[idx].n
        t = [torch.empty((n, n), dtype=torch.float64, device=self.device) for _ in range(4)]
        cavity_fields(self.handle, idx, *(x.data_ptr() for x in t))
        self.stream.synchronize()
        return t

    def fields(self, idx: int = 0):
        """psi, omega, u, v of cavity idx as numpy arrays [j, i]."""
        return tuple(x.cpu().numpy() for x in self.fields_tensors(idx))

    def relax(self, sweeps: int, idx: int = 0, want_psi: bool = False, arith: int = 0):
        """Enqueue `sweeps` smoother sweeps on scratch buffers (no sync)."""
        out = None
        if want_psi:
            n = self.params[idx].n
            out = self._torch.empty((n, n), dtype=self._torch.float64, device=self.device)
        done = cavity_relax(self.handle, idx, sweeps, arith,
                            out.data_ptr() if out is not None else 0)
        return done, out

    def tuning(self, idx: int = 0) -> dict:
        return cavity_get_tuning(self.handle, idx)

    def set_tuning(self, idx: int = 0, **kw) -> dict:
        return cavity_set_tuning(self.handle, idx, **kw)

    def autotune(self, idx: int = 0, cache_path: Optional[str] = None) -> dict:
        return cavity_autotune(self.handle, idx, cache_path)

    def set_exec(self, mode: int) -> None:
        cavity_set_exec(self.handle, mode)

    def exec_mode(self) -> int:
        return cavity_get_exec(self.handle)

    def close(self):
        if getattr(self, "handle", 0):
            cavity_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
