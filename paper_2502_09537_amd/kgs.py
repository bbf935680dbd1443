"""Python binding of libkgs (the C ABI in include/kgs.h).

Argument marshalling only: every step of the solver runs in the HIP kernels
of libkgs.so.  PyTorch is used for device memory (input/output tensors) and
streams (the handle runs on torch's current stream).  If the library is not
built this module raises on first use; there is no fallback.

Raw entry points keep the C names (``kgs_init``, ``kgs_step``, ...);
``Simulation`` wraps a handle.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkgs.so")

KGS_OK, KGS_EINVAL, KGS_EODDN, KGS_ESINGULAR, KGS_ENOMEM, KGS_EDEVICE, KGS_ENONFINITE = range(7)
KGS_FP64, KGS_FP32 = 0, 1
KGS_HOST, KGS_DEVICE = 0, 1
KGS_KERNEL_AUTO, KGS_KERNEL_SWEEP, KGS_KERNEL_STREAM, KGS_KERNEL_RESIDENT, KGS_KERNEL_TILE = range(5)

# every function declared in include/kgs.h
EXPORTS = (
    "kgs_init", "kgs_step", "kgs_energy", "kgs_read_state", "kgs_write_state", "kgs_sync",
    "kgs_free", "kgs_last_error", "kgs_status_string", "kgs_get_tuning", "kgs_set_tuning",
    "kgs_get_info", "kgs_required_bytes", "kgs_autotune",
    "kgs_batch_create", "kgs_batch_step", "kgs_batch_step_each", "kgs_batch_set_graph",
    "kgs_batch_free", "kgs_batch_last_error",
    "kgs_server_create", "kgs_server_submit", "kgs_server_run", "kgs_server_poll",
    "kgs_server_result", "kgs_server_release", "kgs_server_cancel", "kgs_server_stats",
    "kgs_server_free", "kgs_server_last_error", "kgs_step_fields", "kgs_batch_autotune",
)
KGS_REQ_QUEUED, KGS_REQ_RUNNING, KGS_REQ_DONE, KGS_REQ_FAILED, KGS_REQ_CANCELLED = range(5)


class KgsConfig(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("n", ctypes.c_int32),
        ("lo", ctypes.c_double), ("hi", ctypes.c_double), ("tau", ctypes.c_double),
        ("kappa1", ctypes.c_double), ("kappa2", ctypes.c_double),
        ("mu", ctypes.c_double), ("gamma", ctypes.c_double),
        ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class KgsTuning(ctypes.Structure):
    _fields_ = [
        ("kernel", ctypes.c_int32), ("block", ctypes.c_int32),
        ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
        ("chunk", ctypes.c_int32), ("steps_per_launch", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 2),
    ]


class KgsInfo(ctypes.Structure):
    _fields_ = [
        ("points", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
        ("kernel", ctypes.c_int32), ("precision", ctypes.c_int32),
    ]


class KgsServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("max_active", ctypes.c_int32),
                ("steps_per_round", ctypes.c_int32), ("round_work", ctypes.c_int64),
                ("reserved", ctypes.c_int32 * 2)]


class KgsRequestInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32),
                ("steps_done", ctypes.c_int64), ("nsteps", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double),
                ("energy_start", ctypes.c_double), ("energy_end", ctypes.c_double)]


class KgsServerStats(ctypes.Structure):
    _fields_ = [("device_bytes_used", ctypes.c_int64), ("queued_input_bytes", ctypes.c_int64),
                ("running", ctypes.c_int32),
                ("queued", ctypes.c_int32), ("rounds", ctypes.c_int64), ("now", ctypes.c_double)]


class KgsError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{status_string(status)}: {message}")


_lib = None
_DP = ctypes.POINTER(ctypes.c_double)
_VP = ctypes.c_void_p


def lib():
    """Load libkgs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2502_09537_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        sig = {
            "kgs_init": ([P(KgsConfig), _VP, _VP, _VP, _VP, ctypes.c_int32, _VP, P(_VP)], ctypes.c_int),
            "kgs_step": ([_VP, ctypes.c_int64], ctypes.c_int),
            "kgs_energy": ([_VP, _DP], ctypes.c_int),
            "kgs_read_state": ([_VP, _VP, _VP, _VP, _VP, ctypes.c_int32], ctypes.c_int),
            "kgs_write_state": ([_VP, _VP, _VP, _VP, _VP, ctypes.c_int32], ctypes.c_int),
            "kgs_sync": ([_VP], ctypes.c_int),
            "kgs_free": ([_VP], ctypes.c_int),
            "kgs_last_error": ([_VP], ctypes.c_char_p),
            "kgs_status_string": ([ctypes.c_int], ctypes.c_char_p),
            "kgs_get_tuning": ([_VP, P(KgsTuning)], ctypes.c_int),
            "kgs_set_tuning": ([_VP, P(KgsTuning)], ctypes.c_int),
            "kgs_get_info": ([_VP, P(KgsInfo)], ctypes.c_int),
            "kgs_required_bytes": ([P(KgsConfig)], ctypes.c_int64),
            "kgs_autotune": ([_VP, ctypes.c_int32, ctypes.c_int32, P(KgsTuning)], ctypes.c_int),
            "kgs_batch_create": ([P(_VP), ctypes.c_int32, _VP, P(_VP)], ctypes.c_int),
            "kgs_batch_step": ([_VP, ctypes.c_int64], ctypes.c_int),
            "kgs_batch_step_each": ([_VP, P(ctypes.c_int64)], ctypes.c_int),
            "kgs_batch_set_graph": ([_VP, ctypes.c_int32], ctypes.c_int),
            "kgs_batch_free": ([_VP], ctypes.c_int),
            "kgs_batch_autotune": ([_VP, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
            "kgs_batch_last_error": ([_VP], ctypes.c_char_p),
            "kgs_server_create": ([P(KgsServerConfig), _VP, P(_VP)], ctypes.c_int),
            "kgs_server_submit": ([_VP, P(KgsConfig), _VP, _VP, _VP, _VP, ctypes.c_int32,
                                   ctypes.c_int64, P(ctypes.c_int64)], ctypes.c_int),
            "kgs_server_run": ([_VP, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_int32)],
                               ctypes.c_int),
            "kgs_server_poll": ([_VP, ctypes.c_int64, P(KgsRequestInfo)], ctypes.c_int),
            "kgs_server_result": ([_VP, ctypes.c_int64, _VP, _VP, _VP, _VP, ctypes.c_int32],
                                  ctypes.c_int),
            "kgs_server_release": ([_VP, ctypes.c_int64], ctypes.c_int),
            "kgs_server_cancel": ([_VP, ctypes.c_int64], ctypes.c_int),
            "kgs_server_stats": ([_VP, P(KgsServerStats)], ctypes.c_int),
            "kgs_server_free": ([_VP], ctypes.c_int),
            "kgs_server_last_error": ([_VP], ctypes.c_char_p),
            "kgs_step_fields": ([P(KgsConfig), _VP, _VP, _VP, _VP, ctypes.c_int64, _VP],
                                ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def status_string(status: int) -> str:
    try:
        return lib().kgs_status_string(status).decode()
    except ImportError:
        return f"status {status}"


def last_error(handle=None) -> str:
    return lib().kgs_last_error(handle).decode()


def _check(rc: int, handle=None):
    if rc != KGS_OK:
        raise KgsError(rc, last_error(handle))


def make_config(dim, n, lo, hi, tau, kappa1=1.0, kappa2=1.0, mu=1.0, gamma=1.0,
                precision=KGS_FP64) -> KgsConfig:
    return KgsConfig(int(dim), int(n), float(lo), float(hi), float(tau), float(kappa1),
                     float(kappa2), float(mu), float(gamma), int(precision), 0)


def config_of(problem) -> KgsConfig:
    """Config from a workloads.Problem."""
    return make_config(problem.dim, problem.n, problem.lo, problem.hi, problem.tau,
                       problem.kappa1, problem.kappa2, problem.mu, problem.gamma,
                       problem.precision)


def required_bytes(cfg: KgsConfig) -> int:
    return int(lib().kgs_required_bytes(ctypes.byref(cfg)))


# raw entry points ---------------------------------------------------------
def kgs_init(cfg: KgsConfig, psi_re: int, psi_im: int, u: int, v_t: int, mem: int,
             stream: int = 0):
    """Pointers are integers (host addresses or device data_ptr()); returns the handle."""
    h = _VP()
    rc = lib().kgs_init(ctypes.byref(cfg), psi_re, psi_im, u, v_t, mem, stream or None,
                        ctypes.byref(h))
    _check(rc)
    return h


def kgs_step(handle, nsteps: int) -> None:
    _check(lib().kgs_step(handle, int(nsteps)), handle)


# scratch area of kgs_step_fields per device (KGS_STEP_FIELDS_SCRATCH_BYTES)
KGS_STEP_FIELDS_SCRATCH_BYTES = 64 << 20


def kgs_step_fields(cfg: KgsConfig, psi_re: int, psi_im: int, u: int, v_t: int, nsteps: int,
                    stream: int = 0) -> None:
    """Advance four caller-owned float64 device arrays (data_ptr() integers)
    in place by nsteps steps, enqueued on `stream`; allocates nothing."""
    rc = lib().kgs_step_fields(ctypes.byref(cfg), psi_re, psi_im, u, v_t, int(nsteps),
                               stream or None)
    _check(rc)


def kgs_energy(handle) -> float:
    e = ctypes.c_double()
    rc = lib().kgs_energy(handle, ctypes.byref(e))
    if rc == KGS_ENONFINITE:
        return e.value
    _check(rc, handle)
    return e.value


def kgs_read_state(handle, psi_re: int, psi_im: int, u: int, v_t: int, mem: int) -> None:
    _check(lib().kgs_read_state(handle, psi_re, psi_im, u, v_t, mem), handle)


def kgs_write_state(handle, psi_re: int, psi_im: int, u: int, v_t: int, mem: int) -> None:
    _check(lib().kgs_write_state(handle, psi_re, psi_im, u, v_t, mem), handle)


def kgs_sync(handle) -> None:
    _check(lib().kgs_sync(handle), handle)


def kgs_free(handle) -> None:
    rc = lib().kgs_free(handle)
    if rc != KGS_OK:
        raise KgsError(rc, last_error(None))


def kgs_get_tuning(handle) -> KgsTuning:
    t = KgsTuning()
    _check(lib().kgs_get_tuning(handle, ctypes.byref(t)), handle)
    return t


def kgs_set_tuning(handle, t: KgsTuning) -> None:
    _check(lib().kgs_set_tuning(handle, ctypes.byref(t)), handle)


def kgs_get_info(handle) -> KgsInfo:
    i = KgsInfo()
    _check(lib().kgs_get_info(handle, ctypes.byref(i)), handle)
    return i


# convenience wrapper --------------------------------------------------------
def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("libkgs needs a ROCm GPU; torch.cuda.is_available() is False")
    return torch


class Simulation:
    """One DP-AVF2 simulation held on the GPU.

    psi (complex), u and v are numpy arrays (or torch tensors) of shape
    (n,)*dim.  Inputs go through torch device tensors (KGS_DEVICE) on torch's
    current stream unless ``host=True`` (KGS_HOST path of the C ABI).
    """

    def __init__(self, cfg: KgsConfig, psi, u, v, host: bool = False, stream=None,
                 tuning: Optional[KgsTuning] = None):
        self.cfg = cfg
        self.shape = (cfg.n,) * cfg.dim
        self.host = host
        self._torch = None if host else _torch()
        self.stream = stream if stream is not None else self._current_stream()
        self.handle = None
        P, Q, U, V = self._to_boundary(psi, u, v)
        self.handle = kgs_init(cfg, *self._ptrs(P, Q, U, V), KGS_HOST if host else KGS_DEVICE,
                               self.stream)
        if tuning is not None:
            kgs_set_tuning(self.handle, tuning)

    def _current_stream(self) -> int:
        if self._torch is None:
            return 0
        return int(self._torch.cuda.current_stream().cuda_stream)

    def _to_boundary(self, psi, u, v):
        if self.host:
            psi = np.asarray(psi)
            arrs = [np.ascontiguousarray(a, dtype=np.float64)
                    for a in (psi.real, psi.imag, np.asarray(u), np.asarray(v))]
        else:
            t = self._torch
            if isinstance(psi, t.Tensor):
                psi_re, psi_im = (psi.real, psi.imag) if psi.is_complex() else (psi, t.zeros_like(psi))
                src = (psi_re, psi_im, u, v)
            else:
                psi = np.asarray(psi)
                src = (psi.real, psi.imag, np.asarray(u), np.asarray(v))
            arrs = [t.as_tensor(np.ascontiguousarray(a) if not isinstance(a, t.Tensor) else a,
                                dtype=t.float64).to("cuda").contiguous() for a in src]
        for a in arrs:
            if tuple(a.shape) != self.shape:
                raise ValueError(f"array shape {tuple(a.shape)} != {self.shape}")
        return arrs

    def _ptrs(self, *arrs):
        if self.host:
            return [a.ctypes.data for a in arrs]
        return [a.data_ptr() for a in arrs]

    def step(self, nsteps: int = 1) -> "Simulation":
        kgs_step(self.handle, nsteps)
        return self

    def energy(self) -> float:
        return kgs_energy(self.handle)

    def sync(self) -> None:
        kgs_sync(self.handle)

    def read_state(self, as_torch: bool = False):
        """(psi, u, v) as complex128/float64 numpy arrays (or cuda tensors)."""
        if self.host:
            arrs = [np.empty(self.shape, dtype=np.float64) for _ in range(4)]
            kgs_read_state(self.handle, *self._ptrs(*arrs), KGS_HOST)
            P, Q, U, V = arrs
            return P + 1j * Q, U, V
        t = self._torch
        arrs = [t.empty(self.shape, dtype=t.float64, device="cuda") for _ in range(4)]
        kgs_read_state(self.handle, *[a.data_ptr() for a in arrs], KGS_DEVICE)
        if as_torch:
            P, Q, U, V = arrs
            return t.complex(P, Q), U, V
        P, Q, U, V = [a.cpu().numpy() for a in arrs]
        return P + 1j * Q, U, V

    def write_state(self, psi, u, v) -> None:
        P, Q, U, V = self._to_boundary(psi, u, v)
        kgs_write_state(self.handle, *self._ptrs(P, Q, U, V), KGS_HOST if self.host else KGS_DEVICE)

    @property
    def tuning(self) -> KgsTuning:
        return kgs_get_tuning(self.handle)

    @tuning.setter
    def tuning(self, t: KgsTuning) -> None:
        kgs_set_tuning(self.handle, t)

    def info(self) -> KgsInfo:
        return kgs_get_info(self.handle)

    def autotune(self, steps: int = 4, use_cache: bool = True) -> KgsTuning:
        """Pick the fastest launch configuration (state unchanged)."""
        t = KgsTuning()
        _check(lib().kgs_autotune(self.handle, int(steps), int(bool(use_cache)), ctypes.byref(t)),
               self.handle)
        return t

    def close(self) -> None:
        if self.handle is not None:
            h, self.handle = self.handle, None
            kgs_free(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many simulations advanced together (batched launches, optional hipGraph).

    The batch runs on torch's current stream (the stream the simulations were
    created on, by default)."""

    def __init__(self, sims, graph: bool = False, stream=None):
        self.sims = list(sims)
        arr = (_VP * len(self.sims))(*[s.handle for s in self.sims])
        self.stream = stream if stream is not None else self.sims[0].stream
        h = _VP()
        rc = lib().kgs_batch_create(arr, len(self.sims), self.stream or None, ctypes.byref(h))
        if rc != KGS_OK:
            raise KgsError(rc, lib().kgs_batch_last_error(None).decode())
        self.handle = h
        if graph:
            self.set_graph(True)

    def _check(self, rc):
        if rc != KGS_OK:
            raise KgsError(rc, lib().kgs_batch_last_error(self.handle).decode())

    def set_graph(self, enable: bool) -> None:
        self._check(lib().kgs_batch_set_graph(self.handle, int(bool(enable))))

    def step(self, nsteps: int) -> "Batch":
        self._check(lib().kgs_batch_step(self.handle, int(nsteps)))
        return self

    def step_each(self, nsteps) -> "Batch":
        if len(nsteps) != len(self.sims):
            raise ValueError("one step count per simulation")
        arr = (ctypes.c_int64 * len(self.sims))(*[int(k) for k in nsteps])
        self._check(lib().kgs_batch_step_each(self.handle, arr))
        return self

    def autotune(self, steps: int = 4, use_cache: bool = True) -> "Batch":
        """Pick the fastest launch configuration of each streaming group
        (kgs_batch_autotune); the states are unchanged."""
        self._check(lib().kgs_batch_autotune(self.handle, int(steps), int(bool(use_cache))))
        return self

    def close(self) -> None:
        if self.handle is not None:
            h, self.handle = self.handle, None
            rc = lib().kgs_batch_free(h)
            if rc != KGS_OK:
                raise KgsError(rc, "kgs_batch_free")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop with continuous batching (kgs_server_*).  Inputs and
    results are numpy arrays on the host."""

    def __init__(self, budget_bytes: int, max_active: int = 0, steps_per_round: int = 50,
                 round_work: int = 0, stream=None):
        cfg = KgsServerConfig(int(budget_bytes), int(max_active), int(steps_per_round),
                              int(round_work))
        if stream is None:
            try:
                stream = int(_torch().cuda.current_stream().cuda_stream)
            except Exception:
                stream = 0
        self.stream = stream
        h = _VP()
        rc = lib().kgs_server_create(ctypes.byref(cfg), stream or None, ctypes.byref(h))
        if rc != KGS_OK:
            raise KgsError(rc, lib().kgs_server_last_error(None).decode())
        self.handle = h
        self.shapes = {}

    def _check(self, rc):
        if rc != KGS_OK:
            raise KgsError(rc, lib().kgs_server_last_error(self.handle).decode())

    def submit(self, cfg: KgsConfig, psi, u, v, nsteps: int) -> int:
        psi = np.asarray(psi)
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (psi.real, psi.imag, u, v)]
        rid = ctypes.c_int64()
        self._check(lib().kgs_server_submit(self.handle, ctypes.byref(cfg),
                                            *[a.ctypes.data for a in arrs], KGS_HOST,
                                            int(nsteps), ctypes.byref(rid)))
        self.shapes[rid.value] = arrs[0].shape
        return rid.value

    def submit_device(self, cfg: KgsConfig, psi_re, psi_im, u, v, nsteps: int) -> int:
        """Submit torch cuda float64 tensors (copied on the device)."""
        rid = ctypes.c_int64()
        self._check(lib().kgs_server_submit(self.handle, ctypes.byref(cfg), psi_re.data_ptr(),
                                            psi_im.data_ptr(), u.data_ptr(), v.data_ptr(),
                                            KGS_DEVICE, int(nsteps), ctypes.byref(rid)))
        self.shapes[rid.value] = tuple(psi_re.shape)
        return rid.value

    def submit_problem(self, problem, nsteps=None) -> int:
        return self.submit(config_of(problem), problem.psi, problem.u, problem.v,
                           problem.steps if nsteps is None else nsteps)

    def run(self, rounds: int = 1):
        nr, nq = ctypes.c_int32(), ctypes.c_int32()
        self._check(lib().kgs_server_run(self.handle, int(rounds), ctypes.byref(nr),
                                         ctypes.byref(nq)))
        return nr.value, nq.value

    def poll(self, rid: int) -> KgsRequestInfo:
        info = KgsRequestInfo()
        self._check(lib().kgs_server_poll(self.handle, int(rid), ctypes.byref(info)))
        return info

    def result(self, rid: int):
        shape = self.shapes[rid]
        arrs = [np.empty(shape, dtype=np.float64) for _ in range(4)]
        self._check(lib().kgs_server_result(self.handle, int(rid), *[a.ctypes.data for a in arrs],
                                            KGS_HOST))
        P, Q, U, V = arrs
        return P + 1j * Q, U, V

    def release(self, rid: int) -> None:
        self._check(lib().kgs_server_release(self.handle, int(rid)))
        self.shapes.pop(rid, None)

    def cancel(self, rid: int) -> None:
        self._check(lib().kgs_server_cancel(self.handle, int(rid)))

    def stats(self) -> KgsServerStats:
        st = KgsServerStats()
        self._check(lib().kgs_server_stats(self.handle, ctypes.byref(st)))
        return st

    def close(self) -> None:
        if self.handle is not None:
            h, self.handle = self.handle, None
            rc = lib().kgs_server_free(h)
            if rc != KGS_OK:
                raise KgsError(rc, "kgs_server_free")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def simulation_from_problem(problem, host: bool = False, tuning=None) -> Simulation:
    return Simulation(config_of(problem), problem.psi, problem.u, problem.v, host=host,
                      tuning=tuning)
