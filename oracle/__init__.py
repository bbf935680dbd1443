"""TEST INFRASTRUCTURE ONLY: ctypes binding of the FP64 CPU oracle.

The oracle (``kgs_oracle.c``) is a plain sequential double-precision
implementation of the DP-AVF2 scheme for the periodic Klein-Gordon-Schroedinger
equations (arXiv 2502.09537, sec. 3-4).  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this
package; the GPU library never does and shares no code with it.

All arrays are float64, C-contiguous, of shape ``(n,) * dim`` (axis 0
slowest), and are updated in place.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkgs_oracle.so")
SOURCE = os.path.join(_HERE, "kgs_oracle.c")


class _Grid(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("n", ctypes.c_int32),
        ("h", ctypes.c_double),
        ("kappa1", ctypes.c_double),
        ("kappa2", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("gamma", ctypes.c_double),
    ]


@dataclass(frozen=True)
class Grid:
    """Periodic box [lo, hi)^dim with n points per axis and the KGS parameters."""

    dim: int
    n: int
    lo: float
    hi: float
    kappa1: float = 1.0
    kappa2: float = 1.0
    mu: float = 1.0
    gamma: float = 1.0

    @property
    def h(self) -> float:
        return (self.hi - self.lo) / self.n

    @property
    def shape(self) -> tuple:
        return (self.n,) * self.dim

    def _c(self) -> _Grid:
        return _Grid(self.dim, self.n, self.h, self.kappa1, self.kappa2, self.mu, self.gamma)


_lib = None
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int64)
_GP = ctypes.POINTER(_Grid)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, no FMA contraction)."""
    import subprocess

    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SOURCE):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
             "-shared", "-o", tmp, SOURCE, "-lm"],
            check=True,
        )
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.kgso_is_red.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64]
        L.kgso_is_red.restype = ctypes.c_int32
        L.kgso_psi_update.argtypes = [_GP, ctypes.c_double, _DP, _DP, _DP, ctypes.c_int64]
        L.kgso_psi_update.restype = None
        L.kgso_uv_update.argtypes = [_GP, ctypes.c_double, _DP, _DP, _DP, _DP, ctypes.c_int64]
        L.kgso_uv_update.restype = None
        for name in ("kgso_base_half", "kgso_adjoint_half"):
            f = getattr(L, name)
            f.argtypes = [_GP, ctypes.c_double, _DP, _DP, _DP, _DP, _IP, ctypes.c_int64]
            f.restype = None
        L.kgso_step_order.argtypes = [_GP, ctypes.c_double, _DP, _DP, _DP, _DP, _IP, ctypes.c_int64]
        L.kgso_step_order.restype = ctypes.c_int
        L.kgso_checkerboard_order.argtypes = [ctypes.c_int32, ctypes.c_int32, _IP]
        L.kgso_checkerboard_order.restype = ctypes.c_int64
        L.kgso_step.argtypes = [_GP, ctypes.c_double, _DP, _DP, _DP, _DP, ctypes.c_int64]
        L.kgso_step.restype = ctypes.c_int
        L.kgso_step_passes.argtypes = [_GP, ctypes.c_double, _DP, _DP, _DP, _DP, ctypes.c_int64,
                                       ctypes.c_int32, ctypes.c_int32]
        L.kgso_step_passes.restype = ctypes.c_int
        L.kgso_energy.argtypes = [_GP, _DP, _DP, _DP, _DP]
        L.kgso_energy.restype = ctypes.c_double
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    if a.dtype != np.float64 or not a.flags.c_contiguous:
        raise TypeError("oracle arrays must be C-contiguous float64")
    return a.ctypes.data_as(_DP)


def _check(grid: Grid, *arrays):
    for a in arrays:
        if a.size != grid.n ** grid.dim:
            raise ValueError("array size does not match the grid")


class State:
    """The four real fields (P, Q, U, V) = (Re psi, Im psi, u, u_t)."""

    def __init__(self, P, Q, U, V):
        self.P = np.ascontiguousarray(P, dtype=np.float64).copy()
        self.Q = np.ascontiguousarray(Q, dtype=np.float64).copy()
        self.U = np.ascontiguousarray(U, dtype=np.float64).copy()
        self.V = np.ascontiguousarray(V, dtype=np.float64).copy()

    @classmethod
    def from_fields(cls, psi, u, v):
        psi = np.asarray(psi)
        return cls(psi.real, psi.imag, u, v)

    def copy(self) -> "State":
        return State(self.P, self.Q, self.U, self.V)

    def arrays(self):
        return self.P, self.Q, self.U, self.V

    @property
    def psi(self):
        return self.P + 1j * self.Q


def is_red(dim: int, n: int, idx: int) -> bool:
    return bool(lib().kgso_is_red(dim, n, idx))


def checkerboard_order(dim: int, n: int) -> np.ndarray:
    order = np.empty(n ** dim, dtype=np.int64)
    lib().kgso_checkerboard_order(dim, n, order.ctypes.data_as(_IP))
    return order


def block_splitting_rows(n: int, n_proc: int):
    """Row partition of Algorithm 2 (sec. 4.2) on an n x n grid, 0-based
    rows along axis 0: row 0 is the first boundary row (j_0), and the other
    n - 1 rows are n_proc blocks, each followed by one separator row
    (j_1, ..., j_{n_proc}; the last separator is row n - 1, the periodic
    neighbour of row 0).  The n - 1 - n_proc block rows are shared as evenly
    as possible.  Returns (blocks, separators): a list of row ranges and the
    list of separator rows."""
    if n_proc < 1 or n - 1 - n_proc < n_proc:
        raise ValueError("every block needs at least one row")
    inner = n - 1 - n_proc
    blocks, seps, row = [], [], 1
    for l in range(n_proc):
        size = inner // n_proc + (1 if l < inner % n_proc else 0)
        blocks.append(range(row, row + size))
        seps.append(row + size)
        row += size + 1
    assert row == n and seps[-1] == n - 1
    return blocks, seps


def block_splitting_order(n: int, n_proc: int, block_sequence=None) -> np.ndarray:
    """The serial update order that the block-splitting strategy of
    Algorithm 2 executes on a 2-D n x n grid (linear index row * n + col):
    the boundary row j_0, then every block row by row (the blocks are
    independent, so `block_sequence` may list them in any order, which is
    what running them in parallel amounts to), then the separator rows in
    ascending order; columns ascending within a row.  The adjoint half step
    visits the same points in reverse, as Algorithm 2 does."""
    blocks, seps = block_splitting_rows(n, n_proc)
    seq = range(n_proc) if block_sequence is None else block_sequence
    rows = [0] + [r for l in seq for r in blocks[l]] + seps
    return np.array([r * n + c for r in rows for c in range(n)], dtype=np.int64)


def step(grid: Grid, tau: float, s: State, nsteps: int = 1) -> State:
    """nsteps DP-AVF2 steps in the checkerboard order, in place."""
    _check(grid, *s.arrays())
    g = grid._c()
    rc = lib().kgso_step(ctypes.byref(g), tau, *map(_ptr, s.arrays()), nsteps)
    if rc != 0:
        raise RuntimeError(f"kgso_step failed ({rc})")
    return s


def step_passes(grid: Grid, tau: float, s: State, nsteps: int = 1, storage_bits: int = 64,
                threads: int = 1) -> State:
    """nsteps checkerboard DP-AVF2 steps written colour pass by colour pass,
    in place: bitwise equal to step() for storage_bits=64 and any number of
    OpenMP threads; storage_bits=32 rounds the values to float32 where a
    float32 state is stored (on entry, after each red pass, after the blue
    adjoint pass), with float64 arithmetic throughout.  n must be even."""
    _check(grid, *s.arrays())
    g = grid._c()
    rc = lib().kgso_step_passes(ctypes.byref(g), tau, *map(_ptr, s.arrays()), nsteps,
                                storage_bits, threads)
    if rc != 0:
        raise RuntimeError(f"kgso_step_passes failed ({rc})")
    return s


def step_order(grid: Grid, tau: float, s: State, order: np.ndarray, nsteps: int = 1) -> State:
    """nsteps DP-AVF2 steps for an arbitrary grid-point update order, in place."""
    _check(grid, *s.arrays())
    order = np.ascontiguousarray(order, dtype=np.int64)
    if sorted(order.tolist()) != list(range(grid.n ** grid.dim)):
        raise ValueError("order must be a permutation of all grid points")
    g = grid._c()
    rc = lib().kgso_step_order(ctypes.byref(g), tau, *map(_ptr, s.arrays()),
                               order.ctypes.data_as(_IP), nsteps)
    if rc != 0:
        raise RuntimeError(f"kgso_step_order failed ({rc})")
    return s


def base_half(grid: Grid, tau_half: float, s: State, order: np.ndarray) -> State:
    order = np.ascontiguousarray(order, dtype=np.int64)
    g = grid._c()
    lib().kgso_base_half(ctypes.byref(g), tau_half, *map(_ptr, s.arrays()),
                         order.ctypes.data_as(_IP), order.size)
    return s


def adjoint_half(grid: Grid, tau_half: float, s: State, order: np.ndarray) -> State:
    order = np.ascontiguousarray(order, dtype=np.int64)
    g = grid._c()
    lib().kgso_adjoint_half(ctypes.byref(g), tau_half, *map(_ptr, s.arrays()),
                            order.ctypes.data_as(_IP), order.size)
    return s


def psi_update(grid: Grid, tau_half: float, s: State, idx: int) -> State:
    g = grid._c()
    lib().kgso_psi_update(ctypes.byref(g), tau_half, _ptr(s.P), _ptr(s.Q), _ptr(s.U), int(idx))
    return s


def uv_update(grid: Grid, tau_half: float, s: State, idx: int) -> State:
    g = grid._c()
    lib().kgso_uv_update(ctypes.byref(g), tau_half, _ptr(s.P), _ptr(s.Q), _ptr(s.U), _ptr(s.V),
                         int(idx))
    return s


def energy(grid: Grid, s: State) -> float:
    """h^dim times the discrete energy E_h (sec. 2), Neumaier-compensated."""
    _check(grid, *s.arrays())
    g = grid._c()
    return float(lib().kgso_energy(ctypes.byref(g), *map(_ptr, s.arrays())))
