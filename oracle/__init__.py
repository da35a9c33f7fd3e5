"""Python access to the plain FP64 CPU oracle (oracle/hydro_oracle.c).

TEST INFRASTRUCTURE ONLY.  Imported by tests, the smoke check and the
benchmark's CPU-baseline leg; never by the product path.  It shares nothing
with the HIP library: it has its own C source, its own grid description and
its own ctypes binding.  Arrays are numpy float64 in the blocked, guarded
layout ``[nblk, 5, P, P, P]`` (P = n + 2*ng, x fastest).

The method (paper §2 "Software Description": explicit shock-capturing methods
with block-by-block update; §2.2 Hydrodynamics: the predictor-corrector
unsplit compressible solver and the SSP Runge-Kutta one; §2.2 Equations of
State: perfect gas) is
documented function by function in hydro_oracle.h / hydro_oracle.c.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# HYDRO_ORACLE_LIB lets the mutation test load a deliberately broken copy.
LIB_PATH = os.environ.get("HYDRO_ORACLE_LIB", os.path.join(HERE, "libhydro_oracle.so"))

BC_PERIODIC = 0
BC_OUTFLOW = 1

CNT_FLOOR, CNT_FALLBACK, CNT_NONPHYS = 0, 1, 2


class _Grid(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int),
        ("ng", ctypes.c_int),
        ("nb", ctypes.c_int * 3),
        ("dx", ctypes.c_double * 3),
        ("bc", ctypes.c_int * 3),
        ("gamma", ctypes.c_double),
        ("small_p", ctypes.c_double),
    ]


_lib = None


def lib():
    """Load (building first if absent) the oracle's shared library."""
    global _lib
    if _lib is None:
        if "HYDRO_ORACLE_LIB" not in os.environ and (not os.path.exists(LIB_PATH) or (
            os.path.getmtime(LIB_PATH) < os.path.getmtime(os.path.join(HERE, "hydro_oracle.c"))
        )):
            from . import build as _b

            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        gp = ctypes.POINTER(_Grid)
        lp = ctypes.POINTER(ctypes.c_long)
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_block_doubles.argtypes = [gp]
        L.oracle_block_doubles.restype = ctypes.c_size_t
        L.oracle_cons_to_prim.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp]
        L.oracle_cons_to_prim.restype = ctypes.c_int
        L.oracle_van_leer.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_van_leer.restype = ctypes.c_double
        L.oracle_hllc.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double, dp]
        L.oracle_hllc.restype = None
        L.oracle_euler_flux.argtypes = [dp, ctypes.c_int, ctypes.c_double, dp]
        L.oracle_euler_flux.restype = None
        L.oracle_fill_guards_block.argtypes = [gp, dp, ctypes.c_long]
        L.oracle_fill_guards_block.restype = None
        L.oracle_fill_guards.argtypes = [gp, dp]
        L.oracle_fill_guards.restype = None
        L.oracle_step_block.argtypes = [gp, dp, ctypes.c_long, dp, ctypes.c_double, lp]
        L.oracle_step_block.restype = None
        L.oracle_step_block_list.argtypes = [gp, dp, lp, ctypes.c_long, dp, ctypes.c_double, lp]
        L.oracle_step_block_list.restype = None
        L.oracle_step.argtypes = [gp, dp, dp, ctypes.c_double, lp]
        L.oracle_step.restype = None
        L.oracle_step_block_fluxes.argtypes = [gp, dp, ctypes.c_long, dp, ctypes.c_double, dp, dp, dp, lp]
        L.oracle_step_block_fluxes.restype = None
        L.oracle_stage_block.argtypes = [gp, dp, ctypes.c_long, dp, ctypes.c_double, dp, ctypes.c_double,
                                         ctypes.c_double, lp]
        L.oracle_stage_block.restype = None
        L.oracle_step_rk.argtypes = [gp, dp, dp, ctypes.c_double, ctypes.c_int, lp]
        L.oracle_step_rk.restype = ctypes.c_int
        L.oracle_ctu_block.argtypes = [gp, dp, ctypes.c_long, dp, ctypes.c_double, lp]
        L.oracle_ctu_block.restype = None
        L.oracle_step_ctu.argtypes = [gp, dp, dp, ctypes.c_double, lp]
        L.oracle_step_ctu.restype = None
        L.oracle_ctu_char_block.argtypes = [gp, dp, ctypes.c_long, dp, ctypes.c_double, lp]
        L.oracle_ctu_char_block.restype = None
        L.oracle_step_ctu_char.argtypes = [gp, dp, dp, ctypes.c_double, lp]
        L.oracle_step_ctu_char.restype = None
        L.oracle_trace_faces.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp]
        L.oracle_trace_faces.restype = None
        L.oracle_max_signal_dir.argtypes = [gp, dp, ctypes.c_long, ctypes.c_long]
        L.oracle_max_signal_dir.restype = ctypes.c_double
        L.oracle_dt_ctu.argtypes = [gp, dp, ctypes.c_double]
        L.oracle_dt_ctu.restype = ctypes.c_double
        L.oracle_max_signal.argtypes = [gp, dp, ctypes.c_long, ctypes.c_long]
        L.oracle_max_signal.restype = ctypes.c_double
        L.oracle_dt.argtypes = [gp, dp, ctypes.c_double]
        L.oracle_dt.restype = ctypes.c_double
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Grid:
    """Uniform block-structured grid as the oracle sees it."""

    n: int
    nb: Tuple[int, int, int]
    dx: Tuple[float, float, float]
    bc: Tuple[int, int, int] = (BC_PERIODIC, BC_PERIODIC, BC_PERIODIC)
    gamma: float = 1.4
    small_p: float = 1e-10
    ng: int = 4

    @property
    def nblk(self) -> int:
        return self.nb[0] * self.nb[1] * self.nb[2]

    @property
    def P(self) -> int:
        return self.n + 2 * self.ng

    def shape(self):
        return (self.nblk, 5, self.P, self.P, self.P)

    def c(self) -> _Grid:
        g = _Grid()
        g.n, g.ng = self.n, self.ng
        g.nb[:] = list(self.nb)
        g.dx[:] = [float(x) for x in self.dx]
        g.bc[:] = list(self.bc)
        g.gamma, g.small_p = float(self.gamma), float(self.small_p)
        return g

    def check(self, U: np.ndarray) -> None:
        if U.shape != self.shape():
            raise ValueError(f"state shape {U.shape} != {self.shape()}")


def set_threads(n: int) -> int:
    """Host threads for the loops over blocks; returns the previous count."""
    prev = lib().oracle_max_threads()
    lib().oracle_set_threads(int(n))
    return prev


def cons_to_prim(U: Sequence[float], gamma: float, small_p: float = 1e-10):
    """Primitive (rho, u, v, w, p) of one cell and whether the floor was hit."""
    u = np.ascontiguousarray(U, dtype=np.float64)
    w = np.empty(5)
    fl = lib().oracle_cons_to_prim(_dptr(u), gamma, small_p, _dptr(w))
    return w, bool(fl)


def van_leer(dl: float, dr: float) -> float:
    return lib().oracle_van_leer(float(dl), float(dr))


def hllc(WL, WR, d: int, gamma: float) -> np.ndarray:
    a = np.ascontiguousarray(WL, dtype=np.float64)
    b = np.ascontiguousarray(WR, dtype=np.float64)
    f = np.empty(5)
    lib().oracle_hllc(_dptr(a), _dptr(b), int(d), float(gamma), _dptr(f))
    return f


def euler_flux(W, d: int, gamma: float) -> np.ndarray:
    a = np.ascontiguousarray(W, dtype=np.float64)
    f = np.empty(5)
    lib().oracle_euler_flux(_dptr(a), int(d), float(gamma), _dptr(f))
    return f


def fill_guards(g: Grid, U: np.ndarray) -> None:
    """Fill every block's guard layers in place."""
    g.check(U)
    gc = g.c()
    lib().oracle_fill_guards(ctypes.byref(gc), _dptr(U))


def fill_guards_block(g: Grid, U: np.ndarray, b: int) -> None:
    g.check(U)
    gc = g.c()
    lib().oracle_fill_guards_block(ctypes.byref(gc), _dptr(U), int(b))


def step(g: Grid, U: np.ndarray, dt: float):
    """One step: returns (U_new, counters).  U's guards are (re)filled in place;
    the guard layers of U_new are copies of U's (not meaningful)."""
    g.check(U)
    out = U.copy()
    cnt = (ctypes.c_long * 3)(0, 0, 0)
    gc = g.c()
    lib().oracle_step(ctypes.byref(gc), _dptr(U), _dptr(out), float(dt), cnt)
    return out, np.array(list(cnt), dtype=np.int64)


def step_blocks(g: Grid, U: np.ndarray, blocks: Sequence[int], dt: float):
    """New interiors of the listed blocks (guards of those blocks filled first,
    blocks spread over the host cores).  Returns [len(blocks), 5, n, n, n] and
    the summed counters."""
    g.check(U)
    gc = g.c()
    n, ng = g.n, g.ng
    bl = np.ascontiguousarray(blocks, dtype=np.int64)
    tmp = np.empty((len(bl),) + g.shape()[1:])
    cnt = (ctypes.c_long * 3)(0, 0, 0)
    lib().oracle_step_block_list(ctypes.byref(gc), _dptr(U),
                                 bl.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), len(bl),
                                 _dptr(tmp), float(dt), cnt)
    return np.ascontiguousarray(tmp[:, :, ng:ng + n, ng:ng + n, ng:ng + n]), np.array(list(cnt), dtype=np.int64)


def step_rk(g: Grid, U: np.ndarray, dt: float, order: int):
    """One SSP Runge-Kutta step (order 2 or 3) of method-of-lines stages:
    returns (U_new, counters summed over the stages)."""
    g.check(U)
    out = U.copy()
    cnt = (ctypes.c_long * 3)(0, 0, 0)
    gc = g.c()
    rc = lib().oracle_step_rk(ctypes.byref(gc), _dptr(U), _dptr(out), float(dt), int(order), cnt)
    if rc == -1:
        raise ValueError("SSP Runge-Kutta order must be 2 or 3 (got %r)" % (order,))
    if rc != 0:
        raise MemoryError("oracle stage buffers could not be allocated")
    return out, np.array(list(cnt), dtype=np.int64)


def stage_block(g: Grid, U: np.ndarray, b: int, dt: float, U0: np.ndarray = None, a0: float = 0.0,
                a1: float = 0.0):
    """One method-of-lines stage of block b (U's guards must be filled):
    returns block b's new storage (interior updated, guards copied from U)."""
    g.check(U)
    gc = g.c()
    out = np.ascontiguousarray(U[b]).copy()
    cnt = (ctypes.c_long * 3)(0, 0, 0)
    base = None
    if U0 is not None:
        g.check(U0)
        base = np.ascontiguousarray(U0[b])
    lib().oracle_stage_block(ctypes.byref(gc), _dptr(U), int(b), _dptr(out), float(dt),
                             _dptr(base) if base is not None else None, float(a0), float(a1), cnt)
    return out, np.array(list(cnt), dtype=np.int64)


def step_ctu(g: Grid, U: np.ndarray, dt: float, trace: bool = False):
    """One corner-transport-upwind step: returns (U_new, counters).  trace:
    characteristic tracing in the normal predictor."""
    g.check(U)
    out = U.copy()
    cnt = (ctypes.c_long * 3)(0, 0, 0)
    gc = g.c()
    fn = lib().oracle_step_ctu_char if trace else lib().oracle_step_ctu
    fn(ctypes.byref(gc), _dptr(U), _dptr(out), float(dt), cnt)
    return out, np.array(list(cnt), dtype=np.int64)


def step_ctu_blocks(g: Grid, U: np.ndarray, blocks: Sequence[int], dt: float, trace: bool = False):
    """CTU step of the listed blocks only (U's guards are filled here):
    returns (their new interiors [len(blocks), 5, n, n, n], counters)."""
    g.check(U)
    fill_guards(g, U)
    gc = g.c()
    cnt = (ctypes.c_long * 3)(0, 0, 0)
    fn = lib().oracle_ctu_char_block if trace else lib().oracle_ctu_block
    outs = []
    for b in blocks:
        o = np.ascontiguousarray(U[b]).copy()
        fn(ctypes.byref(gc), _dptr(U), int(b), _dptr(o), float(dt), cnt)
        outs.append(o)
    n, ng = g.n, g.ng
    out = np.stack(outs)[:, :, ng:ng + n, ng:ng + n, ng:ng + n]
    return np.ascontiguousarray(out), np.array(list(cnt), dtype=np.int64)


def trace_faces(W, S, d: int, lam: float, gamma: float):
    """Traced (low, high) face states of one cell along d (oracle_trace_faces)."""
    Wa = np.ascontiguousarray(W, dtype=np.float64)
    Sa = np.ascontiguousarray(S, dtype=np.float64)
    lo = np.zeros(5)
    hi = np.zeros(5)
    lib().oracle_trace_faces(_dptr(Wa), _dptr(Sa), int(d), float(lam), float(gamma), _dptr(lo), _dptr(hi))
    return lo, hi


def dt_ctu(g: Grid, U: np.ndarray, cfl: float) -> float:
    """dt of the per-direction CFL rule: cfl / max over cells and d of (|u_d|+c)/dx_d."""
    g.check(U)
    gc = g.c()
    return lib().oracle_dt_ctu(ctypes.byref(gc), _dptr(U), float(cfl))


def max_signal(g: Grid, U: np.ndarray) -> float:
    g.check(U)
    gc = g.c()
    return lib().oracle_max_signal(ctypes.byref(gc), _dptr(U), 0, g.nblk)


def dt(g: Grid, U: np.ndarray, cfl: float) -> float:
    g.check(U)
    gc = g.c()
    return lib().oracle_dt(ctypes.byref(gc), _dptr(U), float(cfl))


def run(g: Grid, U: np.ndarray, nsteps: int, cfl: float = 0.8, callback=None, rk: int = 0, ctu: bool = False,
        trace: bool = False):
    """n repetitions of (dt = CFL/max signal; step(dt)); returns (U, dts, counters).
    rk = 2 or 3 takes SSP Runge-Kutta steps instead of predictor-corrector
    ones; ctu takes corner-transport-upwind steps with the per-direction rule
    (trace: with characteristic tracing)."""
    dts = []
    cnt = np.zeros(3, dtype=np.int64)
    for s in range(nsteps):
        d = dt_ctu(g, U, cfl) if ctu else dt(g, U, cfl)
        if not d > 0:
            raise FloatingPointError("non-positive or non-finite dt at step %d" % s)
        U, c = step_ctu(g, U, d, trace) if ctu else (step_rk(g, U, d, rk) if rk else step(g, U, d))
        cnt += c
        dts.append(d)
        if callback is not None:
            callback(s, U, d)
    return U, np.array(dts), cnt
