"""Thin Python binding of libhydro.so (C ABI declared in include/hydro.h).

Argument marshalling only: torch provides device memory and the stream, every
step of the computation runs in the library's HIP kernels.  Loading fails
loudly (``HydroLibraryMissing``) when the library has not been built; there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# HYDRO_LIB points the binding at another build of the same library (kernel experiments)
LIB_PATH = os.environ.get("HYDRO_LIB") or os.path.join(HERE, "libhydro.so")

HYDRO_OK = 0
HYDRO_EINVAL = -1
HYDRO_ESIZE = -2
HYDRO_EDEVICE = -3
HYDRO_ENONPHYS = -4
BC_PERIODIC = 0
BC_OUTFLOW = 1
NGUARD = 4
SCHEME_MH, SCHEME_RK2, SCHEME_RK3, SCHEME_CTU, SCHEME_CTU_CHAR = 0, 2, 3, 4, 5

# Every entry point include/hydro.h declares, with its ctypes signature.
_dp = ctypes.POINTER(ctypes.c_double)


class Desc(ctypes.Structure):
    """hydro_grid_desc."""

    _fields_ = [
        ("nxb", ctypes.c_int),
        ("nguard", ctypes.c_int),
        ("nblk", ctypes.c_int * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("bc", ctypes.c_int * 3),
        ("gamma", ctypes.c_double),
        ("small_p", ctypes.c_double),
        ("U", ctypes.c_void_p),
        ("U_alt", ctypes.c_void_p),
        ("work", ctypes.c_void_p),
        ("work_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
    ]


_DP = ctypes.POINTER(Desc)
_HP = ctypes.c_void_p
SIGNATURES = {
    "hydro_state_doubles": ([_DP], ctypes.c_size_t),
    "hydro_guarded_doubles": ([_DP], ctypes.c_size_t),
    "hydro_work_bytes": ([_DP], ctypes.c_size_t),
    "hydro_init_grid": ([_DP, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "hydro_fill_guards": ([_HP, ctypes.c_void_p], ctypes.c_int),
    "hydro_step": ([_HP, ctypes.c_double], ctypes.c_int),
    "hydro_step_cfl": ([_HP, ctypes.c_double], ctypes.c_int),
    "hydro_dt": ([_HP, ctypes.c_double, _dp], ctypes.c_int),
    "hydro_last_dt": ([_HP, _dp], ctypes.c_int),
    "hydro_state_changed": ([_HP], ctypes.c_int),
    "hydro_current": ([_HP, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "hydro_counters": ([_HP, ctypes.POINTER(ctypes.c_longlong)], ctypes.c_int),
    "hydro_free_grid": ([_HP], ctypes.c_int),
    "hydro_set_pencils": ([_HP, ctypes.c_int], ctypes.c_int),
    "hydro_amr_fine_blocks": ([ctypes.c_void_p], ctypes.c_size_t),
    "hydro_amr_levels": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_long)], ctypes.c_int),
    "hydro_amr_work_bytes": ([ctypes.c_void_p], ctypes.c_size_t),
    "hydro_amr_create": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "hydro_amr_step": ([ctypes.c_void_p, ctypes.c_double], ctypes.c_int),
    "hydro_amr_step_cfl": ([ctypes.c_void_p, ctypes.c_double], ctypes.c_int),
    "hydro_amr_last_dt": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "hydro_amr_state_changed": ([ctypes.c_void_p], ctypes.c_int),
    "hydro_amr_dt": ([ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "hydro_amr_counters": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_longlong)], ctypes.c_int),
    "hydro_amr_estimate": ([ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_ubyte)], ctypes.c_int),
    "hydro_amr_transfer": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "hydro_amr_estimate_tree": ([ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_ubyte), ctypes.c_size_t,
                                 ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "hydro_amr_set_columns": ([ctypes.c_void_p, ctypes.c_int], ctypes.c_int),
    "hydro_amr_free": ([ctypes.c_void_p], ctypes.c_int),
    "hydro_set_pencil_planes": ([_HP, ctypes.c_int], ctypes.c_int),
    "hydro_set_tile": ([_HP, ctypes.c_int], ctypes.c_int),
    "hydro_set_scheme": ([_HP, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "hydro_set_buffers": ([_HP, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "hydro_batch_work_bytes": ([ctypes.POINTER(ctypes.c_void_p), ctypes.c_int], ctypes.c_size_t),
    "hydro_batch_create": ([ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                            ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "hydro_batch_step": ([_HP, ctypes.c_double, ctypes.c_int], ctypes.c_int),
    "hydro_batch_set_active": ([_HP, ctypes.POINTER(ctypes.c_ubyte)], ctypes.c_int),
    "hydro_batch_set_pencils": ([_HP, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "hydro_batch_set_workgroups": ([_HP, ctypes.c_int], ctypes.c_int),
    "hydro_batch_set_tiles": ([_HP, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "hydro_batch_use_graph": ([_HP, ctypes.c_int], ctypes.c_int),
    "hydro_batch_dts": ([_HP, _dp], ctypes.c_int),
    "hydro_batch_free": ([_HP], ctypes.c_int),
    "hydro_batch_step_static": ([ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                 ctypes.c_double, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "hydro_copy_probe": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "hydro_last_error": ([], ctypes.c_char_p),
}


class HydroLibraryMissing(ImportError):
    pass


class HydroError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libhydro error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded libhydro.so (raises HydroLibraryMissing if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise HydroLibraryMissing(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        # torch first: the library then binds to the HIP runtime torch has
        # loaded (one runtime per process), whatever the import order.
        import torch  # noqa: F401

        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc != HYDRO_OK:
        raise HydroError(rc, lib().hydro_last_error().decode())
    return rc


def make_desc(nxb: int, nblk: Sequence[int], lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
              bc=(BC_PERIODIC,) * 3, gamma: float = 1.4, small_p: float = 1e-10,
              nguard: int = NGUARD) -> Desc:
    d = Desc()
    d.nxb, d.nguard = int(nxb), int(nguard)
    d.nblk[:] = [int(x) for x in nblk]
    d.lo[:] = [float(x) for x in lo]
    d.hi[:] = [float(x) for x in hi]
    d.bc[:] = [int(x) for x in bc]
    d.gamma, d.small_p = float(gamma), float(small_p)
    return d


class Grid:
    """A grid handle over two torch state tensors and a workspace tensor.

    State tensors have the compact shape ``[nblk, 5, nxb, nxb, nxb]``,
    float64, on ``device``; the current one is ``self.state``."""

    def __init__(self, nxb: int, nblk: Sequence[int], lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                 bc=(BC_PERIODIC,) * 3, gamma: float = 1.4, small_p: float = 1e-10,
                 device: str = "cuda", stream=None, nguard: int = NGUARD, buffers=None):
        import torch

        L = lib()
        self._torch = torch
        self.nxb, self.nblk = int(nxb), tuple(int(x) for x in nblk)
        self.nguard = int(nguard)
        self.tile = 8 if self.nxb == 8 else 16
        d = make_desc(nxb, nblk, lo, hi, bc, gamma, small_p, nguard)
        nd = L.hydro_state_doubles(ctypes.byref(d))
        n = self.nxb
        nb = self.nblk[0] * self.nblk[1] * self.nblk[2]
        if nd != nb * 5 * n ** 3:
            raise HydroError(HYDRO_EINVAL, "invalid grid shape")
        self.shape = (nb, 5, n, n, n)
        P = n + 2 * self.nguard
        self.guarded_shape = (nb, 5, P, P, P)
        if buffers is None:
            self.bufs = [torch.empty(self.shape, dtype=torch.float64, device=device) for _ in range(2)]
        else:
            self.bufs = list(buffers)
            for t_ in self.bufs:
                if tuple(t_.shape) != self.shape or t_.dtype != torch.float64 or not t_.is_contiguous():
                    raise HydroError(HYDRO_EINVAL, "state buffers must be contiguous float64 of the grid shape")
        wb = L.hydro_work_bytes(ctypes.byref(d))
        self.work = torch.zeros(max(wb, 256), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.bufs[0].device)
        d.U = self.bufs[0].data_ptr()
        d.U_alt = self.bufs[1].data_ptr()
        d.work = self.work.data_ptr()
        d.work_bytes = self.work.numel()
        d.stream = self.stream.cuda_stream
        self.desc = d
        h = ctypes.c_void_p()
        _check(L.hydro_init_grid(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h

    # -- state access ---------------------------------------------------------
    @property
    def state(self):
        if not self.bufs:
            raise HydroError(HYDRO_EINVAL, "state buffers were released; rebind them with set_buffers")
        p = ctypes.c_void_p()
        _check(lib().hydro_current(self.handle, ctypes.byref(p)))
        return self.bufs[0] if p.value == self.bufs[0].data_ptr() else self.bufs[1]

    def upload(self, U: np.ndarray) -> None:
        """Copy a host state (compact blocked layout) into the current buffer."""
        t = self._torch.from_numpy(np.ascontiguousarray(U, dtype=np.float64))
        with self._torch.cuda.stream(self.stream):
            self.state.copy_(t, non_blocking=False)
        _check(lib().hydro_state_changed(self.handle))

    def download(self) -> np.ndarray:
        self.stream.synchronize()
        return self.state.cpu().numpy()

    # -- the operations ---------------------------------------------------------
    def fill_guards(self, out=None):
        """Guarded view [nblk, 5, P, P, P] of the current state (a torch tensor)."""
        if out is None:
            out = self._torch.empty(self.guarded_shape, dtype=self._torch.float64, device=self.bufs[0].device)
        _check(lib().hydro_fill_guards(self.handle, out.data_ptr()))
        return out

    def step(self, dt: float) -> None:
        _check(lib().hydro_step(self.handle, float(dt)))

    def step_cfl(self, cfl: float) -> None:
        _check(lib().hydro_step_cfl(self.handle, float(cfl)))

    def dt(self, cfl: float) -> float:
        out = ctypes.c_double()
        _check(lib().hydro_dt(self.handle, float(cfl), ctypes.byref(out)))
        return out.value

    def last_dt(self) -> float:
        out = ctypes.c_double()
        _check(lib().hydro_last_dt(self.handle, ctypes.byref(out)))
        return out.value

    def counters(self) -> np.ndarray:
        out = (ctypes.c_longlong * 3)()
        _check(lib().hydro_counters(self.handle, out))
        return np.array(list(out), dtype=np.int64)

    def set_pencils(self, nseg: int) -> None:
        _check(lib().hydro_set_pencils(self.handle, int(nseg)))

    def set_pencil_planes(self, planes: int) -> None:
        _check(lib().hydro_set_pencil_planes(self.handle, int(planes)))

    def set_tile(self, tile: int) -> None:
        """Column tile edge of the step's workgroups (8 or 16)."""
        _check(lib().hydro_set_tile(self.handle, int(tile)))
        self.tile = int(tile)

    def set_scheme(self, scheme: int, stage=None) -> None:
        """Time integration: SCHEME_MH (predictor-corrector), SCHEME_RK2 or
        SCHEME_RK3 (SSP Runge-Kutta over method-of-lines stages), SCHEME_CTU
        (corner transport upwind), SCHEME_CTU_CHAR (the same with
        characteristic tracing).  RK3 needs a third state tensor; one is
        allocated when `stage` is None."""
        torch = self._torch
        if scheme == SCHEME_RK3:
            if stage is None:
                stage = torch.empty(self.shape, dtype=torch.float64, device=self.bufs[0].device)
            if tuple(stage.shape) != self.shape or not stage.is_contiguous():
                raise HydroError(HYDRO_EINVAL, "stage buffer must be a contiguous tensor of the grid shape")
        else:
            stage = None
        ptr = stage.data_ptr() if stage is not None else None
        _check(lib().hydro_set_scheme(self.handle, int(scheme), ptr))
        self.stage_buf = stage
        self.scheme = int(scheme)

    def set_buffers(self, U, U_alt) -> None:
        """Rebind the state buffers: U holds the current state, U_alt receives
        the next step (torch float64 tensors of the grid shape)."""
        for t_ in (U, U_alt):
            if tuple(t_.shape) != self.shape or not t_.is_contiguous():
                raise HydroError(HYDRO_EINVAL, "state buffers must be contiguous tensors of the grid shape")
        _check(lib().hydro_set_buffers(self.handle, U.data_ptr(), U_alt.data_ptr()))
        self.bufs = [U, U_alt]

    def release_buffers(self) -> None:
        """Drop this object's references to the state tensors (a caller that
        owns them elsewhere, e.g. a serving loop, lets them go back to the
        allocator).  Rebind with set_buffers before the next step."""
        self.bufs = []

    def close(self) -> None:
        if getattr(self, "handle", None) is not None:
            lib().hydro_free_grid(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_step_static(grids, cfl: float, nsteps: int = 1, nseg=None, stream=None) -> None:
    """nsteps batched steps of the grids without a batch workspace
    (hydro_batch_step_static: the tables live in the library's static device
    scratch).  stream: a torch stream (default: the current one); it is
    ordered after the work queued on the grids' streams, and the grids'
    streams after it, so later calls on a grid see the new state."""
    import torch

    grids = list(grids)
    n = len(grids)
    arr = (ctypes.c_void_p * max(n, 1))(*[g.handle.value for g in grids])
    s = stream if stream is not None else torch.cuda.current_stream(grids[0].bufs[0].device if n else None)
    for g in grids:
        if g.stream != s:
            s.wait_stream(g.stream)
    segs = None if nseg is None else (ctypes.c_int * 3)(*[int(x) for x in nseg])
    _check(lib().hydro_batch_step_static(arr, n, segs, float(cfl), int(nsteps), s.cuda_stream))
    for g in grids:
        if g.stream != s:
            g.stream.wait_stream(s)


class Batch:
    """Many grids stepped by one persistent launch per step (hydro_batch_*)."""

    def __init__(self, grids, stream=None):
        import torch

        L = lib()
        self.grids = list(grids)
        n = len(self.grids)
        arr = (ctypes.c_void_p * n)(*[g.handle.value for g in self.grids])
        wb = L.hydro_batch_work_bytes(arr, n)
        if wb == 0:
            raise HydroError(HYDRO_EINVAL, "invalid batch")
        dev = self.grids[0].bufs[0].device
        self.work = torch.zeros(wb, dtype=torch.uint8, device=dev)
        # a stream of its own (graph capture cannot use the null stream),
        # ordered after the work already queued on the members' streams
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        for g in self.grids:
            self.stream.wait_stream(g.stream)
        h = ctypes.c_void_p()
        _check(L.hydro_batch_create(arr, n, self.work.data_ptr(), wb, self.stream.cuda_stream, ctypes.byref(h)))
        self.handle = h

    def step(self, cfl: float, nsteps: int = 1) -> None:
        _check(lib().hydro_batch_step(self.handle, float(cfl), int(nsteps)))

    def synchronize(self) -> None:
        """Wait for the batch's work; later work on the members' streams is
        ordered after it too."""
        self.stream.synchronize()

    def set_active(self, mask) -> None:
        m = (ctypes.c_ubyte * len(self.grids))(*[1 if x else 0 for x in mask])
        _check(lib().hydro_batch_set_active(self.handle, m))

    def set_pencils(self, nseg8: int, nseg16: int, nseg32: int) -> None:
        a = (ctypes.c_int * 3)(int(nseg8), int(nseg16), int(nseg32))
        _check(lib().hydro_batch_set_pencils(self.handle, a))

    def set_workgroups(self, per_cu: int) -> None:
        _check(lib().hydro_batch_set_workgroups(self.handle, int(per_cu)))

    def set_tiles(self, t8: int, t16: int, t32: int) -> None:
        a = (ctypes.c_int * 3)(int(t8), int(t16), int(t32))
        _check(lib().hydro_batch_set_tiles(self.handle, a))

    def use_graph(self, enable: bool = True) -> None:
        _check(lib().hydro_batch_use_graph(self.handle, 1 if enable else 0))

    def dts(self) -> np.ndarray:
        out = (ctypes.c_double * len(self.grids))()
        _check(lib().hydro_batch_dts(self.handle, out))
        return np.array(list(out))

    def close(self) -> None:
        if getattr(self, "handle", None) is not None:
            lib().hydro_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def copy_probe(src, dst, stream=None) -> None:
    """Streaming copy of src into dst (float64 torch tensors, same size)."""
    import torch

    if src.dtype != torch.float64 or dst.dtype != torch.float64 or src.numel() != dst.numel():
        raise ValueError("copy_probe needs two float64 tensors of the same size")
    st = stream if stream is not None else torch.cuda.current_stream(src.device)
    _check(lib().hydro_copy_probe(src.data_ptr(), dst.data_ptr(), src.numel(), st.cuda_stream))


def grid_for(problem, device: str = "cuda", stream=None) -> Grid:
    """A Grid shaped for an ``ics.Problem`` with its initial state uploaded."""
    lo = problem.lo
    hi = problem.hi
    g = Grid(problem.n, problem.nb, lo, hi, problem.bc, problem.gamma, problem.small_p,
             device=device, stream=stream, nguard=problem.ng)
    g.upload(problem.Uc)
    return g


class _AmrDesc(ctypes.Structure):
    _fields_ = [
        ("nxb", ctypes.c_int), ("nguard", ctypes.c_int), ("nblk", ctypes.c_int * 3),
        ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3), ("bc", ctypes.c_int * 3),
        ("gamma", ctypes.c_double), ("small_p", ctypes.c_double),
        ("refine", ctypes.POINTER(ctypes.c_ubyte)),
        ("Ur", ctypes.c_void_p), ("Uf", ctypes.c_void_p),
        ("work", ctypes.c_void_p), ("work_bytes", ctypes.c_size_t), ("stream", ctypes.c_void_p),
        ("refine_deep", ctypes.POINTER(ctypes.c_ubyte)), ("nrefine_deep", ctypes.c_size_t),
    ]


def make_amr_desc(nxb, nblk, refine, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), bc=(BC_PERIODIC,) * 3,
                  gamma=1.4, small_p=1e-10, nguard=NGUARD, refine_deep=()):
    d = _AmrDesc()
    d.nxb, d.nguard = int(nxb), int(nguard)
    d.nblk[:] = [int(x) for x in nblk]
    d.lo[:] = [float(x) for x in lo]
    d.hi[:] = [float(x) for x in hi]
    d.bc[:] = [int(x) for x in bc]
    d.gamma, d.small_p = float(gamma), float(small_p)
    flags = (ctypes.c_ubyte * len(refine))(*[1 if f else 0 for f in refine])
    d.refine = ctypes.cast(flags, ctypes.POINTER(ctypes.c_ubyte))
    deep = (ctypes.c_ubyte * max(len(refine_deep), 1))(*[1 if f else 0 for f in refine_deep])
    d.refine_deep = ctypes.cast(deep, ctypes.POINTER(ctypes.c_ubyte)) if len(refine_deep) else None
    d.nrefine_deep = len(refine_deep)
    d._flags = (flags, deep)  # keep the host arrays alive with the descriptor
    return d


class Amr:
    """Block-structured AMR mesh over torch state tensors (hydro_amr_*).

    Ur: root state [nroot, 5, n, n, n]; Uf: the blocks of levels 1, 2, ...
    concatenated (each level: the children of the previous level's refined
    blocks in increasing block index); level_blocks: blocks per level.
    refine: level-0 flags; refine_deep: flags of levels 1, 2, ... concatenated."""

    def __init__(self, nxb, nblk, refine, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), bc=(BC_PERIODIC,) * 3,
                 gamma=1.4, small_p=1e-10, device="cuda", stream=None, refine_deep=()):
        import torch

        L = lib()
        self._torch = torch
        d = make_amr_desc(nxb, nblk, refine, lo, hi, bc, gamma, small_p, refine_deep=refine_deep)
        counts = (ctypes.c_long * 8)()
        nlev = L.hydro_amr_levels(ctypes.byref(d), counts)
        if nlev < 1:
            raise HydroError(nlev, "invalid AMR descriptor")
        self.level_blocks = [int(counts[l]) for l in range(nlev)]
        self.refine_deep = [bool(f) for f in refine_deep]
        self.nxb, self.nblk, self.refine = int(nxb), tuple(int(x) for x in nblk), [bool(f) for f in refine]
        self.lo, self.hi, self.bc = tuple(lo), tuple(hi), tuple(bc)
        self.gamma, self.small_p = float(gamma), float(small_p)
        nfine = L.hydro_amr_fine_blocks(ctypes.byref(d))
        n = int(nxb)
        nroot = int(nblk[0]) * int(nblk[1]) * int(nblk[2])
        self.Ur = torch.zeros((nroot, 5, n, n, n), dtype=torch.float64, device=device)
        self.Uf = torch.zeros((max(nfine, 1), 5, n, n, n), dtype=torch.float64, device=device)
        self.nfine = nfine
        wb = L.hydro_amr_work_bytes(ctypes.byref(d))
        if wb == 0:
            raise HydroError(HYDRO_EINVAL, "invalid AMR descriptor")
        self.work = torch.zeros(wb, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.Ur.device)
        d.Ur, d.Uf = self.Ur.data_ptr(), self.Uf.data_ptr()
        d.work, d.work_bytes = self.work.data_ptr(), self.work.numel()
        d.stream = self.stream.cuda_stream
        self.desc = d
        h = ctypes.c_void_p()
        _check(L.hydro_amr_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h

    def upload(self, Ur, Uf=None) -> None:
        t = self._torch
        with t.cuda.stream(self.stream):
            self.Ur.copy_(t.from_numpy(np.ascontiguousarray(Ur, dtype=np.float64)))
            if Uf is not None and self.nfine:
                self.Uf.copy_(t.from_numpy(np.ascontiguousarray(Uf, dtype=np.float64)))
        self.stream.synchronize()
        _check(lib().hydro_amr_state_changed(self.handle))

    def download(self):
        self.stream.synchronize()
        return self.Ur.cpu().numpy(), self.Uf[:self.nfine].cpu().numpy()

    def step(self, dt: float) -> None:
        _check(lib().hydro_amr_step(self.handle, float(dt)))

    def step_cfl(self, cfl: float) -> None:
        """One step whose dt is formed on the device from the CFL rule."""
        _check(lib().hydro_amr_step_cfl(self.handle, float(cfl)))

    def last_dt(self) -> float:
        out = ctypes.c_double()
        _check(lib().hydro_amr_last_dt(self.handle, ctypes.byref(out)))
        return out.value

    def dt(self, cfl: float) -> float:
        out = ctypes.c_double()
        _check(lib().hydro_amr_dt(self.handle, float(cfl), ctypes.byref(out)))
        return out.value

    def counters(self) -> np.ndarray:
        out = (ctypes.c_longlong * 3)()
        _check(lib().hydro_amr_counters(self.handle, out))
        return np.array(list(out), dtype=np.int64)

    def set_columns(self, cap: int) -> None:
        """Leaf-step pencils over columns of up to cap z-stacked leaves (1, 2
        or 4), or chosen per leaf list (0); results do not depend on it."""
        _check(lib().hydro_amr_set_columns(self.handle, int(cap)))

    def estimate(self, eps: float = 0.01, refine_cutoff: float = 0.8, derefine_cutoff: float = 0.2):
        """(new refinement flags, per-root-block indicator E^2) from the
        current state (hydro_amr_estimate)."""
        n = len(self.refine)
        E2 = (ctypes.c_double * n)()
        flags = (ctypes.c_ubyte * n)()
        _check(lib().hydro_amr_estimate(self.handle, float(eps), float(refine_cutoff), float(derefine_cutoff),
                                        E2, flags))
        return np.array(list(flags), dtype=bool), np.array(list(E2))

    def estimate_tree(self, eps: float = 0.01, refine_cutoff: float = 0.8, derefine_cutoff: float = 0.2,
                      max_levels: int = 3):
        """(level-0 flags, deeper flags, per-level indicators) of the rule for
        meshes of any depth (hydro_amr_estimate_tree)."""
        nall = sum(self.level_blocks)
        E2 = (ctypes.c_double * nall)()
        need = ctypes.c_size_t()
        lib().hydro_amr_estimate_tree(self.handle, float(eps), float(refine_cutoff), float(derefine_cutoff),
                                      int(max_levels), E2, None, 0, ctypes.byref(need))
        flags = (ctypes.c_ubyte * max(need.value, 1))()
        _check(lib().hydro_amr_estimate_tree(self.handle, float(eps), float(refine_cutoff), float(derefine_cutoff),
                                             int(max_levels), E2, flags, need.value, ctypes.byref(need)))
        f = np.array(list(flags)[:need.value], dtype=bool)
        nroot = len(self.refine)
        per_level, o = [], 0
        for nb in self.level_blocks:
            per_level.append(np.array(list(E2)[o:o + nb]))
            o += nb
        return f[:nroot], f[nroot:], per_level

    def regrid(self, flags, refine_deep=()) -> "Amr":
        """A new mesh over the same root grid with level-0 flags `flags` and
        deeper flags `refine_deep`, its state transferred from this one
        (hydro_amr_transfer); this mesh is closed."""
        new = Amr(self.nxb, self.nblk, [bool(f) for f in flags], self.lo, self.hi, self.bc, self.gamma,
                  self.small_p, device=self.Ur.device, stream=self.stream,
                  refine_deep=[bool(f) for f in refine_deep])
        _check(lib().hydro_amr_transfer(self.handle, new.handle))
        self.close()
        return new

    def close(self) -> None:
        if getattr(self, "handle", None) is not None:
            lib().hydro_amr_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
