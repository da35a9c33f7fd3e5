"""Two-level static AMR step of the CPU oracle (test infrastructure only).

The paper's Grid unit manages a block-structured mesh with adaptive
refinement (§2 Software Description): blocks of nxb^3 cells, guard cells
filled across refinement jumps, fluxes reconciled at fine-coarse faces.
Here a root grid of blocks (level 0) is refined block by block into eight
children at half the cell size (level 1), statically, and every leaf block
takes the same step of size dt:

  1. guard fill of each leaf (4 layers):
     * level-0 leaves: the same-level map over the root array, whose refined
       blocks hold the restriction of their children;
     * level-1 leaves: a guard cell whose position lies in a refined root
       block copies that fine cell; otherwise it is prolonged from the root
       cell under it: U_c + sum_d S_d * (+-1/4), S_d the van Leer slope of the
       conserved variable over the root cells d-1, d, d+1 (the level-0 map),
       the sign that of the fine cell's offset from the root cell's centre;
       a prolonged state with rho <= 0 or p <= 0 takes U_c itself;
     (positions beyond the domain are mapped at the guard cell's own level:
     periodic or outflow, per axis);
  2. the predictor-corrector step of every leaf (oracle_step_block_fluxes)
     with lam = dt/dx of its level;
  3. refluxing: on each face between an unrefined root block and a refined
     one, the root cell next to the face replaces its own face flux by the
     mean of the four fine fluxes over the face;
  4. restriction: each refined root block takes the mean of its children's
     eight cells per root cell.
The composite's conserved totals (leaf cells weighted by their volume) are
unchanged by a step on a periodic domain (refluxing makes the fine-coarse
faces conservative).  dt = CFL / max over leaves of the summed signal
speed with each level's dx.

Layout: root state [nroot, 5, n, n, n] (compact, block id
b = bx + nb0*(by + nb1*bz)); fine state [nfine, 5, n, n, n], the children of
the refined root blocks in increasing root id, child c = cx + 2*cy + 4*cz
covering cells (cx*n/2.., cy*n/2.., cz*n/2..) of its parent.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Tuple

import numpy as np

from . import BC_PERIODIC, Grid, _dptr, lib

NG = 4


@dataclass
class Mesh:
    n: int
    nb: Tuple[int, int, int]
    dx: Tuple[float, float, float]           # root cell widths
    refine: np.ndarray                        # bool per root block
    bc: Tuple[int, int, int] = (BC_PERIODIC,) * 3
    gamma: float = 1.4
    small_p: float = 1e-10

    def __post_init__(self):
        self.refine = np.asarray(self.refine, dtype=bool).reshape(-1)
        assert self.refine.size == self.nroot
        assert self.n % 2 == 0
        self.refined = np.flatnonzero(self.refine)
        self.child_base = -np.ones(self.nroot, dtype=np.int64)
        self.child_base[self.refined] = 8 * np.arange(self.refined.size)

    @property
    def nroot(self):
        return self.nb[0] * self.nb[1] * self.nb[2]

    @property
    def nfine(self):
        return 8 * int(self.refine.sum())

    def root_grid(self) -> Grid:
        return Grid(self.n, self.nb, self.dx, self.bc, self.gamma, self.small_p, NG)

    def fine_grid(self) -> Grid:
        """Level-1 description for per-block steps (nb only sizes the array)."""
        return Grid(self.n, (max(self.nfine, 1), 1, 1), tuple(h / 2 for h in self.dx), self.bc, self.gamma,
                    self.small_p, NG)

    def fine_origin(self, f):
        """Level-1 global cell index of the first cell of fine block f."""
        r = int(self.refined[f // 8])
        c = f % 8
        bx, by, bz = r % self.nb[0], (r // self.nb[0]) % self.nb[1], r // (self.nb[0] * self.nb[1])
        n = self.n
        return (2 * bx * n + (c & 1) * n, 2 * by * n + ((c >> 1) & 1) * n, 2 * bz * n + ((c >> 2) & 1) * n)


def _map(I, N, bc):
    if bc == BC_PERIODIC:
        return np.mod(I, N)
    return np.clip(I, 0, N - 1)


def _van_leer(a, b):
    out = np.zeros_like(a)
    m = a * b > 0
    out[m] = (2.0 * (a[m] * b[m])) / (a[m] + b[m])
    return out


def root_value(mesh: Mesh, Ur, I, J, K):
    """Root-level conserved values at level-0 global indices (mapped), [5, ...]."""
    n, nb = mesh.n, mesh.nb
    I = _map(I, nb[0] * n, mesh.bc[0])
    J = _map(J, nb[1] * n, mesh.bc[1])
    K = _map(K, nb[2] * n, mesh.bc[2])
    b = I // n + nb[0] * (J // n + nb[1] * (K // n))
    return Ur[b, :, K % n, J % n, I % n].T  # [5, ...] after transpose of (..., 5)


def fine_guarded(mesh: Mesh, Ur, Uf, f):
    """Guarded view [5, P, P, P] of fine block f (interior and all guards)."""
    n = mesh.n
    P = n + 2 * NG
    X0, Y0, Z0 = mesh.fine_origin(f)
    r = np.arange(-NG, n + NG)
    K, J, I = np.meshgrid(r + Z0, r + Y0, r + X0, indexing="ij")
    NF = [2 * mesh.nb[d] * n for d in range(3)]
    I = _map(I, NF[0], mesh.bc[0])
    J = _map(J, NF[1], mesh.bc[1])
    K = _map(K, NF[2], mesh.bc[2])
    out = np.empty((5, P, P, P))
    # root block under each position
    rb = I // (2 * n) + mesh.nb[0] * (J // (2 * n) + mesh.nb[1] * (K // (2 * n)))
    fine_here = mesh.refine[rb]
    # copies from fine blocks
    if fine_here.any():
        cx, cy, cz = (I // n) % 2, (J // n) % 2, (K // n) % 2
        fb = mesh.child_base[rb] + cx + 2 * cy + 4 * cz
        sel = fine_here
        out[:, sel] = Uf[fb[sel], :, K[sel] % n, J[sel] % n, I[sel] % n].T
    # prolongation from the root cells under the others
    sel = ~fine_here
    if sel.any():
        out[:, sel] = prolong(mesh, Ur, I[sel], J[sel], K[sel])
    return out


def prolong(mesh: Mesh, Ur, I, J, K):
    """Conserved values [5, m] prolonged from the root state to level-1
    global cells (I, J, K) (1-D arrays, inside the domain): the root cell
    under each, U_c + sum_d S_d * (+-1/4), S_d the van Leer slope of the
    conserved variable over root cells d-1, d, d+1 (level-0 map), the sign
    that of the fine cell's offset from the root cell's centre; U_c itself
    where that gives rho <= 0 or p <= 0."""
    Ic, Jc, Kc = I // 2, J // 2, K // 2
    Uc = root_value(mesh, Ur, Ic, Jc, Kc)
    val = Uc.copy()
    offs = [(I % 2) * 2 - 1, (J % 2) * 2 - 1, (K % 2) * 2 - 1]   # -1 / +1
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        Um = root_value(mesh, Ur, Ic - e[0], Jc - e[1], Kc - e[2])
        Up = root_value(mesh, Ur, Ic + e[0], Jc + e[1], Kc + e[2])
        S = _van_leer(Uc - Um, Up - Uc)
        val = val + S * (0.25 * offs[d])
    rho = val[0]
    kin = 0.5 * ((val[1] ** 2 + val[2] ** 2) + val[3] ** 2) / np.where(rho > 0, rho, 1.0)
    p = (mesh.gamma - 1.0) * (val[4] - kin)
    bad = ~((rho > 0) & (p > 0))
    val[:, bad] = Uc[:, bad]
    return val


def _to_guarded(U, n):
    P = n + 2 * NG
    G = np.zeros((U.shape[0], 5, P, P, P))
    G[:, :, NG:NG + n, NG:NG + n, NG:NG + n] = U
    return G


def restrict(mesh: Mesh, Ur, Uf):
    """Each refined root block takes the mean of its children (in place)."""
    n, h = mesh.n, mesh.n // 2
    for q, r in enumerate(mesh.refined):
        for c in range(8):
            cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
            ch = Uf[8 * q + c]
            avg = ch.reshape(5, h, 2, h, 2, h, 2).mean(axis=(2, 4, 6))
            Ur[r, :, cz * h:(cz + 1) * h, cy * h:(cy + 1) * h, cx * h:(cx + 1) * h] = avg


def max_signal(mesh: Mesh, Ur, Uf):
    from . import max_signal as _ms

    s0 = 0.0
    leaves = np.flatnonzero(~mesh.refine)
    if leaves.size:
        g = Grid(mesh.n, (leaves.size, 1, 1), mesh.dx, mesh.bc, mesh.gamma, mesh.small_p, NG)
        s0 = _ms(g, _to_guarded(np.ascontiguousarray(Ur[leaves]), mesh.n))
    s1 = 0.0
    if mesh.nfine:
        s1 = _ms(mesh.fine_grid(), _to_guarded(Uf, mesh.n))
    return max(s0, s1)


def dt(mesh: Mesh, Ur, Uf, cfl: float) -> float:
    return cfl / max_signal(mesh, Ur, Uf)


def _leaf_step(grid: Grid, G, idx: int, dt: float):
    """The predictor-corrector step of block idx of the guarded stack G
    (oracle_step_block_fluxes): its new interior [5, n, n, n], its face
    fluxes per direction and its event counters."""
    n = grid.n
    nf = 5 * (n + 1) * n * n
    out = np.empty(G.shape[1:])
    F = [np.empty(nf) for _ in range(3)]
    c = (ctypes.c_long * 3)(0, 0, 0)
    gc = grid.c()
    lib().oracle_step_block_fluxes(ctypes.byref(gc), _dptr(G), int(idx), _dptr(out), float(dt),
                                   _dptr(F[0]), _dptr(F[1]), _dptr(F[2]), c)
    return out[:, NG:NG + n, NG:NG + n, NG:NG + n], F, np.array(list(c), dtype=np.int64)


def _reflux_block(mesh: Mesh, b: int, Ub, flux0, flux1, lam0):
    """Refluxing of unrefined root block b (new interior Ub, in place) on
    each face it shares with a refined root block."""
    n, nb = mesh.n, mesh.nb
    bx, by, bz = b % nb[0], (b // nb[0]) % nb[1], b // (nb[0] * nb[1])
    for d in range(3):
        for side in (0, 1):            # 0: low face of the block, 1: high face
            pos = [bx, by, bz]
            pos[d] += 1 if side else -1
            if mesh.bc[d] == BC_PERIODIC:
                pos[d] %= nb[d]
            elif not (0 <= pos[d] < nb[d]):
                continue
            nbr = pos[0] + nb[0] * (pos[1] + nb[1] * pos[2])
            if not mesh.refine[nbr]:
                continue
            Fc = _face(flux0[b][d], d, n, n if side else 0)            # [5, n(t1), n(t0)]
            Ff = _fine_face_mean(mesh, flux1, int(mesh.child_base[nbr]), d, side)
            corr = lam0[d] * (Fc - Ff) * (1.0 if side else -1.0)
            cell = n - 1 if side else 0
            sl = [slice(None)] * 3
            sl[2 - d] = cell                                          # array axes (z, y, x)
            Ub[(slice(None),) + tuple(sl)] += corr


def step(mesh: Mesh, Ur, Uf, dt: float):
    """One step; returns (Ur_new, Uf_new, counters)."""
    n = mesh.n
    cnt = np.zeros(3, dtype=np.int64)
    # 1. guard fill
    g0 = mesh.root_grid()
    G0 = _to_guarded(Ur, n)
    from . import fill_guards

    fill_guards(g0, G0)
    G1 = np.stack([fine_guarded(mesh, Ur, Uf, f) for f in range(mesh.nfine)]) if mesh.nfine else None
    # 2. steps with face fluxes
    Ur_new, Uf_new = Ur.copy(), Uf.copy()
    flux0 = {}
    for b in np.flatnonzero(~mesh.refine):
        Ur_new[b], flux0[int(b)], c = _leaf_step(g0, G0, int(b), dt)
        cnt += c
    flux1 = {}
    if mesh.nfine:
        g1 = mesh.fine_grid()
        G1 = np.ascontiguousarray(G1)
        for f in range(mesh.nfine):
            Uf_new[f], flux1[f], c = _leaf_step(g1, G1, f, dt)
            cnt += c
    # 3. refluxing on faces between an unrefined and a refined root block
    lam0 = [dt / h for h in mesh.dx]
    for b in np.flatnonzero(~mesh.refine):
        _reflux_block(mesh, int(b), Ur_new[int(b)], flux0, flux1, lam0)
    # 4. restriction
    restrict(mesh, Ur_new, Uf_new)
    return Ur_new, Uf_new, cnt


def root_guarded(mesh: Mesh, Ur, b: int):
    """Guarded view [5, P, P, P] of root block b by the same-level map over
    the root state (the values fill_guards gives it)."""
    n = mesh.n
    P = n + 2 * NG
    bx, by, bz = b % mesh.nb[0], (b // mesh.nb[0]) % mesh.nb[1], b // (mesh.nb[0] * mesh.nb[1])
    r = np.arange(-NG, n + NG)
    K, J, I = np.meshgrid(r + bz * n, r + by * n, r + bx * n, indexing="ij")
    return root_value(mesh, Ur, I.ravel(), J.ravel(), K.ravel()).reshape(5, P, P, P)


def step_sampled(mesh: Mesh, Ur, Uf, dt: float, roots=(), fines=(), refined=()):
    """What step() gives on chosen blocks, each formed the same way but
    without stepping the rest of the mesh: ``roots`` unrefined root blocks
    (leaf step and refluxing; the fine blocks on their fine-coarse faces are
    stepped for their fluxes), ``fines`` fine blocks, ``refined`` refined
    root blocks (the restriction of their stepped children).  Returns
    ({root block: [5, n, n, n]}, {fine block: [5, n, n, n]})."""
    n = mesh.n
    h = mesh.dx
    g0 = Grid(n, (1, 1, 1), h, mesh.bc, mesh.gamma, mesh.small_p, NG)
    g1 = Grid(n, (1, 1, 1), tuple(x / 2 for x in h), mesh.bc, mesh.gamma, mesh.small_p, NG)
    fine_new = {}

    class _Fluxes(dict):
        def __missing__(self, f):
            V = np.ascontiguousarray(fine_guarded(mesh, Ur, Uf, f)[None])
            fine_new[f], F, _ = _leaf_step(g1, V, 0, dt)
            self[f] = F
            return F

    flux1 = _Fluxes()
    lam0 = [dt / x for x in h]
    out_r = {}
    for b in roots:
        b = int(b)
        assert not mesh.refine[b]
        V = np.ascontiguousarray(root_guarded(mesh, Ur, b)[None])
        Ub, F, _ = _leaf_step(g0, V, 0, dt)
        Ub = Ub.copy()
        _reflux_block(mesh, b, Ub, {b: F}, flux1, lam0)
        out_r[b] = Ub
    for f in fines:
        flux1[int(f)]
    if len(refined):
        Uf_part = np.zeros_like(Uf)
        Ur_part = np.zeros_like(Ur)
        for r in refined:
            for c in range(8):
                f = int(mesh.child_base[int(r)]) + c
                flux1[f]
                Uf_part[f] = fine_new[f]
        restrict(mesh, Ur_part, Uf_part)
        for r in refined:
            out_r[int(r)] = Ur_part[int(r)].copy()
    return out_r, {int(f): fine_new[int(f)].copy() for f in fines}


def _face(F, d, n, idx):
    """Fluxes [5, n, n] (array order: the two transverse axes, slower first)
    on the d-face layer idx (0..n) of one block's flux array."""
    if d == 0:
        A = F.reshape(n, n, n + 1, 5)      # (k, j, i, v)
        return np.moveaxis(A[:, :, idx, :], -1, 0)
    if d == 1:
        A = F.reshape(n, n + 1, n, 5)      # (k, j, i, v)
        return np.moveaxis(A[:, idx, :, :], -1, 0)
    A = F.reshape(n + 1, n, n, 5)          # (k, j, i, v)
    return np.moveaxis(A[idx, :, :, :], -1, 0)


def _fine_face_mean(mesh, flux1, base, d, side):
    """Mean of the four fine fluxes over each root cell face of the refined
    block's face adjacent to the coarse neighbour (side 1: the coarse block's
    high face, so the refined block's low face, and vice versa)."""
    n, h = mesh.n, mesh.n // 2
    out = np.zeros((5, n, n))
    for c in range(8):
        co = [c & 1, (c >> 1) & 1, (c >> 2) & 1]
        if co[d] != (0 if side else 1):
            continue
        F = _face(flux1[base + c][d], d, n, 0 if side else n)      # [5, n, n] fine faces of this child
        # the transverse axes in array order: for d=0 (k, j), d=1 (k, i), d=2 (j, i)
        ta = [t for t in (2, 1, 0) if t != d]                      # slower axis first: z/y/x order
        o0 = co[ta[0]] * h
        o1 = co[ta[1]] * h
        avg = F.reshape(5, h, 2, h, 2).mean(axis=(2, 4))
        out[:, o0:o0 + h, o1:o1 + h] = avg
    return out


# ---- adaptivity: refinement estimator and regridding --------------------------

def _root_global(mesh: Mesh, Ur):
    """Root state as a global array [5, Z, Y, X]."""
    n, nb = mesh.n, mesh.nb
    A = Ur.reshape(nb[2], nb[1], nb[0], 5, n, n, n)
    return np.ascontiguousarray(A.transpose(3, 0, 4, 1, 5, 2, 6)).reshape(5, nb[2] * n, nb[1] * n, nb[0] * n)


def _second_difference_ratio(mesh: Mesh, f, eps: float):
    """Squared Loehner indicator of field f [Z, Y, X] per cell: with
    fL, f0, fR the cell and its neighbours along d (the root map),
    num_d = (fR - f0) - (f0 - fL),
    den_d = (|fR - f0| + |f0 - fL|) + eps ((|fR| + 2|f0|) + |fL|),
    E^2 = sum_d num_d^2 / sum_d den_d^2 (0 where the denominator is 0)."""
    num2 = None
    den2 = None
    for d in range(3):
        ax = 2 - d                                      # array axis of direction d
        N = f.shape[ax]
        idx = np.arange(N)
        lo = _map(idx - 1, N, mesh.bc[d])
        hi = _map(idx + 1, N, mesh.bc[d])
        fL = np.take(f, lo, axis=ax)
        fR = np.take(f, hi, axis=ax)
        num = (fR - f) - (f - fL)
        den = (np.abs(fR - f) + np.abs(f - fL)) + eps * ((np.abs(fR) + 2.0 * np.abs(f)) + np.abs(fL))
        num2 = num * num if num2 is None else num2 + num * num
        den2 = den * den if den2 is None else den2 + den * den
    out = np.zeros_like(f)
    ok = den2 > 0
    out[ok] = num2[ok] / den2[ok]
    return out


def indicator(mesh: Mesh, Ur, eps: float = 0.01):
    """Refinement indicator per root block: the largest squared Loehner
    second-derivative ratio over its cells, of density and of pressure,
    evaluated on the root state (refined blocks hold their children's
    restriction).  Values lie in [0, 1]."""
    n, nb = mesh.n, mesh.nb
    G = _root_global(mesh, Ur)
    rho = G[0]
    kin = 0.5 * ((G[1] * G[1] + G[2] * G[2]) + G[3] * G[3]) / rho
    p = (mesh.gamma - 1.0) * (G[4] - kin)
    E2 = np.maximum(_second_difference_ratio(mesh, rho, eps), _second_difference_ratio(mesh, p, eps))
    B = E2.reshape(nb[2], n, nb[1], n, nb[0], n)
    return B.max(axis=(1, 3, 5)).reshape(-1)


def refine_flags(mesh: Mesh, E2, refine_cutoff: float = 0.8, derefine_cutoff: float = 0.2):
    """New flags from the indicator: refine where E^2 > refine_cutoff^2,
    derefine a refined block where E^2 < derefine_cutoff^2, keep the rest."""
    new = mesh.refine.copy()
    new[E2 > refine_cutoff * refine_cutoff] = True
    new[mesh.refine & (E2 < derefine_cutoff * derefine_cutoff)] = False
    return new


def regrid(mesh: Mesh, Ur, Uf, flags):
    """The mesh with refinement flags `flags` and its state: children of
    blocks refined before are kept as they are; blocks refined now get
    children prolonged from the root state (conservative: each 2x2x2 group
    averages to its root cell); derefined blocks keep their root values
    (the restriction of the children they lose); then every refined root
    block takes the restriction of its children.  Returns (mesh, Ur, Uf)."""
    n = mesh.n
    new = Mesh(n, mesh.nb, mesh.dx, np.asarray(flags, dtype=bool), mesh.bc, mesh.gamma, mesh.small_p)
    Uf2 = np.empty((new.nfine, 5, n, n, n))
    r_ = np.arange(n)
    for q, r in enumerate(new.refined):
        for c in range(8):
            f = 8 * q + c
            if mesh.refine[r]:
                Uf2[f] = Uf[int(mesh.child_base[r]) + c]
                continue
            X0, Y0, Z0 = new.fine_origin(f)
            K, J, I = np.meshgrid(r_ + Z0, r_ + Y0, r_ + X0, indexing="ij")
            Uf2[f] = prolong(new, Ur, I.ravel(), J.ravel(), K.ravel()).reshape(5, n, n, n)
    Ur2 = Ur.copy()
    restrict(new, Ur2, Uf2)
    return new, Ur2, Uf2

