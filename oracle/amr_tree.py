"""Block-structured AMR of any depth (an octree of blocks) in the CPU
oracle: test infrastructure only.

The Grid unit's adaptive mesh (§2 Software Description) refines blocks
recursively: level 0 is the root grid of nb blocks of n^3 cells; a refined
block of level l is covered by eight children of level l+1 at half its cell
width.  The blocks of level l+1 are the children of the refined blocks of
level l in increasing block index, child c = cx + 2 cy + 4 cz covering cells
(cx n/2.., cy n/2.., cz n/2..) of its parent.  Leaves (unrefined blocks)
are advanced; refined blocks hold the restriction of their children.

Nesting: every refined block of level >= 1 has all 26 neighbours (mapped
by the boundary conditions; outflow positions beyond the domain excluded)
present at its own level.  Then leaf levels differ by at most one across
faces, edges and corners, and every value a prolongation needs exists one
level up.

A step of size dt (every leaf, one dt):
  1. guard fill of every leaf (4 layers): a guard position (mapped at the
     block's level) inside a block of that level copies its cell; otherwise
     it is prolonged from the level above: U_c + sum_d S_d * (+-1/4), U_c the
     level-(l-1) cell under it and S_d the van Leer slope of the conserved
     variable over level-(l-1) cells d-1, d, d+1 (read through the level-(l-1)
     block lookup, mapped at that level), keeping U_c where the result has
     rho <= 0 or p <= 0;
  2. the predictor-corrector step of every leaf with lam = dt/dx of its
     level (oracle_step_block_fluxes);
  3. refluxing: a leaf of level l next to a refined block of level l
     replaces the flux of its cells on that face by the mean of the four
     level-(l+1) fluxes over each;
  4. restriction, finest level first: each refined block takes the mean of
     its children.
dt = CFL / max over leaves of the summed signal speed with each level's dx.
With two levels this is oracle.amr's step, bit for bit.

State: U[l] of shape [nblocks(l), 5, n, n, n] per level.
"""
from __future__ import annotations

import itertools
from typing import List, Sequence

import numpy as np

from . import BC_PERIODIC, Grid
from . import amr as _amr

NG = 4


class Tree:
    def __init__(self, n: int, nb, dx, flags: Sequence[Sequence[bool]], bc=(BC_PERIODIC,) * 3,
                 gamma: float = 1.4, small_p: float = 1e-10):
        """flags[l]: refinement flag of every block of level l (levels whose
        flags are all False may be omitted at the end)."""
        assert n % 2 == 0
        self.n, self.nb0, self.dx0 = n, tuple(int(x) for x in nb), tuple(float(x) for x in dx)
        self.bc, self.gamma, self.small_p = tuple(bc), float(gamma), float(small_p)
        nroot = self.nb0[0] * self.nb0[1] * self.nb0[2]
        # block positions per level
        self.pos: List[np.ndarray] = [np.array([(b % self.nb0[0], (b // self.nb0[0]) % self.nb0[1],
                                                 b // (self.nb0[0] * self.nb0[1])) for b in range(nroot)])]
        self.refine: List[np.ndarray] = []
        self.child_base: List[np.ndarray] = []
        self.parent: List[np.ndarray] = [-np.ones(nroot, dtype=np.int64)]
        l = 0
        while True:
            nbl = len(self.pos[l])
            f = np.zeros(nbl, dtype=bool)
            if l < len(flags):
                f = np.asarray(flags[l], dtype=bool).reshape(-1)
                assert f.size == nbl, f"level {l} has {nbl} blocks, got {f.size} flags"
            self.refine.append(f)
            cb = -np.ones(nbl, dtype=np.int64)
            ref = np.flatnonzero(f)
            cb[ref] = 8 * np.arange(ref.size)
            self.child_base.append(cb)
            if not ref.size:
                break
            kids, par = [], []
            for r in ref:
                for c in range(8):
                    kids.append(2 * self.pos[l][r] + np.array([c & 1, (c >> 1) & 1, (c >> 2) & 1]))
                    par.append(r)
            self.pos.append(np.array(kids))
            self.parent.append(np.array(par))
            l += 1
        self.levels = len(self.pos)
        # dense lookup per level: block index at each level-l block position, or -1
        self.lookup = []
        for l in range(self.levels):
            nbl = self.nb(l)
            L = -np.ones(nbl[2] * nbl[1] * nbl[0], dtype=np.int64)
            p = self.pos[l]
            L[p[:, 0] + nbl[0] * (p[:, 1] + nbl[1] * p[:, 2])] = np.arange(len(p))
            self.lookup.append(L)
        self.check_nesting()

    def nb(self, l):
        return tuple(x << l for x in self.nb0)

    def dx(self, l):
        return tuple(h / (1 << l) for h in self.dx0)

    def nblocks(self, l):
        return len(self.pos[l])

    def leaves(self, l):
        return np.flatnonzero(~self.refine[l])

    def block_at(self, l, bx, by, bz):
        """Level-l block at level-l block position (mapped), or -1 (positions
        beyond an outflow boundary: -2)."""
        nbl = self.nb(l)
        p = [bx, by, bz]
        for d in range(3):
            if self.bc[d] == BC_PERIODIC:
                p[d] %= nbl[d]
            elif not 0 <= p[d] < nbl[d]:
                return -2
        return int(self.lookup[l][p[0] + nbl[0] * (p[1] + nbl[1] * p[2])])

    def check_nesting(self):
        for l in range(1, self.levels):
            for r in np.flatnonzero(self.refine[l]):
                x, y, z = self.pos[l][r]
                for dx_, dy, dz in itertools.product((-1, 0, 1), repeat=3):
                    if self.block_at(l, x + dx_, y + dy, z + dz) == -1:
                        raise ValueError(f"refined block {r} of level {l} lacks a same-level neighbour")

    def grid(self, l, nblk):
        return Grid(self.n, (max(nblk, 1), 1, 1), self.dx(l), self.bc, self.gamma, self.small_p, NG)


def _map(I, N, bc):
    if bc == BC_PERIODIC:
        return np.mod(I, N)
    return np.clip(I, 0, N - 1)


def level_value(t: Tree, U, l, I, J, K):
    """Conserved values [5, m] of level-l cells at level-l global indices
    (mapped at level l; each must lie in a block of level l)."""
    n = t.n
    nbl = t.nb(l)
    I = _map(I, nbl[0] * n, t.bc[0])
    J = _map(J, nbl[1] * n, t.bc[1])
    K = _map(K, nbl[2] * n, t.bc[2])
    b = t.lookup[l][I // n + nbl[0] * (J // n + nbl[1] * (K // n))]
    assert np.all(b >= 0), "a prolongation reached a region absent at the level above"
    return U[l][b, :, K % n, J % n, I % n].T


def prolong(t: Tree, U, l, I, J, K):
    """Values [5, m] prolonged from level l-1 to level-l cells (I, J, K)
    (1-D, mapped): the same operations, in the same order, as the two-level
    prolongation."""
    Ic, Jc, Kc = I // 2, J // 2, K // 2
    Uc = level_value(t, U, l - 1, Ic, Jc, Kc)
    val = Uc.copy()
    offs = [(I % 2) * 2 - 1, (J % 2) * 2 - 1, (K % 2) * 2 - 1]
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        Um = level_value(t, U, l - 1, Ic - e[0], Jc - e[1], Kc - e[2])
        Up = level_value(t, U, l - 1, Ic + e[0], Jc + e[1], Kc + e[2])
        S = _amr._van_leer(Uc - Um, Up - Uc)
        val = val + S * (0.25 * offs[d])
    rho = val[0]
    kin = 0.5 * ((val[1] ** 2 + val[2] ** 2) + val[3] ** 2) / np.where(rho > 0, rho, 1.0)
    p = (t.gamma - 1.0) * (val[4] - kin)
    bad = ~((rho > 0) & (p > 0))
    val[:, bad] = Uc[:, bad]
    return val


def guarded(t: Tree, U, l, b):
    """Guarded view [5, P, P, P] of block b of level l."""
    n = t.n
    P = n + 2 * NG
    X0, Y0, Z0 = (t.pos[l][b] * n).tolist()
    r = np.arange(-NG, n + NG)
    K, J, I = np.meshgrid(r + Z0, r + Y0, r + X0, indexing="ij")
    nbl = t.nb(l)
    I = _map(I, nbl[0] * n, t.bc[0]).ravel()
    J = _map(J, nbl[1] * n, t.bc[1]).ravel()
    K = _map(K, nbl[2] * n, t.bc[2]).ravel()
    blk = t.lookup[l][I // n + nbl[0] * (J // n + nbl[1] * (K // n))]
    out = np.empty((5, I.size))
    here = blk >= 0
    if here.any():
        out[:, here] = U[l][blk[here], :, K[here] % n, J[here] % n, I[here] % n].T
    if (~here).any():
        assert l > 0
        out[:, ~here] = prolong(t, U, l, I[~here], J[~here], K[~here])
    return out.reshape(5, P, P, P)


def restrict(t: Tree, U):
    """Every refined block takes the mean of its children, finest level first (in place)."""
    h = t.n // 2
    for l in range(t.levels - 2, -1, -1):
        for r in np.flatnonzero(t.refine[l]):
            base = int(t.child_base[l][r])
            for c in range(8):
                cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
                avg = U[l + 1][base + c].reshape(5, h, 2, h, 2, h, 2).mean(axis=(2, 4, 6))
                U[l][r, :, cz * h:(cz + 1) * h, cy * h:(cy + 1) * h, cx * h:(cx + 1) * h] = avg


def max_signal(t: Tree, U):
    from . import max_signal as _ms

    s = 0.0
    for l in range(t.levels):
        lv = t.leaves(l)
        if lv.size:
            s = max(s, _ms(t.grid(l, lv.size), _amr._to_guarded(np.ascontiguousarray(U[l][lv]), t.n)))
    return s


def dt(t: Tree, U, cfl: float) -> float:
    return cfl / max_signal(t, U)


def step(t: Tree, U, dt: float):
    """One step; returns (new state per level, counters)."""
    n = t.n
    cnt = np.zeros(3, dtype=np.int64)
    new = [u.copy() for u in U]
    flux = [dict() for _ in range(t.levels)]
    g1 = [t.grid(l, 1) for l in range(t.levels)]
    for l in range(t.levels):
        for b in t.leaves(l):
            V = np.ascontiguousarray(guarded(t, U, l, int(b))[None])
            new[l][b], flux[l][int(b)], c = _amr._leaf_step(g1[l], V, 0, dt)
            cnt += c
    # refluxing: leaves of level l next to refined blocks of level l
    for l in range(t.levels - 1):
        lam = [dt / h for h in t.dx(l)]
        for b in t.leaves(l):
            b = int(b)
            x, y, z = t.pos[l][b]
            for d in range(3):
                for side in (0, 1):
                    q = [x, y, z]
                    q[d] += 1 if side else -1
                    r = t.block_at(l, *q)
                    if r < 0 or not t.refine[l][r]:
                        continue
                    Fc = _amr._face(flux[l][b][d], d, n, n if side else 0)
                    Ff = _fine_mean(t, flux[l + 1], int(t.child_base[l][r]), d, side)
                    corr = lam[d] * (Fc - Ff) * (1.0 if side else -1.0)
                    sl = [slice(None)] * 3
                    sl[2 - d] = n - 1 if side else 0
                    new[l][b][(slice(None),) + tuple(sl)] += corr
    restrict(t, new)
    return new, cnt


def _fine_mean(t: Tree, flux1, base, d, side):
    """Mean of the four fine fluxes over each coarse cell face (the two-level
    oracle's rule; mesh only supplies n)."""
    class _M:
        n = t.n
    return _amr._fine_face_mean(_M, flux1, base, d, side)


# ---- adaptivity of a tree ------------------------------------------------------

def indicator(t: Tree, U, eps: float = 0.01):
    """Refinement indicator of every leaf, per level ([array per level],
    refined blocks 0): the largest, over the leaf's cells, of the squared
    Loehner ratio of density and of pressure (oracle.amr's per-cell
    formula), its neighbours read at the leaf's own level (boundary map,
    block lookup); a neighbour position with no block of that level (a
    coarser region) takes the cell's own value."""
    n = t.n
    out = []
    for l in range(t.levels):
        E = np.zeros(t.nblocks(l))
        nbl = t.nb(l)
        for b in t.leaves(l):
            X0, Y0, Z0 = (t.pos[l][b] * n).tolist()
            r = np.arange(n)
            K, J, I = np.meshgrid(r + Z0, r + Y0, r + X0, indexing="ij")
            c = (I.ravel(), J.ravel(), K.ravel())

            def fields(I, J, K, own):
                Im = _map(I, nbl[0] * n, t.bc[0])
                Jm = _map(J, nbl[1] * n, t.bc[1])
                Km = _map(K, nbl[2] * n, t.bc[2])
                blk = t.lookup[l][Im // n + nbl[0] * (Jm // n + nbl[1] * (Km // n))]
                u = np.empty((5, Im.size))
                ok = blk >= 0
                u[:, ok] = U[l][blk[ok], :, Km[ok] % n, Jm[ok] % n, Im[ok] % n].T
                if own is not None:
                    u[:, ~ok] = own[:, ~ok]
                rho = u[0]
                kin = 0.5 * ((u[1] * u[1] + u[2] * u[2]) + u[3] * u[3]) / rho
                return u, rho, (t.gamma - 1.0) * (u[4] - kin)

            u0, r0, p0 = fields(*c, None)
            num = {"r": None, "p": None}
            den = {"r": None, "p": None}
            for d in range(3):
                e = [0, 0, 0]
                e[d] = 1
                _, rL, pL = fields(c[0] - e[0], c[1] - e[1], c[2] - e[2], u0)
                _, rR, pR = fields(c[0] + e[0], c[1] + e[1], c[2] + e[2], u0)
                for key, fL, f0, fR in (("r", rL, r0, rR), ("p", pL, p0, pR)):
                    nn = (fR - f0) - (f0 - fL)
                    dd = (np.abs(fR - f0) + np.abs(f0 - fL)) + eps * ((np.abs(fR) + 2.0 * np.abs(f0)) + np.abs(fL))
                    num[key] = nn * nn if num[key] is None else num[key] + nn * nn
                    den[key] = dd * dd if den[key] is None else den[key] + dd * dd
            E2 = np.zeros(r0.size)
            for key in ("r", "p"):
                ok = den[key] > 0
                e2 = np.zeros(r0.size)
                e2[ok] = num[key][ok] / den[key][ok]
                E2 = np.maximum(E2, e2)
            E[b] = E2.max()
        out.append(E)
    return out


def _refined_sets(t: Tree):
    return [set(map(tuple, t.pos[l][np.flatnonzero(t.refine[l])].tolist())) for l in range(t.levels)]


def _flags_from_sets(t: Tree, R):
    """Per-level flags in block order for refined-position sets R."""
    flags = [[tuple(p) in R[0] for p in t.pos[0].tolist()]]
    l = 0
    while any(flags[l]):
        kids = []
        blocks = [tuple(p) for p, f in zip(_level_positions(t, flags, l), flags[l]) if f]
        for (x, y, z) in blocks:
            for c in range(8):
                kids.append((2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + ((c >> 2) & 1)))
        R_next = R[l + 1] if l + 1 < len(R) else set()
        flags.append([k in R_next for k in kids])
        l += 1
    return flags


def _level_positions(t: Tree, flags, l):
    if l == 0:
        return t.pos[0].tolist()
    prev = [tuple(p) for p, f in zip(_level_positions(t, flags, l - 1), flags[l - 1]) if f]
    out = []
    for (x, y, z) in prev:
        for c in range(8):
            out.append((2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + ((c >> 2) & 1)))
    return out


def refine_flags(t: Tree, E2, refine_cutoff: float = 0.8, derefine_cutoff: float = 0.2, max_levels: int = 3):
    """New per-level flags from the indicator: a leaf with E^2 >
    refine_cutoff^2 below the deepest allowed level is refined; a refined
    block whose eight children are leaves with E^2 < derefine_cutoff^2 loses
    them; then nesting is restored by refining (level by level, coarsest
    first, in increasing block position) the blocks whose absence leaves a
    refined block of level >= 1 without a same-level neighbour, until
    nothing changes."""
    rc2, dc2 = refine_cutoff * refine_cutoff, derefine_cutoff * derefine_cutoff
    R = _refined_sets(t)
    while len(R) < max_levels:
        R.append(set())
    for l in range(t.levels):
        for b in t.leaves(l):
            if E2[l][b] > rc2 and l + 1 < max_levels:
                R[l].add(tuple(t.pos[l][b].tolist()))
    for l in range(t.levels - 1):
        for r in np.flatnonzero(t.refine[l]):
            base = int(t.child_base[l][r])
            kids = range(base, base + 8)
            if all((not t.refine[l + 1][k]) and E2[l + 1][k] < dc2 for k in kids):
                R[l].discard(tuple(t.pos[l][r].tolist()))
    _restore_nesting(t, R)
    return _flags_from_sets(t, R)


def _is_block(R, l, p):
    return l == 0 or (p[0] // 2, p[1] // 2, p[2] // 2) in R[l - 1]


def _restore_nesting(t: Tree, R):
    nb0 = t.nb0

    def wrap(l, q):
        q = list(q)
        for d in range(3):
            N = nb0[d] << l
            if t.bc[d] == BC_PERIODIC:
                q[d] %= N
            elif not 0 <= q[d] < N:
                return None
        return tuple(q)

    def ensure_block(l, p):
        """Make position p of level l a block (refine its ancestors)."""
        if _is_block(R, l, p):
            return
        par = (p[0] // 2, p[1] // 2, p[2] // 2)
        ensure_block(l - 1, par)
        R[l - 1].add(par)

    changed = True
    while changed:
        changed = False
        # drop refined positions that are no longer blocks (an ancestor lost its children)
        for l in range(1, len(R)):
            for p in sorted(R[l]):
                if not _is_block(R, l, p):
                    R[l].discard(p)
                    changed = True
        for l in range(1, len(R)):
            for p in sorted(R[l]):
                for dz in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            q = wrap(l, (p[0] + dx, p[1] + dy, p[2] + dz))
                            if q is not None and not _is_block(R, l, q):
                                ensure_block(l, q)
                                changed = True


def regrid(t: Tree, U, flags):
    """The tree with per-level flags `flags` and its state: level 0 as is;
    at each deeper level, in order, a block present before (same level and
    position) keeps its cells, a new one is prolonged from the level above
    (already final); then restriction, finest level first.  Returns (tree, U)."""
    new = Tree(t.n, t.nb0, t.dx0, flags, t.bc, t.gamma, t.small_p)
    n = t.n
    V = [U[0].copy()]
    r_ = np.arange(n)
    for l in range(1, new.levels):
        Ul = np.empty((new.nblocks(l), 5, n, n, n))
        for i, p in enumerate(new.pos[l].tolist()):
            old = t.block_at(l, *p) if l < t.levels else -1
            if old >= 0:
                Ul[i] = U[l][old]
                continue
            X0, Y0, Z0 = (np.array(p) * n).tolist()
            K, J, I = np.meshgrid(r_ + Z0, r_ + Y0, r_ + X0, indexing="ij")
            Ul[i] = prolong(new, V, l, I.ravel(), J.ravel(), K.ravel()).reshape(5, n, n, n)
        V.append(Ul)
    restrict(new, V)
    return new, V
