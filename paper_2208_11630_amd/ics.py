"""Seeded synthetic inputs and the blocked, guarded storage layout.

This module is shared by the HIP path's tests and the oracle's tests: it
draws initial states and rearranges arrays between the global ``[5, Z, Y, X]``
order, the compact blocked storage ``[nblk, 5, n, n, n]`` of the HIP library
and the guarded blocked storage ``[nblk, 5, P, P, P]`` (P = n + 2*ng) the
oracle works on; x fastest, block id b = bx + nbx*(by + nby*bz).  It holds
none of the step's arithmetic.  The only formula it evaluates is the definition of the initial
total energy of a gamma-law gas, E = p/(gamma-1) + rho*|v|^2/2, which sets up
the problem.

The workloads are the paper's kind of problem (§2: compressible flow with
strong shocks on a uniform block grid) in five synthetic configurations:
a Sod shock tube, a Sedov point blast, a Kelvin-Helmholtz shear layer, a
batched ensemble of small random-state simulations and a served stream of
many resident simulations.  Every random draw uses numpy's PCG64
(``default_rng(seed)``), arrays drawn in global C order (z, y, x).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

PERIODIC = 0
OUTFLOW = 1
NGUARD = 4


@dataclass
class Problem:
    """A grid plus its initial conserved state.

    ``data`` is either the compact blocked array ``[nblk, 5, n, n, n]`` (the
    state layout of the HIP library) or the guarded blocked array
    ``[nblk, 5, P, P, P]`` (P = n + 2*ng, the textbook layout the oracle works
    on); ``Uc`` and ``U`` give each view, converting (and caching) on demand."""

    name: str
    n: int                      # interior cells per block edge
    nb: Tuple[int, int, int]    # blocks per axis
    dx: Tuple[float, float, float]
    bc: Tuple[int, int, int]
    gamma: float
    data: np.ndarray
    small_p: float = 1e-10
    cfl: float = 0.8
    steps: int = 1
    ng: int = NGUARD
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        P = self.n + 2 * self.ng
        if self.data.shape[2:] == (self.n,) * 3:
            self._c, self._g = self.data, None
        elif self.data.shape[2:] == (P,) * 3:
            self._c, self._g = None, self.data
        else:
            raise ValueError(f"state shape {self.data.shape} fits neither layout")

    @property
    def U(self) -> np.ndarray:
        """Guarded layout [nblk, 5, P, P, P] (guards zero until filled)."""
        if self._g is None:
            self._g = guard_layout(self._c, self.n, self.ng)
        return self._g

    @property
    def Uc(self) -> np.ndarray:
        """Compact layout [nblk, 5, n, n, n]."""
        if self._c is None:
            self._c = np.ascontiguousarray(interior(self._g, self.n, self.ng))
        return self._c

    @property
    def nblk(self) -> int:
        return self.nb[0] * self.nb[1] * self.nb[2]

    @property
    def cells(self) -> int:
        return self.nblk * self.n ** 3

    @property
    def lo(self):
        return (0.0, 0.0, 0.0)

    @property
    def hi(self):
        return tuple(self.nb[d] * self.n * self.dx[d] for d in range(3))


# ---- layout ---------------------------------------------------------------

def kelvin_helmholtz_amr(root=(256, 256, 128), n: int = 16, seed_root: int = 1, seed_fine: int = 5):
    """Two-level Kelvin-Helmholtz mesh: the shear layer of kelvin_helmholtz
    on a root grid of ``root`` cells, the root blocks whose y range touches an
    interface (y = 0.25, 0.75) refined once.  The root state samples the
    problem at the root resolution, the fine blocks at twice it (independent
    seeded perturbations; the first step's restriction makes the levels
    agree).  Returns (nb, refine flags, Ur [nroot,5,n,n,n], Uf [nfine,5,n,n,n],
    dx of the root level, gamma); fine blocks are the children of the refined
    root blocks in increasing root id, child cx + 2 cy + 4 cz."""
    X, Y, Z = root
    nb = (X // n, Y // n, Z // n)
    P0 = kelvin_helmholtz(shape=root, n=n, seed=seed_root)
    # root block rows whose y range [by, by+1) * n/Y has 0.25 or 0.75 on an edge or inside
    by = np.arange(nb[1])
    y0, y1 = by * n / Y, (by + 1) * n / Y
    touch = np.zeros(nb[1], bool)
    for yi in (0.25, 0.75):
        touch |= (y0 <= yi) & (y1 >= yi)
    flags = np.broadcast_to(touch[None, :, None], (nb[2], nb[1], nb[0])).reshape(-1).copy()
    refined = np.flatnonzero(flags)
    Pf = kelvin_helmholtz(shape=(2 * X, 2 * Y, 2 * Z), n=n, seed=seed_fine)
    fb = Pf.Uc.reshape(2 * nb[2], 2 * nb[1], 2 * nb[0], 5, n, n, n)
    Uf = np.empty((8 * refined.size, 5, n, n, n))
    for q, r in enumerate(refined):
        bx, byy, bz = r % nb[0], (r // nb[0]) % nb[1], r // (nb[0] * nb[1])
        for c in range(8):
            Uf[8 * q + c] = fb[2 * bz + (c >> 2), 2 * byy + ((c >> 1) & 1), 2 * bx + (c & 1)]
    return nb, flags, P0.Uc, Uf, P0.dx, P0.gamma


def kelvin_helmholtz_amr3(root=(256, 256, 128), n: int = 16, seed_root: int = 1, seed_fine: int = 5):
    """Three-level Kelvin-Helmholtz mesh: kelvin_helmholtz_amr's two levels,
    plus the level-1 block rows that hold an interface (y = 0.25, 0.75 on a
    block edge) refined again.  Level-2 blocks start as copies of their
    parent cells (each level-1 cell value on its 2x2x2 children; the first
    step's restriction reconciles the levels).  Returns (nb, flags0, flags1,
    Ur, Uf) with Uf the level-1 blocks then the level-2 blocks."""
    nb, flags0, Ur, Uf1, dx, gamma = kelvin_helmholtz_amr(root, n, seed_root, seed_fine)
    refined0 = np.flatnonzero(flags0)
    # level-1 block rows (y positions at level 1) that touch an interface
    ny1 = 2 * nb[1]
    rows = set()
    for yi in (0.25, 0.75):
        r = int(round(yi * ny1))
        rows.update({r - 1, r})
    flags1 = np.zeros(8 * refined0.size, bool)
    for q, r in enumerate(refined0):
        by = (r // nb[0]) % nb[1]
        for c in range(8):
            flags1[8 * q + c] = (2 * by + ((c >> 1) & 1)) in rows
    ref1 = np.flatnonzero(flags1)
    h = n // 2
    Uf2 = np.empty((8 * ref1.size, 5, n, n, n))
    for q, f in enumerate(ref1):
        for c in range(8):
            cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
            part = Uf1[f, :, cz * h:(cz + 1) * h, cy * h:(cy + 1) * h, cx * h:(cx + 1) * h]
            Uf2[8 * q + c] = part.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)
    return nb, flags0, flags1, Ur, np.concatenate([Uf1, Uf2]), dx, gamma


def to_blocks(G: np.ndarray, n: int, ng: int = NGUARD, out: np.ndarray | None = None) -> np.ndarray:
    """Global ``[5, Z, Y, X]`` -> blocked ``[nblk, 5, P, P, P]`` (guards zero)."""
    _, Z, Y, X = G.shape
    if X % n or Y % n or Z % n:
        raise ValueError("grid extent must be a multiple of the block size")
    nbx, nby, nbz = X // n, Y // n, Z // n
    P = n + 2 * ng
    if out is None:
        out = np.zeros((nbx * nby * nbz, 5, P, P, P))
    # [5, nbz, n, nby, n, nbx, n] -> [nbz, nby, nbx, 5, n, n, n]
    v = G.reshape(5, nbz, n, nby, n, nbx, n).transpose(1, 3, 5, 0, 2, 4, 6)
    out.reshape(nbz, nby, nbx, 5, P, P, P)[..., ng:ng + n, ng:ng + n, ng:ng + n] = v
    return out


def to_compact(G: np.ndarray, n: int) -> np.ndarray:
    """Global ``[5, Z, Y, X]`` -> compact blocked ``[nblk, 5, n, n, n]``."""
    _, Z, Y, X = G.shape
    if X % n or Y % n or Z % n:
        raise ValueError("grid extent must be a multiple of the block size")
    nbx, nby, nbz = X // n, Y // n, Z // n
    v = G.reshape(5, nbz, n, nby, n, nbx, n).transpose(1, 3, 5, 0, 2, 4, 6)
    return np.ascontiguousarray(v).reshape(nbx * nby * nbz, 5, n, n, n)


def guard_layout(C: np.ndarray, n: int, ng: int = NGUARD) -> np.ndarray:
    """Compact ``[nblk, 5, n, n, n]`` -> guarded ``[nblk, 5, P, P, P]`` (guards zero)."""
    P = n + 2 * ng
    out = np.zeros((C.shape[0], 5, P, P, P))
    out[:, :, ng:ng + n, ng:ng + n, ng:ng + n] = C
    return out


def from_blocks(B: np.ndarray, n: int, nb: Tuple[int, int, int], ng: int = NGUARD) -> np.ndarray:
    """Blocked storage (guarded or compact) -> global interior ``[5, Z, Y, X]``."""
    nbx, nby, nbz = nb
    I = interior(B, n, ng)
    I = I.reshape(nbz, nby, nbx, 5, n, n, n)
    return np.ascontiguousarray(I.transpose(3, 0, 4, 1, 5, 2, 6)).reshape(5, nbz * n, nby * n, nbx * n)


def interior(B: np.ndarray, n: int, ng: int = NGUARD) -> np.ndarray:
    """Interiors ``[nblk, 5, n, n, n]`` of blocked storage (a view; compact
    storage is returned as is)."""
    if B.shape[2] == n:
        return B
    return B[:, :, ng:ng + n, ng:ng + n, ng:ng + n]


def conserved(rho, u, v, w, p, gamma) -> np.ndarray:
    """Initial conserved state [5, ...] from primitive fields (problem set-up)."""
    rho = np.asarray(rho, dtype=np.float64)
    shape = np.broadcast(rho, u, v, w, p).shape
    G = np.empty((5,) + shape)
    G[0] = rho
    G[1] = rho * u
    G[2] = rho * v
    G[3] = rho * w
    G[4] = p / (gamma - 1.0) + 0.5 * rho * ((u * u + v * v) + w * w)
    return G


def block_arrangement(nblk: int) -> Tuple[int, int, int]:
    """Factor nblk = nbx*nby*nbz, most nearly cubic (min max/min), nbx >= nby >= nbz."""
    best = None
    for a in range(1, nblk + 1):
        if nblk % a:
            continue
        for b in range(1, nblk // a + 1):
            if (nblk // a) % b:
                continue
            c = nblk // (a * b)
            t = tuple(sorted((a, b, c), reverse=True))
            key = (t[0] / t[2], t)
            if best is None or key < best[0]:
                best = (key, t)
    return best[1]


# ---- problems ---------------------------------------------------------------

def sod(N: int = 64, n: int = 16, axis: int = 0, shape=None) -> Problem:
    """Sod shock tube along ``axis``: rho=1, p=1 for x<0.5, rho=0.125, p=0.1 else,
    at rest, gamma=1.4; outflow along the tube, periodic across it; unit cube,
    CFL 0.8, 20 steps.  ``shape`` (X, Y, Z) overrides the cubic N^3 grid."""
    X, Y, Z = shape if shape is not None else (N, N, N)
    ext = (X, Y, Z)
    L = ext[axis]
    h = 1.0 / L
    idx = np.arange(L)
    left = (2 * idx + 1) < L          # cell centre < 0.5
    rho1 = np.where(left, 1.0, 0.125)
    p1 = np.where(left, 1.0, 0.1)
    bshape = [1, 1, 1]
    bshape[2 - axis] = L               # arrays are (z, y, x)
    rho = np.broadcast_to(rho1.reshape(bshape), (Z, Y, X))
    p = np.broadcast_to(p1.reshape(bshape), (Z, Y, X))
    zero = np.zeros((Z, Y, X))
    G = conserved(rho, zero, zero, zero, p, 1.4)
    bc = [PERIODIC] * 3
    bc[axis] = OUTFLOW
    return Problem("sod", n, (X // n, Y // n, Z // n), (h, h, h), tuple(bc), 1.4,
                   to_compact(G, n), steps=20, meta={"axis": axis})


def sedov_deposit_mask(N: int) -> np.ndarray:
    """Cells of an N^3 unit-cube grid whose centres lie within 3.5 dx of the
    centre (0.5, 0.5, 0.5): (2i+1-N)^2 + (2j+1-N)^2 + (2k+1-N)^2 < 49, exact."""
    a = (2 * np.arange(N) + 1 - N) ** 2
    return (a[:, None, None] + a[None, :, None] + a[None, None, :]) < 49


def sedov(N: int = 256, n: int = 16, steps: int = 100) -> Problem:
    """Sedov point blast: rho=1, p=1e-5, at rest, gamma=1.4, periodic unit cube;
    total energy 1 deposited uniformly (replacing the ambient energy) in the
    cells whose centres lie within 3.5 dx of the centre."""
    gamma = 1.4
    h = 1.0 / N
    rho = np.ones((N, N, N))
    zero = np.zeros((N, N, N))
    G = conserved(rho, zero, zero, zero, np.full((N, N, N), 1e-5), gamma)
    mask = sedov_deposit_mask(N)
    nin = int(mask.sum())
    G[4][mask] = 1.0 / (nin * h ** 3)
    return Problem("sedov", n, (N // n,) * 3, (h, h, h), (PERIODIC,) * 3, gamma,
                   to_compact(G, n), steps=steps, meta={"n_deposit": nin})


def kelvin_helmholtz(shape=(512, 512, 256), n: int = 16, seed: int = 1, steps: int = 10) -> Problem:
    """Kelvin-Helmholtz shear layer on [0,1] x [0,1] x [0, Z/X] with cubic cells:
    gamma=5/3, p=2.5; rho=2, vx=+0.5 for |y-0.5|<0.25, else rho=1, vx=-0.5;
    i.i.d. U(-0.01, 0.01) perturbations on vx then vy (seeded); periodic."""
    X, Y, Z = shape
    gamma = 5.0 / 3.0
    h = 1.0 / X
    j = np.arange(Y)
    band = (4 * (2 * j + 1) > Y * 2) & (4 * (2 * j + 1) < Y * 6)  # 0.25 < y_c < 0.75
    rho = np.broadcast_to(np.where(band, 2.0, 1.0)[None, :, None], (Z, Y, X))
    vx0 = np.broadcast_to(np.where(band, 0.5, -0.5)[None, :, None], (Z, Y, X))
    rng = np.random.default_rng(seed)
    dvx = rng.uniform(-0.01, 0.01, size=(Z, Y, X))
    dvy = rng.uniform(-0.01, 0.01, size=(Z, Y, X))
    G = conserved(rho, vx0 + dvx, dvy, np.zeros((Z, Y, X)), np.full((Z, Y, X), 2.5), gamma)
    return Problem("kh", n, (X // n, Y // n, Z // n), (h, h, h), (PERIODIC,) * 3, gamma,
                   to_compact(G, n), steps=steps)


def random_state(rng: np.random.Generator, shape, gamma: float = 1.4) -> np.ndarray:
    """rho = exp(N(0, 0.3)), p = exp(N(0, 0.3)), u, v, w ~ N(0, 0.2) per cell,
    drawn in that order; returns the conserved global array [5, Z, Y, X]."""
    rho = np.exp(rng.normal(0.0, 0.3, size=shape))
    p = np.exp(rng.normal(0.0, 0.3, size=shape))
    u = rng.normal(0.0, 0.2, size=shape)
    v = rng.normal(0.0, 0.2, size=shape)
    w = rng.normal(0.0, 0.2, size=shape)
    return conserved(rho, u, v, w, p, gamma)


def ensemble_shapes(count: int = 512, seed: int = 2) -> List[Tuple[int, int]]:
    """(nblk, nxb) of each ensemble member: nblk ~ U{1..64}, nxb in {8, 16, 32}."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        nblk = int(rng.integers(1, 65))
        nxb = int(rng.choice([8, 16, 32]))
        out.append((nblk, nxb))
    return out


def ensemble(count: int = 512, seed: int = 2, steps: int = 50, shapes=None) -> List[Problem]:
    """Independent periodic simulations with random states (gamma=1.4).  All
    shapes are drawn first, then each member's fields in member order, from
    one generator.  Cells are cubic with dx = 1/(cells along x)."""
    rng = np.random.default_rng(seed)
    if shapes is None:
        shapes = []
        for _ in range(count):
            nblk = int(rng.integers(1, 65))
            nxb = int(rng.choice([8, 16, 32]))
            shapes.append((nblk, nxb))
    sims = []
    for s, (nblk, n) in enumerate(shapes):
        nb = block_arrangement(nblk)
        X, Y, Z = nb[0] * n, nb[1] * n, nb[2] * n
        G = random_state(rng, (Z, Y, X))
        h = 1.0 / X
        sims.append(Problem(f"ens{s}", n, nb, (h, h, h), (PERIODIC,) * 3, 1.4,
                            to_compact(G, n), steps=steps))
    return sims


def served_sizes(count: int = 2000, seed: int = 3) -> List[int]:
    """Edge L of each served simulation: 16*round(exp(U(ln 32, ln 256))/16)."""
    rng = np.random.default_rng(seed)
    e = rng.uniform(math.log(32.0), math.log(256.0), size=count)
    return [int(16 * round(math.exp(x) / 16.0)) for x in e]


def served_sim(sim: int, L: int, seed: int = 3, n: int = 16) -> Problem:
    """Initial state of served simulation ``sim`` (cubic L^3, 16^3 blocks),
    drawn from its own generator seeded with (seed, sim) so that any member can
    be materialised without drawing the others."""
    rng = np.random.default_rng([seed, sim])
    G = random_state(rng, (L, L, L))
    h = 1.0 / L
    return Problem(f"srv{sim}", n, (L // n,) * 3, (h, h, h), (PERIODIC,) * 3, 1.4,
                   to_compact(G, n), steps=1)


def uniform(n: int = 16, nb=(2, 2, 2), rho=1.3, vel=(0.3, -0.2, 0.1), p=0.7, gamma=1.4,
            bc=(PERIODIC,) * 3, dx=None) -> Problem:
    """A uniform state (for exact-preservation checks)."""
    X, Y, Z = nb[0] * n, nb[1] * n, nb[2] * n
    one = np.ones((Z, Y, X))
    G = conserved(rho * one, vel[0] * one, vel[1] * one, vel[2] * one, p * one, gamma)
    h = dx if dx is not None else (1.0 / X,) * 3
    return Problem("uniform", n, tuple(nb), tuple(h), tuple(bc), gamma, to_compact(G, n))


def from_primitive(name: str, n: int, rho, u, v, w, p, gamma: float, dx, bc) -> Problem:
    """Blocked problem from primitive global fields [Z, Y, X] (helper for tests)."""
    G = conserved(rho, u, v, w, p, gamma)
    Z, Y, X = G.shape[1:]
    return Problem(name, n, (X // n, Y // n, Z // n), tuple(dx), tuple(bc), gamma, to_compact(G, n))


def served_state_device(sim: int, L: int, out, seed: int = 3, n: int = 16, gamma: float = 1.4):
    """Initial state of served simulation ``sim`` drawn on the device into the
    torch tensor ``out`` ([nblk, 5, n, n, n], compact blocked layout): the
    ensemble's random state (rho, p log-normal with sigma 0.3; u, v, w normal
    with sigma 0.2) from torch's device generator seeded with
    seed * 1000003 + sim, so a served population of any size materialises on
    first use without host-side generation or transfer."""
    import torch

    g = torch.Generator(device=out.device)
    g.manual_seed(seed * 1000003 + sim)
    shape = (L, L, L)
    kw = dict(generator=g, device=out.device, dtype=torch.float64)
    rho = torch.exp(0.3 * torch.randn(shape, **kw))
    p = torch.exp(0.3 * torch.randn(shape, **kw))
    u = 0.2 * torch.randn(shape, **kw)
    v = 0.2 * torch.randn(shape, **kw)
    w = 0.2 * torch.randn(shape, **kw)
    G = torch.stack([rho, rho * u, rho * v, rho * w,
                     p / (gamma - 1.0) + 0.5 * rho * ((u * u + v * v) + w * w)])
    nb = L // n
    out.copy_(G.reshape(5, nb, n, nb, n, nb, n).permute(1, 3, 5, 0, 2, 4, 6).reshape(nb ** 3, 5, n, n, n))
    return out
