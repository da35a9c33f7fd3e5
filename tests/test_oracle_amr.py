"""Pins of the oracle's two-level static AMR step (the Grid unit's
block-structured refinement: guard fill across refinement jumps,
prolongation, restriction and refluxing).

Checked against facts other than the AMR code itself: no refinement gives
the uniform root step bit for bit; refinement everywhere gives the uniform
fine-grid step bit for bit; composite conservation to roundoff on periodic
grids (the refluxing pin); exact preservation of a uniform state;
prolongation that conserves each root cell and reproduces linear data
exactly; a smooth wave crossing a refined block stays as accurate as on the
root grid alone.
"""
import numpy as np
import pytest

import oracle
from oracle import amr
from paper_2208_11630_amd import ics


def _random_root(nb, n, seed, gamma=1.4):
    rng = np.random.default_rng(seed)
    X, Y, Z = nb[0] * n, nb[1] * n, nb[2] * n
    G = ics.random_state(rng, (Z, Y, X))
    return ics.to_compact(G, n), G


def _fine_from_root(mesh, Ur):
    """Children initialised by piecewise-constant injection (every fine cell
    takes its root cell), consistent with the restriction."""
    n, h = mesh.n, mesh.n // 2
    Uf = np.empty((mesh.nfine, 5, n, n, n))
    for q, r in enumerate(mesh.refined):
        for c in range(8):
            cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
            part = Ur[r, :, cz * h:(cz + 1) * h, cy * h:(cy + 1) * h, cx * h:(cx + 1) * h]
            Uf[8 * q + c] = part.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)
    return Uf


def _totals(mesh, Ur, Uf):
    vol0 = np.prod(mesh.dx)
    leaves = np.flatnonzero(~mesh.refine)
    t = Ur[leaves].sum(axis=(0, 2, 3, 4)) * vol0
    if mesh.nfine:
        t = t + Uf.sum(axis=(0, 2, 3, 4)) * vol0 / 8
    return t


def test_no_refinement_is_the_uniform_step():
    n, nb = 8, (2, 2, 1)
    Ur, G = _random_root(nb, n, 41)
    mesh = amr.Mesh(n, nb, (1 / 16,) * 3, np.zeros(4, bool))
    dt = 0.5 * amr.dt(mesh, Ur, np.zeros((0, 5, n, n, n)), 0.8)
    a, _, cnt = amr.step(mesh, Ur, np.zeros((0, 5, n, n, n)), dt)
    P = ics.Problem("r", n, nb, mesh.dx, mesh.bc, 1.4, Ur)
    g = oracle.Grid(n, nb, mesh.dx, mesh.bc, 1.4, 1e-10, 4)
    b, cnt2 = oracle.step(g, P.U.copy(), dt)
    assert np.array_equal(a, ics.interior(b, n))
    assert cnt.tolist() == cnt2.tolist()


def test_refinement_everywhere_is_the_uniform_fine_step():
    n, nb = 8, (2, 1, 1)
    Ur, _ = _random_root(nb, n, 42)
    mesh = amr.Mesh(n, nb, (1 / 16,) * 3, np.ones(2, bool))
    rng = np.random.default_rng(43)
    Gf = ics.random_state(rng, (2 * n, 2 * n, 4 * n))          # the fine field (z, y, x)
    Uf = np.empty((mesh.nfine, 5, n, n, n))
    for f in range(mesh.nfine):
        x0, y0, z0 = mesh.fine_origin(f)
        Uf[f] = Gf[:, z0:z0 + n, y0:y0 + n, x0:x0 + n]
    Ur2 = Ur.copy()
    amr.restrict(mesh, Ur2, Uf)
    dt = 0.5 * amr.dt(mesh, Ur2, Uf, 0.8)
    _, Uf_new, _ = amr.step(mesh, Ur2, Uf, dt)
    gf = oracle.Grid(n, (4, 2, 2), (1 / 32,) * 3, mesh.bc, 1.4, 1e-10, 4)
    Pf = ics.Problem("f", n, (4, 2, 2), gf.dx, mesh.bc, 1.4, ics.to_compact(Gf, n))
    ref, _ = oracle.step(gf, Pf.U.copy(), dt)
    Gref = ics.from_blocks(ref, n, (4, 2, 2), 4)
    for f in range(mesh.nfine):
        x0, y0, z0 = mesh.fine_origin(f)
        assert np.array_equal(Uf_new[f], Gref[:, z0:z0 + n, y0:y0 + n, x0:x0 + n]), f


@pytest.mark.parametrize("refined", [[3], [0, 5], [1, 2, 6]])
def test_composite_conservation_periodic(refined):
    n, nb = 8, (2, 2, 2)
    Ur, _ = _random_root(nb, n, 44)
    flags = np.zeros(8, bool)
    flags[refined] = True
    mesh = amr.Mesh(n, nb, (1 / 16,) * 3, flags)
    Uf = _fine_from_root(mesh, Ur)
    t0 = _totals(mesh, Ur, Uf)
    Ur1, Uf1 = Ur, Uf
    for _ in range(2):
        d = amr.dt(mesh, Ur1, Uf1, 0.8)
        Ur1, Uf1, cnt = amr.step(mesh, Ur1, Uf1, d)
        assert cnt[2] == 0
    t1 = _totals(mesh, Ur1, Uf1)
    scale = _totals(mesh, np.abs(Ur), np.abs(Uf))
    assert np.all(np.abs(t1 - t0) <= 1e-13 * scale), (t1 - t0) / scale


def test_uniform_state_preserved_with_refinement():
    n, nb = 8, (2, 2, 1)
    P = ics.uniform(n=n, nb=nb, bc=(0, 1, 0))
    mesh = amr.Mesh(n, nb, P.dx, np.array([1, 0, 0, 1], bool), bc=(0, 1, 0))
    Ur = P.Uc.copy()
    Uf = _fine_from_root(mesh, Ur)
    Ur1, Uf1, cnt = amr.step(mesh, Ur, Uf, 1e-3)
    assert np.array_equal(Ur1, Ur) and np.array_equal(Uf1, Uf)


def test_prolongation_conserves_root_cells_and_is_exact_for_linear_data():
    """Fine guard cells over unrefined root cells: every complete 2x2x2 group
    averages to its root cell; for linear conserved fields (no limiting),
    each prolonged value is the field at the fine cell centre."""
    n, nb = 8, (2, 2, 2)
    X, Y, Z = nb[0] * n, nb[1] * n, nb[2] * n
    z, y, x = np.meshgrid(np.arange(Z) + 0.5, np.arange(Y) + 0.5, np.arange(X) + 0.5, indexing="ij")
    G = np.stack([2.0 + 0.01 * x + 0.02 * y - 0.01 * z, 0.1 + 0.003 * x, -0.2 + 0.004 * z,
                  0.05 + 0.001 * y, 8.0 + 0.01 * (x + y + z)])
    Ur = ics.to_compact(G, n)
    flags = np.zeros(8, bool)
    flags[7] = True                            # the block at (1, 1, 1): guards reach in from lower blocks
    mesh = amr.Mesh(n, nb, (1.0, 1.0, 1.0), flags, bc=(1, 1, 1))
    Uf = _fine_from_root(mesh, Ur)
    f = 0                                      # child (0, 0, 0): its low guards lie over unrefined blocks
    V = amr.fine_guarded(mesh, Ur, Uf, f)
    x0, y0, z0 = mesh.fine_origin(f)
    # fine cells -4..-1 along x (root cells just below the refined block), interior range in y, z
    xs = np.arange(-4, 0)
    sub = V[:, 4:4 + n, 4:4 + n, 0:4]          # (v, z, y, x) with x = -4..-1
    fx = (x0 + xs + 0.5) / 2.0
    fy = (y0 + np.arange(n) + 0.5) / 2.0
    fz = (z0 + np.arange(n) + 0.5) / 2.0
    FZ, FY, FX = np.meshgrid(fz, fy, fx, indexing="ij")
    exact = np.stack([2.0 + 0.01 * FX + 0.02 * FY - 0.01 * FZ, 0.1 + 0.003 * FX, -0.2 + 0.004 * FZ,
                      0.05 + 0.001 * FY, 8.0 + 0.01 * (FX + FY + FZ)])
    np.testing.assert_allclose(sub, exact, rtol=1e-14, atol=1e-15)
    # conservation of each root cell by its eight children
    groups = sub.reshape(5, n // 2, 2, n // 2, 2, 2, 2).mean(axis=(2, 4, 6))
    rc = Ur[mesh.refined[0] - 1]               # root block (0, 1, 1): cells x = n-2, n-1, y, z = 0..n/2-1
    ref = rc[:, :n // 2, :n // 2, n - 2:]
    np.testing.assert_allclose(groups, ref, rtol=1e-14)


def test_smooth_wave_through_a_refined_block():
    """An entropy wave advected along x across a refined root block: the
    composite error against the exact profile is no larger than the root
    grid's alone, and the state stays physical."""
    n, nb = 8, (4, 1, 1)
    L = nb[0] * n
    h = 1.0 / L
    x = (np.arange(L) + 0.5) * h
    one = np.ones((n, n, L))
    rho = np.broadcast_to(1.0 + 0.2 * np.sin(2 * np.pi * x), (n, n, L)).copy()
    P = ics.from_primitive("w", n, rho, one, 0 * one, 0 * one, one, 1.4, (h, h, h), (0, 0, 0))
    flags = np.array([0, 1, 0, 0], bool)
    mesh = amr.Mesh(n, nb, (h, h, h), flags)
    Ur = P.Uc.copy()
    # children from the exact profile at the fine cell centres
    Uf = np.empty((mesh.nfine, 5, n, n, n))
    for f in range(mesh.nfine):
        x0, y0, z0 = mesh.fine_origin(f)
        xf = (x0 + np.arange(n) + 0.5) * h / 2
        r = np.broadcast_to(1.0 + 0.2 * np.sin(2 * np.pi * xf), (n, n, n))
        Uf[f] = ics.conserved(r, np.ones_like(r), 0 * r, 0 * r, np.ones_like(r), 1.4)
    amr.restrict(mesh, Ur, Uf)
    g = oracle.Grid(n, nb, (h, h, h), (0, 0, 0), 1.4, 1e-10, 4)
    U0 = P.U.copy()
    T, t = 0.3, 0.0
    while t < T - 1e-14:
        d = min(amr.dt(mesh, Ur, Uf, 0.8), T - t)
        Ur, Uf, cnt = amr.step(mesh, Ur, Uf, d)
        U0, _ = oracle.step(g, U0, d)
        t += d
        assert cnt[2] == 0
    exact = 1.0 + 0.2 * np.sin(2 * np.pi * (x - t))
    e_amr = 0.0
    for b in np.flatnonzero(~mesh.refine):
        e_amr += np.abs(Ur[b, 0, 0, 0, :] - exact[b * n:(b + 1) * n]).sum() * h
    for f in range(mesh.nfine):
        x0, y0, z0 = mesh.fine_origin(f)
        if y0 or z0:
            continue
        xf = (x0 + np.arange(n) + 0.5) * h / 2
        e_amr += np.abs(Uf[f, 0, 0, 0, :] - (1.0 + 0.2 * np.sin(2 * np.pi * (xf - t)))).sum() * h / 2
    e_root = np.abs(ics.from_blocks(U0, n, nb, 4)[0, 0, 0] - exact).sum() * h
    assert e_amr <= 1.05 * e_root, (e_amr, e_root)


def test_sampled_step_equals_full_step():
    """The per-block sampled step (used to check the full-size mesh) gives
    exactly what the whole-mesh step gives on the chosen blocks."""
    n, nb = 8, (3, 2, 2)
    Ur, _ = _random_root(nb, n, 45)
    flags = np.zeros(12, bool)
    flags[[0, 5, 7]] = True
    mesh = amr.Mesh(n, nb, (1 / 24,) * 3, flags, bc=(1, 0, 1))
    Uf = _fine_from_root(mesh, Ur)
    rng = np.random.default_rng(46)
    Uf *= 1.0 + 0.05 * rng.random(Uf.shape)            # fine detail beyond the injection
    amr.restrict(mesh, Ur, Uf)
    dt = amr.dt(mesh, Ur, Uf, 0.8)
    R, F, _ = amr.step(mesh, Ur, Uf, dt)
    roots = [1, 4, 6, 11]                                # 1, 4, 6: next to refined blocks
    fines = [0, 9, mesh.nfine - 1]
    out_r, out_f = amr.step_sampled(mesh, Ur, Uf, dt, roots=roots, fines=fines, refined=[5])
    for b in roots + [5]:
        assert np.array_equal(out_r[b], R[b]), b
    for f in fines:
        assert np.array_equal(out_f[f], F[f]), f
    # block 1 meets refined block 0 across its low x face and refined block 7
    # across its high z face: refluxing changes exactly those two layers
    g = oracle.Grid(n, (1, 1, 1), mesh.dx, mesh.bc, 1.4, 1e-10, 4)
    plain, _, _ = amr._leaf_step(g, np.ascontiguousarray(amr.root_guarded(mesh, Ur, 1)[None]), 0, dt)
    assert not np.array_equal(plain[:, :, :, 0], R[1][:, :, :, 0])
    assert not np.array_equal(plain[:, -1], R[1][:, -1])
    assert np.array_equal(plain[:, :-1, :, 1:], R[1][:, :-1, :, 1:])
