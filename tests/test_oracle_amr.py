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


# ---- adaptivity -----------------------------------------------------------

def _prim_state(rho, p, gamma):
    z = np.zeros_like(rho)
    return ics.conserved(rho, z, z, z, p, gamma)


def test_indicator_lies_in_unit_interval():
    n, nb = 8, (2, 2, 2)
    Ur, _ = _random_root(nb, n, 47)
    mesh = amr.Mesh(n, nb, (1 / 16,) * 3, np.zeros(8, bool))
    E2 = amr.indicator(mesh, Ur)
    assert E2.shape == (8,) and np.all(E2 >= 0.0) and np.all(E2 <= 1.0)
    assert E2.max() > 0.1                          # a random field has curvature everywhere


def test_indicator_vanishes_on_linear_fields():
    """Integer-valued linear density and pressure (gamma = 2, at rest: the
    pressure is recovered exactly): every second difference is exactly 0
    away from the outflow boundaries."""
    n, nb = 8, (4, 3, 3)
    Z, Y, X = nb[2] * n, nb[1] * n, nb[0] * n
    k, j, i = np.meshgrid(np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    rho = 2.0 + i + 2 * j + 3 * k
    p = 5.0 + 3 * i + j + 2 * k
    Ur = ics.to_compact(_prim_state(rho.astype(float), p.astype(float), 2.0), n)
    mesh = amr.Mesh(n, nb, (1.0,) * 3, np.zeros(nb[0] * nb[1] * nb[2], bool), bc=(1, 1, 1), gamma=2.0)
    E2 = amr.indicator(mesh, Ur).reshape(nb[2], nb[1], nb[0])
    assert np.all(E2[1:-1, 1:-1, 1:-1] == 0.0)
    assert E2[0, 0, 0] > 0.0                       # the clamped boundary is a kink


@pytest.mark.parametrize("field", ["rho", "p"])
def test_indicator_is_one_at_a_jump_without_the_filter(field):
    """A jump along x and nothing else: with eps = 0 the ratio is exactly 1
    in the two cells beside the jump and 0 (flat: 0/0 taken as 0) elsewhere."""
    n, nb = 8, (4, 2, 1)
    Z, Y, X = nb[2] * n, nb[1] * n, nb[0] * n
    one = np.ones((Z, Y, X))
    step = np.where(np.arange(X) < X // 2 + 3, 1.0, 3.5)[None, None, :] * one
    rho, p = (step, 2.0 * one) if field == "rho" else (2.0 * one, step)
    Ur = ics.to_compact(_prim_state(rho, p, 2.0), n)
    mesh = amr.Mesh(n, nb, (1.0,) * 3, np.zeros(8, bool), bc=(1, 0, 0), gamma=2.0)
    E2 = amr.indicator(mesh, Ur, eps=0.0).reshape(nb[2], nb[1], nb[0])
    # the jump sits between cells X/2+2 and X/2+3: both in block bx = 2
    assert np.all(E2[:, :, 2] == 1.0) and np.all(E2[:, :, [0, 1, 3]] == 0.0)
    # the filter lowers it below 1
    assert np.all(amr.indicator(mesh, Ur, eps=0.01).reshape(nb[2], nb[1], nb[0])[:, :, 2] < 1.0)


def test_refine_flags_rule():
    mesh = amr.Mesh(8, (3, 2, 1), (1.0,) * 3, np.array([1, 1, 1, 0, 0, 0], bool))
    E2 = np.array([0.9, 0.01, 0.3, 0.65, 0.639, 0.039])
    new = amr.refine_flags(mesh, E2, 0.8, 0.2)    # cutoffs squared: 0.64, 0.04
    assert new.tolist() == [True, False, True, True, False, False]


def test_regrid_is_conservative_and_derefinement_returns_the_root_state():
    n, nb = 8, (2, 2, 2)
    Ur, _ = _random_root(nb, n, 48)
    m0 = amr.Mesh(n, nb, (1 / 16,) * 3, np.zeros(8, bool))
    m1, Ur1, Uf1 = amr.regrid(m0, Ur, np.zeros((0, 5, n, n, n)), [0, 1, 0, 0, 1, 0, 0, 1])
    assert m1.nfine == 24
    scale = _totals(m0, np.abs(Ur), np.zeros((0, 5, n, n, n)))
    assert np.all(np.abs(_totals(m1, Ur1, Uf1) - _totals(m0, Ur, np.zeros((0, 5, n, n, n)))) <= 1e-14 * scale)
    # every group of eight children averages to its root cell (to rounding,
    # relative to each variable's scale)
    for v in range(5):
        assert np.abs(Ur1[:, v] - Ur[:, v]).max() <= 2e-15 * np.abs(Ur[:, v]).max(), v
    # derefining everything keeps the root values the children restricted to
    m2, Ur2, Uf2 = amr.regrid(m1, Ur1, Uf1, np.zeros(8, bool))
    assert Uf2.shape[0] == 0 and np.array_equal(Ur2, Ur1)


def test_regrid_keeps_surviving_children_and_prolongs_new_ones():
    n, nb = 8, (2, 2, 2)
    Ur, _ = _random_root(nb, n, 49)
    m0 = amr.Mesh(n, nb, (1 / 16,) * 3, np.array([1, 0, 0, 0, 0, 1, 0, 0], bool))
    rng = np.random.default_rng(50)
    Uf = _fine_from_root(m0, Ur) * (1.0 + 0.05 * rng.random((16, 5, n, n, n)))
    amr.restrict(m0, Ur, Uf)
    m1, Ur1, Uf1 = amr.regrid(m0, Ur, Uf, [0, 0, 0, 0, 0, 1, 0, 1])
    assert np.array_equal(Uf1[0:8], Uf[8:16])                   # block 5's children, now first
    assert np.array_equal(Ur1[0], Ur[0])                        # block 0 derefined: its restriction stays
    # block 7's children are the prolongation of its root cells
    X0, Y0, Z0 = m1.fine_origin(8)
    r = np.arange(n)
    K, J, I = np.meshgrid(r + Z0, r + Y0, r + X0, indexing="ij")
    assert np.array_equal(Uf1[8], amr.prolong(m1, Ur, I.ravel(), J.ravel(), K.ravel()).reshape(5, n, n, n))


def test_regrid_prolongs_linear_data_exactly():
    n, nb = 8, (2, 2, 2)
    X, Y, Z = nb[0] * n, nb[1] * n, nb[2] * n
    z, y, x = np.meshgrid(np.arange(Z) + 0.5, np.arange(Y) + 0.5, np.arange(X) + 0.5, indexing="ij")
    G = np.stack([2.0 + 0.01 * x + 0.02 * y - 0.01 * z, 0.1 + 0.003 * x, -0.2 + 0.004 * z,
                  0.05 + 0.001 * y, 8.0 + 0.01 * (x + y + z)])
    Ur = ics.to_compact(G, n)
    m0 = amr.Mesh(n, nb, (1.0,) * 3, np.zeros(8, bool), bc=(1, 1, 1))
    m1, _, Uf1 = amr.regrid(m0, Ur, np.zeros((0, 5, n, n, n)), [0, 0, 0, 0, 0, 0, 0, 1])
    X0, Y0, Z0 = m1.fine_origin(0)
    fz, fy, fx = np.meshgrid((Z0 + np.arange(n) + 0.5) / 2, (Y0 + np.arange(n) + 0.5) / 2,
                             (X0 + np.arange(n) + 0.5) / 2, indexing="ij")
    exact = np.stack([2.0 + 0.01 * fx + 0.02 * fy - 0.01 * fz, 0.1 + 0.003 * fx, -0.2 + 0.004 * fz,
                      0.05 + 0.001 * fy, 8.0 + 0.01 * (fx + fy + fz)])
    np.testing.assert_allclose(Uf1[0], exact, rtol=1e-14, atol=1e-15)
