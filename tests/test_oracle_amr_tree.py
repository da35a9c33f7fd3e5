"""Pins of the oracle's AMR of any depth (oracle.amr_tree): with two levels
it is the two-level step bit for bit; refined everywhere it is the uniform
finest-grid step bit for bit; three levels conserve the composite totals on
periodic meshes, keep a uniform state exactly and prolong linear data
exactly through a refined intermediate level; bad nesting is refused."""
import numpy as np
import pytest

import oracle
from oracle import amr, amr_tree
from paper_2208_11630_amd import ics
from tests.test_oracle_amr import _fine_from_root, _random_root


def _tree_state(t, Ur, seed):
    """Children by injection plus 5% seeded detail, level by level, then
    restricted so the levels agree."""
    rng = np.random.default_rng(seed)
    U = [Ur.copy()]
    n, h = t.n, t.n // 2
    for l in range(1, t.levels):
        Ul = np.empty((t.nblocks(l), 5, n, n, n))
        for i, par in enumerate(t.parent[l]):
            c = i - int(t.child_base[l - 1][par])
            cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
            part = U[l - 1][par, :, cz * h:(cz + 1) * h, cy * h:(cy + 1) * h, cx * h:(cx + 1) * h]
            Ul[i] = part.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)
        Ul *= 1.0 + 0.05 * rng.random(Ul.shape)
        U.append(Ul)
    amr_tree.restrict(t, U)
    return U


def _totals(t, U):
    tot = 0.0
    for l in range(t.levels):
        lv = t.leaves(l)
        tot = tot + U[l][lv].sum(axis=(0, 2, 3, 4)) * (1.0 / 8 ** l)
    return tot


@pytest.mark.parametrize("nb,refined,bc", [((3, 2, 2), [0, 5, 7], (1, 0, 1)), ((2, 2, 2), [3], (0, 0, 0)),
                                           ((2, 1, 1), [0, 1], (0, 0, 0))])
def test_two_levels_are_the_two_level_step(nb, refined, bc):
    n = 8
    Ur, _ = _random_root(nb, n, 71)
    flags = np.zeros(nb[0] * nb[1] * nb[2], bool)
    flags[refined] = True
    mesh = amr.Mesh(n, nb, (1 / 24,) * 3, flags, bc=bc)
    Uf = _fine_from_root(mesh, Ur) * (1.0 + 0.05 * np.random.default_rng(72).random((mesh.nfine, 5, n, n, n)))
    amr.restrict(mesh, Ur, Uf)
    t = amr_tree.Tree(n, nb, (1 / 24,) * 3, [flags], bc=bc)
    dt = amr.dt(mesh, Ur, Uf, 0.8)
    assert amr_tree.dt(t, [Ur, Uf], 0.8) == dt
    R, F, c = amr.step(mesh, Ur, Uf, dt)
    new, c2 = amr_tree.step(t, [Ur, Uf], dt)
    assert np.array_equal(new[0], R) and np.array_equal(new[1], F) and c.tolist() == c2.tolist()


def test_refined_everywhere_is_the_uniform_finest_step():
    n, nb = 8, (1, 1, 1)
    t = amr_tree.Tree(n, nb, (1 / 8,) * 3, [[True], [True] * 8])
    assert t.levels == 3 and t.nblocks(2) == 64
    rng = np.random.default_rng(73)
    Gf = ics.random_state(rng, (4 * n, 4 * n, 4 * n))              # the finest field
    U = [np.zeros((1, 5, n, n, n)), np.zeros((8, 5, n, n, n)), np.empty((64, 5, n, n, n))]
    for i, (x, y, z) in enumerate(t.pos[2]):
        U[2][i] = Gf[:, z * n:(z + 1) * n, y * n:(y + 1) * n, x * n:(x + 1) * n]
    amr_tree.restrict(t, U)
    dt = 0.5 * amr_tree.dt(t, U, 0.8)
    new, _ = amr_tree.step(t, U, dt)
    g = oracle.Grid(n, (4, 4, 4), (1 / 32,) * 3, (0, 0, 0), 1.4, 1e-10, 4)
    P = ics.Problem("f", n, (4, 4, 4), g.dx, (0, 0, 0), 1.4, ics.to_compact(Gf, n))
    ref, _ = oracle.step(g, P.U.copy(), dt)
    Gref = ics.from_blocks(ref, n, (4, 4, 4), 4)
    for i, (x, y, z) in enumerate(t.pos[2]):
        assert np.array_equal(new[2][i], Gref[:, z * n:(z + 1) * n, y * n:(y + 1) * n, x * n:(x + 1) * n]), i


def _three_levels(seed, bc=(0, 0, 0)):
    """4x4x4 root blocks of 8^3: the 3x3x3 cube of blocks at the low corner
    refined, and four of the eight children of its centre block refined
    again (their 26 level-1 neighbours all lie inside the cube)."""
    n, nb = 8, (4, 4, 4)
    f0 = np.zeros(64, bool)
    for b in range(64):
        f0[b] = b % 4 <= 2 and (b // 4) % 4 <= 2 and b // 16 <= 2
    t1 = amr_tree.Tree(n, nb, (1 / 32,) * 3, [f0], bc=bc)
    centre = 1 + 4 * (1 + 4 * 1)
    base = int(t1.child_base[0][centre])
    f1 = np.zeros(t1.nblocks(1), bool)
    f1[[base + 0, base + 3, base + 5, base + 6]] = True
    t = amr_tree.Tree(n, nb, (1 / 32,) * 3, [f0, f1], bc=bc)
    Ur, _ = _random_root(nb, n, seed)
    return t, _tree_state(t, Ur, seed + 1)


def test_three_levels_conserve_on_periodic_meshes():
    t, U = _three_levels(74)
    assert t.levels == 3
    t0 = _totals(t, U)
    scale = _totals(t, [np.abs(u) for u in U])
    for _ in range(2):
        U, cnt = amr_tree.step(t, U, amr_tree.dt(t, U, 0.8))
        assert cnt[2] == 0
    assert np.all(np.abs(_totals(t, U) - t0) <= 1e-13 * scale)
    # every refined block holds, to rounding, the total of its leaf
    # descendants (restriction runs finest level first)
    def leaf_total(l, b):
        if not t.refine[l][b]:
            return U[l][b].sum(axis=(1, 2, 3)) / 8 ** l
        base = int(t.child_base[l][b])
        return sum(leaf_total(l + 1, base + c) for c in range(8))
    for l in range(t.levels - 1):
        for b in np.flatnonzero(t.refine[l]):
            own = U[l][b].sum(axis=(1, 2, 3)) / 8 ** l
            assert np.all(np.abs(own - leaf_total(l, b)) <= 1e-13 * np.abs(own).max()), (l, b)


def test_three_levels_keep_a_uniform_state():
    t, U = _three_levels(75, bc=(1, 0, 1))
    P = ics.uniform(n=8, nb=(4, 4, 4), bc=(1, 0, 1))
    U = [np.broadcast_to(P.Uc[0], u.shape).copy() for u in U]
    new, _ = amr_tree.step(t, U, 1e-3)
    assert all(np.array_equal(a, b) for a, b in zip(new, U))


def test_linear_data_is_prolonged_exactly_through_a_middle_level():
    """Level-1 blocks hold the exact linear field at their cell centres;
    guards of level-2 blocks over unrefined level-1 regions are prolonged
    from them and equal the field at level-2 centres."""
    t, _ = _three_levels(76, bc=(1, 1, 1))
    n = t.n

    def field(l, I, J, K):
        h = 1.0 / (1 << l)
        x, y, z = (I + 0.5) * h, (J + 0.5) * h, (K + 0.5) * h
        return np.stack([2.0 + 0.01 * x + 0.02 * y - 0.01 * z, 0.1 + 0.003 * x, -0.2 + 0.004 * z,
                         0.05 + 0.001 * y, 8.0 + 0.01 * (x + y + z)])

    U = []
    r = np.arange(n)
    for l in range(t.levels):
        Ul = np.empty((t.nblocks(l), 5, n, n, n))
        for i, (bx, by, bz) in enumerate(t.pos[l]):
            K, J, I = np.meshgrid(r + bz * n, r + by * n, r + bx * n, indexing="ij")
            Ul[i] = field(l, I, J, K)
        U.append(Ul)
    b = 0
    V = amr_tree.guarded(t, U, 2, b)
    X0, Y0, Z0 = (t.pos[2][b] * n).tolist()
    rr = np.arange(-4, n + 4)
    K, J, I = np.meshgrid(rr + Z0, rr + Y0, rr + X0, indexing="ij")
    np.testing.assert_allclose(V, field(2, I, J, K), rtol=1e-14, atol=1e-15)


def test_bad_nesting_is_refused():
    n, nb = 8, (3, 1, 1)
    f0 = np.array([0, 1, 0], bool)
    f1 = np.zeros(8, bool)
    f1[0] = True           # its level-1 neighbours at x-1 lie in unrefined root block 0
    with pytest.raises(ValueError):
        amr_tree.Tree(n, nb, (1.0,) * 3, [f0, f1], bc=(1, 1, 1))


# ---- adaptivity of a tree ------------------------------------------------------

def test_tree_indicator_on_root_leaves_is_the_two_level_indicator():
    """Neighbours of root leaves all exist at level 0: the per-leaf indicator
    equals the root indicator of oracle.amr bit for bit on the leaves."""
    n, nb = 8, (3, 2, 2)
    Ur, _ = _random_root(nb, n, 92)
    flags = np.zeros(12, bool)
    flags[[0, 5, 7]] = True
    mesh = amr.Mesh(n, nb, (1 / 24,) * 3, flags, bc=(1, 0, 1))
    Uf = _fine_from_root(mesh, Ur)
    amr.restrict(mesh, Ur, Uf)
    t = amr_tree.Tree(n, nb, (1 / 24,) * 3, [flags], bc=(1, 0, 1))
    E = amr_tree.indicator(t, [Ur, Uf])
    ref = amr.indicator(mesh, Ur)
    leaves = np.flatnonzero(~flags)
    assert np.array_equal(E[0][leaves], ref[leaves]) and np.all(E[0][flags] == 0.0)
    assert np.all(E[1] >= 0.0) and np.all(E[1] <= 1.0) and E[1].max() > 0.0


def test_tree_indicator_vanishes_on_linear_fields_inside_a_level():
    """Integer-valued linear density and pressure (gamma 2, at rest) on a
    three-level tree: leaves whose neighbours all exist at their level have
    indicator 0 exactly (the zero-gradient stand-in for a missing coarser
    neighbour is a kink, so leaves at a refinement jump may not)."""
    t, _ = _three_levels(93, bc=(0, 0, 0))
    n = t.n
    t = amr_tree.Tree(n, t.nb0, t.dx0, t.refine, bc=(0, 0, 0), gamma=2.0)
    U = []
    r = np.arange(n)
    for l in range(t.levels):
        Ul = np.empty((t.nblocks(l), 5, n, n, n))
        for i, (bx, by, bz) in enumerate(t.pos[l]):
            K, J, I = np.meshgrid(r + bz * n, r + by * n, r + bx * n, indexing="ij")
            # periodic in the interior blocks only: keep the field linear away from the wrap
            rho = 500.0 + I + 2 * J + 3 * K
            p = 700.0 + 3 * I + J + 2 * K
            z = np.zeros_like(rho, dtype=float)
            Ul[i] = ics.conserved(rho.astype(float), z, z, z, p.astype(float), 2.0)
        U.append(Ul)
    E = amr_tree.indicator(t, U, eps=0.01)
    checked = 0
    for l in range(t.levels):
        nbl = t.nb(l)
        for b in t.leaves(l):
            x, y, z = t.pos[l][b]
            inside = all(1 <= c <= nbl[d] - 2 for d, c in enumerate((x, y, z)))
            full = all(t.block_at(l, x + a, y + bb, z + c) >= 0 for a in (-1, 0, 1) for bb in (-1, 0, 1)
                       for c in (-1, 0, 1))
            if inside and full:
                assert E[l][b] == 0.0, (l, b)
                checked += 1
    assert checked > 10


@pytest.mark.parametrize("seed", [94, 95, 96])
def test_tree_flags_always_give_a_nested_tree(seed):
    """Random indicators on a three-level tree: the rule's flags build a
    tree that passes the nesting check; every leaf above the refine cutoff
    below the deepest level is refined; a block loses its children only if
    all were leaves below the derefine cutoff."""
    t, _ = _three_levels(seed)
    rng = np.random.default_rng(seed)
    E2 = [rng.random(t.nblocks(l)) for l in range(t.levels)]
    for rc, dc in [(0.95, 0.5), (0.7, 0.3), (0.99, 0.05)]:
        flags = amr_tree.refine_flags(t, E2, rc, dc, max_levels=4)
        new = amr_tree.Tree(t.n, t.nb0, t.dx0, flags, bc=t.bc)         # raises on bad nesting
        for l in range(t.levels):
            for b in t.leaves(l):
                if E2[l][b] > rc * rc and l + 1 < 4:
                    q = new.block_at(l, *t.pos[l][b])
                    assert q >= 0 and new.refine[l][q], (l, b)
            for r in np.flatnonzero(t.refine[l]):
                q = new.block_at(l, *t.pos[l][r])
                if q >= 0 and not new.refine[l][q]:
                    base = int(t.child_base[l][r])
                    assert all(not t.refine[l + 1][k] and E2[l + 1][k] < dc * dc for k in range(base, base + 8))


def test_tree_regrid_conserves_and_keeps_surviving_blocks():
    t, U = _three_levels(97)
    rng = np.random.default_rng(98)
    E2 = [rng.random(t.nblocks(l)) for l in range(t.levels)]
    flags = amr_tree.refine_flags(t, E2, 0.9, 0.6, max_levels=4)
    new, V = amr_tree.regrid(t, U, flags)
    assert new.levels >= 3
    tot = lambda tt, W: sum(W[l][tt.leaves(l)].sum(axis=(0, 2, 3, 4)) / 8 ** l for l in range(tt.levels))
    scale = tot(t, [np.abs(u) for u in U])
    assert np.all(np.abs(tot(new, V) - tot(t, U)) <= 1e-13 * scale)
    kept = 0
    for l in range(1, new.levels):
        for i, p in enumerate(new.pos[l].tolist()):
            old = t.block_at(l, *p) if l < t.levels else -1
            if old >= 0 and not new.refine[l][i] and not t.refine[l][old]:
                assert np.array_equal(V[l][i], U[l][old])
                kept += 1
    assert kept > 0
    # every refined block holds the restriction of its children, exactly as restrict() forms it
    W = [v.copy() for v in V]
    amr_tree.restrict(new, W)
    assert all(np.array_equal(a, b) for a, b in zip(V, W))


def test_tree_indicator_is_zero_for_a_uniform_state():
    """Flat fields at every level, refinement jumps included (a missing
    coarser neighbour stands in with the cell's own value)."""
    t, U = _three_levels(99, bc=(1, 0, 1))
    P = ics.uniform(n=8, nb=(4, 4, 4), bc=(1, 0, 1))
    U = [np.broadcast_to(P.Uc[0], u.shape).copy() for u in U]
    E = amr_tree.indicator(t, U)
    assert all(np.all(e == 0.0) for e in E)


def test_tree_regrid_prolongs_linear_data_exactly():
    """A new level-2 block over linear data: the field at its cell centres."""
    t, _ = _three_levels(100, bc=(1, 1, 1))
    n = t.n

    def field(l, I, J, K):
        h = 1.0 / (1 << l)
        x, y, z = (I + 0.5) * h, (J + 0.5) * h, (K + 0.5) * h
        return np.stack([2.0 + 0.01 * x + 0.02 * y - 0.01 * z, 0.1 + 0.003 * x, -0.2 + 0.004 * z,
                         0.05 + 0.001 * y, 8.0 + 0.01 * (x + y + z)])

    r = np.arange(n)
    U = []
    for l in range(t.levels):
        Ul = np.empty((t.nblocks(l), 5, n, n, n))
        for i, (bx, by, bz) in enumerate(t.pos[l]):
            K, J, I = np.meshgrid(r + bz * n, r + by * n, r + bx * n, indexing="ij")
            Ul[i] = field(l, I, J, K)
        U.append(Ul)
    R = amr_tree._refined_sets(t)
    base = int(t.child_base[0][1 + 4 * (1 + 4 * 1)])
    R[1].add(tuple(t.pos[1][base + 1].tolist()))    # a new refinement inside the centre block
    new, V = amr_tree.regrid(t, U, amr_tree._flags_from_sets(t, R))
    fresh = [i for i, p in enumerate(new.pos[2].tolist()) if t.block_at(2, *p) < 0]
    assert len(fresh) == 8
    for i in fresh:
        bx, by, bz = new.pos[2][i]
        K, J, I = np.meshgrid(r + bz * n, r + by * n, r + bx * n, indexing="ij")
        np.testing.assert_allclose(V[2][i], field(2, I, J, K), rtol=1e-14, atol=1e-15)
