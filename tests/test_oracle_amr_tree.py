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
