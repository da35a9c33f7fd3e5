"""Parity of the two-level static AMR step of the HIP path (hydro_amr_*)
with the CPU oracle's (oracle.amr), through the C ABI.

Bar as for the uniform grid: after every step, per conserved variable, the
normwise relative error over all leaf and restricted cells is at most 1e-12;
the dt each side chooses agrees to 1e-14; the event counters match.  Inputs:
a seeded field at the fine resolution (random per cell, or smooth with a
pressure jump), the fine blocks cut from it and the root state its 2x2x2
means, so the two levels start consistent.
"""
import numpy as np
import pytest

import oracle
from oracle import amr
from paper_2208_11630_amd import ics

pytestmark = pytest.mark.gpu

TOL = 1e-12
DT_TOL = 1e-14


@pytest.fixture(scope="module")
def hy():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2208_11630_amd import hydro

    hydro.lib()
    return hydro


def fine_field(nb, n, kind, seed, gamma=1.4):
    """Conserved field [5, Z, Y, X] at the fine resolution (2 n nb per axis)."""
    shape = (2 * n * nb[2], 2 * n * nb[1], 2 * n * nb[0])
    rng = np.random.default_rng(seed)
    if kind == "random":
        return ics.random_state(rng, shape, gamma)
    z, y, x = np.meshgrid(*[(np.arange(s) + 0.5) / s for s in shape], indexing="ij")
    rho = 1.0 + 0.5 * np.exp(-40.0 * ((x - 0.4) ** 2 + (y - 0.5) ** 2 + (z - 0.45) ** 2))
    u = 0.6 * np.tanh(20.0 * (y - 0.5))
    v = 0.05 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * z)
    w = 0.1 * np.cos(2 * np.pi * y)
    p = np.where((x - 0.3) ** 2 + (y - 0.6) ** 2 + (z - 0.5) ** 2 < 0.04, 10.0, 1.0)
    return ics.conserved(rho, u, v, w, p, gamma)


def mesh_state(mesh, F):
    """Root state (2x2x2 means of the field) and the fine blocks cut from it."""
    n = mesh.n
    Z, Y, X = F.shape[1:]
    coarse = F.reshape(5, Z // 2, 2, Y // 2, 2, X // 2, 2).mean(axis=(2, 4, 6))
    Ur = ics.to_compact(coarse, n)
    Uf = np.empty((mesh.nfine, 5, n, n, n))
    for f in range(mesh.nfine):
        x0, y0, z0 = mesh.fine_origin(f)
        Uf[f] = F[:, z0:z0 + n, y0:y0 + n, x0:x0 + n]
    amr.restrict(mesh, Ur, Uf)
    return Ur, Uf


def rel_errors(A, B):
    """Per-variable normwise relative error over compact blocks [nb, 5, ...]."""
    mom = np.sqrt((B[:, 1] ** 2 + B[:, 2] ** 2) + B[:, 3] ** 2).max()
    out = []
    for v in range(5):
        den = mom if v in (1, 2, 3) else np.abs(B[:, v]).max()
        out.append(np.abs(A[:, v] - B[:, v]).max() / (den if den > 0 else np.abs(B[:, 0]).max()))
    return np.array(out)


def assert_close(gpu, ref, what):
    A = np.concatenate([gpu[0], gpu[1]]) if ref[1].size else gpu[0]
    B = np.concatenate([ref[0], ref[1]]) if ref[1].size else ref[0]
    e = rel_errors(A, B)
    assert np.all(e <= TOL), f"{what}: relative errors {e}"


# name: (n, nb, refined root blocks, bc, field kind, seed)
CASES = {
    "n8_2x2x2_one": (8, (2, 2, 2), [3], (0, 0, 0), "random", 51),
    "n8_3x2x2_mixed_bc": (8, (3, 2, 2), [0, 5, 7], (1, 0, 1), "random", 52),
    "n16_2x2x1_periodic_z1": (16, (2, 2, 1), [1, 2], (0, 0, 0), "smooth", 53),
    "n8_4x1x1_outflow": (8, (4, 1, 1), [1, 2], (1, 1, 1), "smooth", 54),
    "n8_all_refined": (8, (2, 1, 1), [0, 1], (0, 0, 0), "random", 55),
    "n8_none_refined": (8, (2, 2, 1), [], (0, 1, 0), "random", 56),
    "n32_2x1x1": (32, (2, 1, 1), [1], (0, 0, 0), "smooth", 57),
}


def make(hy, case):
    n, nb, refined, bc, kind, seed = CASES[case]
    flags = np.zeros(nb[0] * nb[1] * nb[2], bool)
    flags[refined] = True
    h = 1.0 / (nb[0] * n)
    mesh = amr.Mesh(n, nb, (h, h, h), flags, bc=bc)
    Ur, Uf = mesh_state(mesh, fine_field(nb, n, kind, seed))
    hi = tuple(nb[d] * n * h for d in range(3))
    A = hy.Amr(n, nb, flags.tolist(), hi=hi, bc=bc)
    A.upload(Ur, Uf if mesh.nfine else None)
    return mesh, Ur, Uf, A


@pytest.mark.parametrize("case", list(CASES))
def test_amr_trajectory_parity(hy, case):
    """Three steps, dt from the oracle's CFL rule; the device's dt agrees."""
    print(f"\n[amr] {case}", flush=True)
    mesh, Ur, Uf, A = make(hy, case)
    cnt_ref = np.zeros(3, np.int64)
    for s in range(3):
        dt = amr.dt(mesh, Ur, Uf, 0.8)
        d_gpu = A.dt(0.8)
        assert abs(d_gpu / dt - 1.0) <= DT_TOL, (s, d_gpu, dt)
        Ur, Uf, c = amr.step(mesh, Ur, Uf, dt)
        cnt_ref += c
        A.step(dt)
        assert_close(A.download(), (Ur, Uf), f"{case} step {s}")
    assert A.counters().tolist() == cnt_ref.tolist()
    A.close()


@pytest.mark.parametrize("case", ["n8_3x2x2_mixed_bc", "n16_2x2x1_periodic_z1", "n8_all_refined", "n32_2x1x1"])
def test_amr_trajectory_with_device_dt(hy, case):
    """Three steps whose dt the device forms from the signal speed the
    previous step reduced (fused into the leaf steps and refluxing)."""
    print(f"\n[amr] device dt {case}", flush=True)
    mesh, Ur, Uf, A = make(hy, case)
    for s in range(3):
        dt = amr.dt(mesh, Ur, Uf, 0.8)
        A.step_cfl(0.8)
        assert abs(A.last_dt() / dt - 1.0) <= DT_TOL, (s, A.last_dt(), dt)
        Ur, Uf, _ = amr.step(mesh, Ur, Uf, dt)
        assert_close(A.download(), (Ur, Uf), f"{case} device-dt step {s}")
    # the signal speed the last step reduced gives the next dt
    assert abs(A.dt(0.8) / amr.dt(mesh, Ur, Uf, 0.8) - 1.0) <= DT_TOL
    A.close()


def test_amr_conserves_composite_totals(hy):
    """Periodic mesh: leaf totals weighted by cell volume change by roundoff only."""
    mesh, Ur, Uf, A = make(hy, "n8_2x2x2_one")
    vol = [1.0, 1.0 / 8]

    def totals(R, F):
        leaves = np.flatnonzero(~mesh.refine)
        return R[leaves].sum(axis=(0, 2, 3, 4)) * vol[0] + F.sum(axis=(0, 2, 3, 4)) * vol[1]

    t0 = totals(Ur, Uf)
    scale = totals(np.abs(Ur), np.abs(Uf))
    for _ in range(3):
        A.step(A.dt(0.8))
    R, F = A.download()
    assert np.all(np.abs(totals(R, F) - t0) <= 1e-13 * scale)
    A.close()


def test_amr_without_refinement_equals_uniform_step(hy):
    """No flagged block: the AMR step is the uniform grid's step."""
    n, nb = 16, (2, 1, 2)
    rng = np.random.default_rng(58)
    G = ics.random_state(rng, (nb[2] * n, nb[1] * n, nb[0] * n))
    Ur = ics.to_compact(G, n)
    h = 1.0 / 32
    A = hy.Amr(n, nb, [0] * 4, hi=(nb[0] * n * h, nb[1] * n * h, nb[2] * n * h), bc=(1, 0, 1))
    A.upload(Ur)
    g = oracle.Grid(n, nb, (h, h, h), (1, 0, 1), 1.4, 1e-10, 4)
    P = ics.Problem("r", n, nb, (h, h, h), (1, 0, 1), 1.4, Ur)
    dt = oracle.dt(g, P.U, 0.8)
    ref, _ = oracle.step(g, P.U.copy(), dt)
    A.step(dt)
    e = rel_errors(A.download()[0], ics.interior(ref, n))
    assert np.all(e <= TOL), e
    A.close()


def test_amr_abi_rejects_bad_descriptors(hy):
    with pytest.raises(hy.HydroError):
        hy.Amr(12, (2, 1, 1), [0, 1])
    with pytest.raises(hy.HydroError):
        hy.Amr(8, (2, 1, 1), [0, 1], bc=(0, 5, 0))
    A = hy.Amr(8, (2, 1, 1), [0, 1])
    with pytest.raises(hy.HydroError):
        A.step(float("nan"))
    with pytest.raises(hy.HydroError):
        A.step(-1.0)
    A.close()


def test_amr_full_size_sampled_blocks(hy):
    """The two-level Kelvin-Helmholtz mesh the benchmark times (root
    256x256x128 in 16^3 blocks, the 512 blocks of the interface rows
    refined): dt over the whole mesh, then one step checked on sampled root
    leaves (inside a level, next to refined rows, at the periodic edges),
    fine blocks and refined root blocks against the oracle's per-block step."""
    nb, flags, Ur, Uf, dx, gamma = ics.kelvin_helmholtz_amr(root=(256, 256, 128), n=16)
    n = 16
    mesh = amr.Mesh(n, nb, dx, flags, gamma=gamma)
    A = hy.Amr(n, nb, flags.tolist(), hi=tuple(nb[d] * n * dx[d] for d in range(3)), gamma=gamma)
    A.upload(Ur, Uf)
    dt = amr.dt(mesh, Ur, Uf, 0.8)
    d_gpu = A.dt(0.8)
    assert abs(d_gpu / dt - 1.0) <= DT_TOL, (d_gpu, dt)
    A.step(dt)
    R, F = A.download()
    blk = lambda bx, by, bz: bx + nb[0] * (by + nb[1] * bz)
    roots = [blk(5, 7, 3), blk(0, 2, 0), blk(15, 5, 7), blk(3, 10, 4), blk(9, 13, 7), blk(15, 15, 0)]
    assert not flags[roots].any() and flags[[blk(0, 3, 0), blk(15, 4, 7), blk(3, 11, 4), blk(9, 12, 7)]].all()
    refined = [int(mesh.refined[0]), int(mesh.refined[200]), int(mesh.refined[-1])]
    fines = [0, 1, 777, 2048, mesh.nfine - 1]
    out_r, out_f = amr.step_sampled(mesh, Ur, Uf, dt, roots=roots, fines=fines, refined=refined)
    assert_close((np.stack([R[b] for b in out_r]), np.stack([F[f] for f in out_f])),
                 (np.stack(list(out_r.values())), np.stack(list(out_f.values()))), "full-size sampled")
    assert A.counters().tolist() == [0, 0, 0]
    A.close()


# ---- adaptivity --------------------------------------------------------------

ADAPT_CASES = {
    # name: (n, nb, refined, bc, field kind, seed)
    "random_n8": (8, (3, 2, 2), [0, 5, 7], (1, 0, 1), "random", 61),
    "smooth_n16": (16, (2, 2, 2), [1, 6], (0, 0, 0), "smooth", 62),
    "smooth_n8_outflow": (8, (4, 2, 2), [2, 9], (1, 1, 1), "smooth", 63),
}


def _adapt_mesh(hy, case):
    n, nb, refined, bc, kind, seed = ADAPT_CASES[case]
    CASES[case] = ADAPT_CASES[case]
    try:
        return make(hy, case)
    finally:
        del CASES[case]


@pytest.mark.parametrize("case", list(ADAPT_CASES))
@pytest.mark.parametrize("eps", [0.01, 0.0])
def test_amr_indicator_is_bitwise_the_oracles(hy, case, eps):
    """Refinement decisions: the indicator is computed with every operation
    rounded as written on both sides, so it agrees bit for bit, and so do
    the flags."""
    mesh, Ur, Uf, A = _adapt_mesh(hy, case)
    flags, E2 = A.estimate(eps=eps, refine_cutoff=0.5, derefine_cutoff=0.1)
    ref = amr.indicator(mesh, Ur, eps=eps)
    assert np.array_equal(E2, ref), np.abs(E2 - ref).max()
    assert flags.tolist() == amr.refine_flags(mesh, ref, 0.5, 0.1).tolist()
    A.close()


@pytest.mark.parametrize("case", list(ADAPT_CASES))
def test_amr_regrid_matches_the_oracle(hy, case):
    """Transfer to a new refinement: surviving children copied bit for bit,
    new ones prolonged (1e-12), refined root blocks restricted."""
    mesh, Ur, Uf, A = _adapt_mesh(hy, case)
    rng = np.random.default_rng(64)
    flags = mesh.refine.copy()
    flip = rng.choice(flags.size, size=max(2, flags.size // 3), replace=False)
    flags[flip] = ~flags[flip]
    B = A.regrid(flags)
    R, F = B.download()
    m1, R_ref, F_ref = amr.regrid(mesh, Ur, Uf, flags)
    assert B.nfine == m1.nfine
    for q, r in enumerate(m1.refined):
        if mesh.refine[r]:
            old = int(mesh.child_base[r])
            assert np.array_equal(F[8 * q:8 * q + 8], Uf[old:old + 8]), r
    assert_close((R, F), (R_ref, F_ref), f"{case} regrid")
    B.close()


def test_amr_adaptive_trajectory(hy):
    """Steps with regridding every two steps: estimate on both sides (the
    decisions agree wherever the indicator is not within 1e-9 of a cutoff),
    regrid both sides to the oracle's flags, parity after every step."""
    print("\n[amr] adaptive trajectory", flush=True)
    mesh, Ur, Uf, A = _adapt_mesh(hy, "smooth_n16")
    for cycle in range(3):
        for s in range(2):
            dt = amr.dt(mesh, Ur, Uf, 0.8)
            Ur, Uf, _ = amr.step(mesh, Ur, Uf, dt)
            A.step(dt)
            assert_close(A.download(), (Ur, Uf), f"cycle {cycle} step {s}")
        flags_gpu, E2_gpu = A.estimate(0.01, 0.93, 0.9)
        E2 = amr.indicator(mesh, Ur, 0.01)
        flags = amr.refine_flags(mesh, E2, 0.93, 0.9)
        clear = (np.abs(E2 - 0.93 * 0.93) > 1e-9) & (np.abs(E2 - 0.9 * 0.9) > 1e-9)
        assert np.array_equal(flags_gpu[clear], flags[clear])
        assert np.allclose(E2_gpu, E2, rtol=1e-10, atol=1e-14)
        if cycle == 0:  # this field refines five blocks and derefines one
            assert (flags & ~mesh.refine).sum() == 5 and (mesh.refine & ~flags).sum() == 1
        mesh, Ur, Uf = amr.regrid(mesh, Ur, Uf, flags)
        A = A.regrid(flags)
        assert_close(A.download(), (Ur, Uf), f"cycle {cycle} regrid")
    A.close()


# ---- more than two levels ------------------------------------------------------

def _tree_case(name):
    from oracle import amr_tree
    from tests.test_oracle_amr import _random_root
    from tests.test_oracle_amr_tree import _tree_state

    if name == "n8_three_levels":
        n, nb, bc = 8, (4, 4, 4), (0, 0, 0)
        f0 = np.array([b % 4 <= 2 and (b // 4) % 4 <= 2 and b // 16 <= 2 for b in range(64)])
        t1 = amr_tree.Tree(n, nb, (1 / 32,) * 3, [f0], bc=bc)
        base = int(t1.child_base[0][1 + 4 * (1 + 4 * 1)])
        f1 = np.zeros(t1.nblocks(1), bool)
        f1[[base + 0, base + 3, base + 5, base + 6]] = True
        flags = [f0, f1]
    elif name == "n8_three_levels_outflow":
        n, nb, bc = 8, (4, 4, 4), (1, 0, 1)
        f0 = np.array([b % 4 <= 2 and (b // 4) % 4 <= 2 and b // 16 <= 2 for b in range(64)])
        t1 = amr_tree.Tree(n, nb, (1 / 32,) * 3, [f0], bc=bc)
        f1 = np.zeros(t1.nblocks(1), bool)
        f1[int(t1.child_base[0][0]) + 7] = True           # next to the outflow corner
        f1[int(t1.child_base[0][1 + 4 * (1 + 4 * 1)]) + 2] = True
        flags = [f0, f1]
    elif name == "n16_three_levels":
        n, nb, bc = 16, (2, 2, 2), (0, 0, 0)
        f0 = np.ones(8, bool)
        f1 = np.zeros(64, bool)
        f1[[0, 21, 42]] = True
        flags = [f0, f1]
    elif name == "n32_two_levels":
        n, nb, bc = 32, (2, 1, 1), (0, 1, 0)
        flags = [[True, False]]
    else:  # four levels: everything refined twice, then one block again
        n, nb, bc = 8, (1, 1, 1), (0, 0, 0)
        flags = [[True], [True] * 8, [False] * 63 + [True]]
    t = amr_tree.Tree(n, nb, (1.0 / (nb[0] * n),) * 3, flags, bc=bc)
    Ur, _ = _random_root(nb, n, 81)
    return t, _tree_state(t, Ur, 82)


TREE_CASES = ["n8_three_levels", "n8_three_levels_outflow", "n16_three_levels", "n8_four_levels", "n32_two_levels"]


def _tree_gpu(hy, t, U):
    deep = np.concatenate([np.asarray(f, bool) for f in t.refine[1:]]) if t.levels > 1 else []
    hi = tuple(t.nb0[d] * t.n * t.dx0[d] for d in range(3))
    A = hy.Amr(t.n, t.nb0, t.refine[0].tolist(), hi=hi, bc=t.bc, gamma=t.gamma, refine_deep=list(deep))
    assert A.level_blocks == [t.nblocks(l) for l in range(t.levels)]
    A.upload(U[0], np.concatenate(U[1:]) if t.levels > 1 else None)
    return A


def _tree_split(A, R, F):
    out, o = [R], 0
    for nbk in A.level_blocks[1:]:
        out.append(F[o:o + nbk])
        o += nbk
    return out


@pytest.mark.parametrize("case", TREE_CASES)
@pytest.mark.parametrize("device_dt", [False, True])
def test_amr_tree_trajectory_parity(hy, case, device_dt):
    """Three steps on meshes of three and four levels (nesting by the
    26-neighbour rule), every level at 1e-12, dt to 1e-14, counters equal."""
    from oracle import amr_tree

    print(f"\n[amr] tree {case} device_dt={device_dt}", flush=True)
    t, U = _tree_case(case)
    A = _tree_gpu(hy, t, U)
    cnt = np.zeros(3, np.int64)
    for s in range(3):
        dt = amr_tree.dt(t, U, 0.8)
        if device_dt:
            A.step_cfl(0.8)
            assert abs(A.last_dt() / dt - 1.0) <= DT_TOL, (s, A.last_dt(), dt)
        else:
            assert abs(A.dt(0.8) / dt - 1.0) <= DT_TOL
            A.step(dt)
        U, c = amr_tree.step(t, U, dt)
        cnt += c
        got = _tree_split(A, *A.download())
        assert_close((got[0], np.concatenate(got[1:])), (U[0], np.concatenate(U[1:])), f"{case} step {s}")
    assert A.counters().tolist() == cnt.tolist()
    A.close()


# ---- adaptivity of meshes of any depth ---------------------------------------

def _flat(flags):
    return np.concatenate([np.asarray(f, bool) for f in flags])


@pytest.mark.parametrize("case", TREE_CASES)
def test_amr_tree_indicator_and_flags_are_the_oracles(hy, case):
    """Per-leaf indicator of every level bit for bit (rounded as written,
    same-level data only), and the rule's flags, nesting repair included."""
    from oracle import amr_tree

    t, U = _tree_case(case)
    A = _tree_gpu(hy, t, U)
    for rc, dc, ml in [(0.93, 0.9, 4), (0.7, 0.5, 3), (0.99, 0.95, 5)]:
        f0, deep, E2 = A.estimate_tree(0.01, rc, dc, ml)
        ref = amr_tree.indicator(t, U, 0.01)
        for l in range(t.levels):
            assert np.array_equal(E2[l], ref[l]), (case, l)
        flags = amr_tree.refine_flags(t, ref, rc, dc, max_levels=ml)
        assert np.array_equal(np.concatenate([f0, deep]), _flat(flags)), (case, rc, dc, ml)
    A.close()


@pytest.mark.parametrize("case", TREE_CASES)
def test_amr_tree_regrid_matches_the_oracle(hy, case):
    """Regrid to flags from a random indicator (nesting restored by the
    oracle's rule): blocks present before copied bit for bit, new ones
    prolonged (1e-12), restriction finest level first."""
    from oracle import amr_tree

    t, U = _tree_case(case)
    A = _tree_gpu(hy, t, U)
    rng = np.random.default_rng(101)
    E2 = [rng.random(t.nblocks(l)) for l in range(t.levels)]
    flags = amr_tree.refine_flags(t, E2, 0.9, 0.6, max_levels=4)
    new, V = amr_tree.regrid(t, U, flags)
    B = A.regrid(flags[0], _flat(flags[1:]) if len(flags) > 1 else [])
    assert B.level_blocks == [new.nblocks(l) for l in range(new.levels)]
    got = _tree_split(B, *B.download())
    for l in range(1, new.levels):
        for i, p in enumerate(new.pos[l].tolist()):
            old = t.block_at(l, *p) if l < t.levels else -1
            if old >= 0 and not new.refine[l][i]:
                assert np.array_equal(got[l][i], U[l][old]), (l, i)
    assert_close((got[0], np.concatenate(got[1:])), (V[0], np.concatenate(V[1:])), f"{case} tree regrid")
    B.close()


def test_amr_tree_adaptive_trajectory(hy):
    """Three levels at most: steps with an estimate and a regrid every two
    steps on both sides (flags compared where the indicator is clear of the
    cutoffs), parity after every step and regrid."""
    from oracle import amr_tree

    print("\n[amr] tree adaptive trajectory", flush=True)
    t, U = _tree_case("n16_three_levels")
    A = _tree_gpu(hy, t, U)
    changed = 0
    for cycle in range(3):
        for s in range(2):
            dt = amr_tree.dt(t, U, 0.8)
            U, _ = amr_tree.step(t, U, dt)
            A.step(dt)
            got = _tree_split(A, *A.download())
            assert_close((got[0], np.concatenate(got[1:])), (U[0], np.concatenate(U[1:])), f"cycle {cycle} step {s}")
        ref = amr_tree.indicator(t, U, 0.01)
        flags = amr_tree.refine_flags(t, ref, 0.95, 0.9, max_levels=3)
        f0, deep, E2 = A.estimate_tree(0.01, 0.95, 0.9, 3)
        clear = all(np.all((np.abs(r - 0.95 ** 2) > 1e-9) & (np.abs(r - 0.81) > 1e-9)) for r in ref)
        if clear:
            assert np.array_equal(np.concatenate([f0, deep]), _flat(flags))
        for l in range(t.levels):
            assert np.allclose(E2[l], ref[l], rtol=1e-8, atol=1e-10)
        before = [np.asarray(f, bool).copy() for f in t.refine]
        t, U = amr_tree.regrid(t, U, flags)
        changed += int(any(len(a) != len(b) or np.any(a != b) for a, b in zip(before, t.refine)) or
                       len(before) != len(t.refine))
        A = A.regrid(flags[0], _flat(flags[1:]) if len(flags) > 1 else [])
        got = _tree_split(A, *A.download())
        assert_close((got[0], np.concatenate(got[1:])), (U[0], np.concatenate(U[1:])), f"cycle {cycle} regrid")
    assert changed >= 1
    A.close()


# ---- tuning -----------------------------------------------------------------

def _run_columns(hy, build, cap, steps=3):
    A = build()
    A.set_columns(cap)
    for _ in range(steps):
        A.step_cfl(0.8)
    out = (A.download(), A.last_dt(), A.counters())
    A.close()
    return out


@pytest.mark.parametrize("case", ["n8_2x2x2_one", "n8_3x2x2_mixed_bc", "n16_2x2x1_periodic_z1", "n8_4x1x1_outflow",
                                  "n32_2x1x1", "n8_none_refined"])
def test_amr_column_length_is_bitwise_invariant(hy, case):
    """Leaf-step pencils over columns of one, two or four z-stacked leaves
    (and the length chosen per list) give the same bits: states, dt and
    counters after three steps with device dt."""
    ref = _run_columns(hy, lambda: make(hy, case)[3], 1)
    for cap in (2, 4, 0):
        (R, F), d, c = _run_columns(hy, lambda: make(hy, case)[3], cap)
        assert np.array_equal(R, ref[0][0]) and np.array_equal(F, ref[0][1]), (case, cap)
        assert d == ref[1] and np.array_equal(c, ref[2]), (case, cap)


@pytest.mark.parametrize("case", TREE_CASES)
def test_amr_tree_column_length_is_bitwise_invariant(hy, case):
    t, U = _tree_case(case)
    ref = _run_columns(hy, lambda: _tree_gpu(hy, t, U), 1)
    for cap in (2, 4):
        (R, F), d, c = _run_columns(hy, lambda: _tree_gpu(hy, t, U), cap)
        assert np.array_equal(R, ref[0][0]) and np.array_equal(F, ref[0][1]), (case, cap)
        assert d == ref[1] and np.array_equal(c, ref[2]), (case, cap)


@pytest.mark.parametrize("case", ["n8_2x2x2_one", "n16_2x2x1_periodic_z1", "tree:n8_three_levels"])
def test_amr_column_length_change_mid_run_is_bitwise(hy, case):
    """Changing the column length between steps rebuilds the column,
    halo-plane and launch tables: a block that ends a column only after the
    change gets its whole halo planes written again, so five steps with
    lengths 4, 4, 1, 2, 2 give the bits of five steps with length 1."""
    if case.startswith("tree:"):
        t, U = _tree_case(case[5:])
        build = lambda: _tree_gpu(hy, t, U)
    else:
        build = lambda: make(hy, case)[3]
    ref = _run_columns(hy, build, 1, steps=5)
    A = build()
    for cap in (4, 4, 1, 2, 2):
        A.set_columns(cap)
        A.step_cfl(0.8)
    (R, F), d, c = A.download(), A.last_dt(), A.counters()
    A.close()
    assert np.array_equal(R, ref[0][0]) and np.array_equal(F, ref[0][1]), case
    assert d == ref[1] and np.array_equal(c, ref[2]), case


def test_amr_column_argument_errors(hy):
    A = make(hy, "n8_2x2x2_one")[3]
    for bad in (-1, 3, 5, 8):
        with pytest.raises(hy.HydroError):
            A.set_columns(bad)
    A.close()
