"""Batched mode: many grids in one persistent launch per step.

Each member's state after k batch steps must be bitwise the state it reaches
alone through the plain grid API (same kernels, same per-grid device dt),
whatever the tuning (pencils, workgroups, graph replay) and whichever other
members are active; and it must match the CPU oracle to the 1e-12 bar.
"""
import numpy as np
import pytest

import oracle
from paper_2208_11630_amd import ics

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hy():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2208_11630_amd import hydro

    hydro.lib()
    return hydro


def members(count=14, seed=7):
    # small mixed ensemble: every block size, 1..6 blocks each
    rng = np.random.default_rng(seed)
    shapes = [(int(rng.integers(1, 7)), [8, 16, 32][i % 3]) for i in range(count)]
    return ics.ensemble(count=count, seed=seed, steps=4, shapes=shapes)


def alone(hy, P, k, cfl=0.8, nseg=1):
    G = hy.grid_for(P)
    G.set_pencils(nseg)
    for _ in range(k):
        G.step_cfl(cfl)
    return G.download(), G.last_dt()


def batched(hy, sims, k, cfl=0.8, pencils=None, per_cu=None, graph=False, chunks=None, tiles=None):
    grids = [hy.grid_for(P) for P in sims]
    B = hy.Batch(grids)
    if pencils:
        B.set_pencils(*pencils)
    if per_cu:
        B.set_workgroups(per_cu)
    if tiles:
        B.set_tiles(*tiles)
    B.use_graph(graph)
    for c in (chunks or [k]):
        B.step(cfl, c)
        B.stream.synchronize()
    out = [G.download() for G in grids]
    dts = B.dts()
    B.close()
    return out, dts


def test_batch_bitwise_equals_alone(hy):
    sims = members()
    k = 4
    ref = [alone(hy, P, k) for P in sims]
    out, dts = batched(hy, sims, k)
    for i, (U, d) in enumerate(ref):
        assert np.array_equal(out[i], U), f"member {i} (n={sims[i].n}, nblk={sims[i].nblk})"
        assert dts[i] == d


@pytest.mark.parametrize("n", [8, 16, 32])
def test_single_size_batch_bitwise_equals_alone(hy, n):
    """Batches whose members share one block size run the kernel that holds
    only that size's tile step: bitwise the members' steps alone, also with
    a graph, and when a mask leaves one size active in a mixed batch."""
    rng = np.random.default_rng(12 + n)
    shapes = [(int(rng.integers(1, 7)), n) for _ in range(5)]
    sims = ics.ensemble(count=5, seed=12 + n, steps=4, shapes=shapes)
    ref = [alone(hy, P, 7) for P in sims]
    out, dts = batched(hy, sims, 7, graph=True, chunks=[6, 1])
    for i, (U, d) in enumerate(ref):
        assert np.array_equal(out[i], U), i
        assert dts[i] == d
    mixed = members(count=9, seed=20)
    grids = [hy.grid_for(P) for P in mixed]
    B = hy.Batch(grids)
    mask = [P.n == n for P in mixed]
    B.set_active(mask)
    B.step(0.8, 2)
    B.stream.synchronize()
    for i, P in enumerate(mixed):
        U = alone(hy, P, 2)[0] if mask[i] else hy.grid_for(P).download()
        assert np.array_equal(grids[i].download(), U), (n, i)
    B.close()


@pytest.mark.parametrize("pencils,per_cu,tiles", [((2, 2, 4), 2, None), ((4, 4, 2), 1, (8, 8, 8)),
                                                  ((1, 4, 4), 3, (8, 16, 8)), ((1, 1, 1), 2, (8, 8, 16))])
def test_batch_tuning_is_bitwise_invariant(hy, pencils, per_cu, tiles):
    sims = members(count=9, seed=8)
    base, _ = batched(hy, sims, 3)
    out, _ = batched(hy, sims, 3, pencils=pencils, per_cu=per_cu, tiles=tiles)
    for a, b in zip(base, out):
        assert np.array_equal(a, b)


def test_batch_graph_replays_match_direct_launches(hy):
    sims = members(count=10, seed=9)
    base, d0 = batched(hy, sims, 15)
    # graph of 6 steps replayed twice (with host syncs between replays), then 3 direct steps
    out, d1 = batched(hy, sims, 15, graph=True, chunks=[6, 6, 3])
    for a, b in zip(base, out):
        assert np.array_equal(a, b)
    assert np.array_equal(d0, d1)


@pytest.mark.parametrize("nseg", [2, 4])
def test_grid_pencils_bitwise_invariant(hy, nseg):
    P = ics.kelvin_helmholtz(shape=(64, 64, 64), n=16)
    a, da = alone(hy, P, 3)
    b, db = alone(hy, P, 3, nseg=nseg)
    assert np.array_equal(a, b) and da == db


@pytest.mark.parametrize("planes", [2, 8, 32, 64, 128])
@pytest.mark.parametrize("case", ["kh", "outflow_n8"])
def test_grid_pencil_planes_bitwise_invariant(hy, planes, case):
    """Pencils spanning several blocks along z (or part of one) give the same
    bits as one pencil per block, with periodic and outflow z boundaries."""
    if case == "kh":
        P = ics.kelvin_helmholtz(shape=(32, 32, 128), n=16)
    else:
        P = ics.sod(N=16, n=8, axis=2, shape=(16, 8, 128))
    nz = P.nb[2] * P.n
    if nz % planes:
        pytest.skip("planes must divide the z extent")
    a, da = alone(hy, P, 3)
    G = hy.grid_for(P)
    G.set_pencil_planes(planes)
    for _ in range(3):
        G.step_cfl(0.8)
    assert np.array_equal(G.download(), a) and G.last_dt() == da


@pytest.mark.parametrize("n,shape,planes", [(16, (64, 64, 64), 16), (16, (32, 48, 64), 32), (32, (64, 32, 64), 64),
                                             (32, (32, 32, 96), 16)])
def test_grid_tile_bitwise_invariant(hy, n, shape, planes):
    """8x8 column tiles give the same bits as 16x16 ones, for the
    predictor-corrector step and an SSP-RK2 step, at several pencil
    lengths."""
    P = ics.kelvin_helmholtz(shape=shape, n=n)
    a, da = alone(hy, P, 3)
    G = hy.grid_for(P)
    G.set_tile(8)
    G.set_pencil_planes(planes)
    for _ in range(3):
        G.step_cfl(0.8)
    assert np.array_equal(G.download(), a) and G.last_dt() == da
    R16 = hy.grid_for(P)
    R16.set_scheme(hy.SCHEME_RK2)
    R8 = hy.grid_for(P)
    R8.set_scheme(hy.SCHEME_RK2)
    R8.set_tile(8)
    for _ in range(2):
        R16.step_cfl(0.8)
        R8.step_cfl(0.8)
    assert np.array_equal(R16.download(), R8.download())


def test_tile_argument_errors(hy):
    G = hy.grid_for(ics.kelvin_helmholtz(shape=(32, 32, 32), n=8))
    for bad in (0, 4, 12, 16, 32):
        with pytest.raises(hy.HydroError):
            G.set_tile(bad)
    G.set_tile(8)
    H = hy.grid_for(ics.kelvin_helmholtz(shape=(32, 32, 32), n=16))
    B = hy.Batch([H])
    with pytest.raises(hy.HydroError):
        H.set_tile(8)                        # a member of a batch
    with pytest.raises(hy.HydroError):
        B.set_tiles(16, 16, 16)              # 8^3 blocks take 8x8 tiles
    with pytest.raises(hy.HydroError):
        B.set_tiles(8, 4, 16)
    B.close()


def test_pencil_planes_argument_errors(hy):
    P = ics.kelvin_helmholtz(shape=(32, 32, 48), n=16)
    G = hy.grid_for(P)
    for bad in (0, 1, 5, 96):
        with pytest.raises(hy.HydroError):
            G.set_pencil_planes(bad)
    G.set_pencil_planes(48)


def test_batch_active_mask(hy):
    sims = members(count=8, seed=10)
    grids = [hy.grid_for(P) for P in sims]
    B = hy.Batch(grids)
    mask = [i % 2 == 0 for i in range(len(sims))]
    B.set_active(mask)
    B.step(0.8, 3)
    B.set_active([True] * len(sims))
    B.step(0.8, 1)
    B.stream.synchronize()
    for i, P in enumerate(sims):
        U, _ = alone(hy, P, 4 if mask[i] else 1)
        assert np.array_equal(grids[i].download(), U), i
    B.close()


def test_batch_members_match_oracle(hy):
    sims = members(count=6, seed=11)
    k = 3
    out, dts = batched(hy, sims, k)
    for i, P in enumerate(sims):
        g = oracle.Grid(P.n, P.nb, P.dx, P.bc, P.gamma, P.small_p)
        U = P.U.copy()
        for _ in range(k):
            d = oracle.dt(g, U, 0.8)
            U, _ = oracle.step(g, U, d)
        assert abs(dts[i] / d - 1) <= 1e-14
        a = out[i]
        b = ics.interior(U, P.n)
        for v in range(5):
            den = np.abs(b[:, v]).max() if v in (0, 4) else np.sqrt((b[:, 1:4] ** 2).sum(axis=1)).max()
            assert np.abs(a[:, v] - b[:, v]).max() <= 1e-12 * den, (i, v)


def test_full_ensemble_sampled_members_match_oracle(hy):
    """The benchmarked ensemble (512 members, 1-64 blocks of 8^3/16^3/32^3,
    seed 2) run for its 50 steps as one persistent launch per step (HIP
    graph), each member with its own device dt; sampled members - the
    largest, the smallest, and members of every block size - follow their
    own oracle trajectory to 1e-12, and their last step's dt to 1e-14."""
    print("\n[batch] full ensemble", flush=True)
    sims = ics.ensemble(count=512, seed=2, steps=50)
    grids = [hy.grid_for(P) for P in sims]
    B = hy.Batch(grids)
    B.use_graph(True)
    B.step(0.8, 48)
    B.use_graph(False)
    B.step(0.8, 2)
    B.stream.synchronize()
    dts = B.dts()
    cells = np.array([P.cells for P in sims])
    pick = {int(np.argmax(cells)), int(np.argmin(cells))}
    for n in (8, 16, 32):
        idx = [i for i, P in enumerate(sims) if P.n == n]
        pick.update(idx[:1] + idx[len(idx) // 2:len(idx) // 2 + 1])
    for i in sorted(pick):
        P = sims[i]
        print(f"[batch] member {i}: {P.nb} blocks of {P.n}^3", flush=True)
        g = oracle.Grid(P.n, P.nb, P.dx, P.bc, P.gamma, P.small_p)
        U = P.U.copy()
        for _ in range(50):
            d = oracle.dt(g, U, 0.8)
            U, _ = oracle.step(g, U, d)
        a = grids[i].download()
        b = ics.interior(U, P.n)
        for v in range(5):
            den = np.abs(b[:, v]).max() if v in (0, 4) else np.sqrt((b[:, 1:4] ** 2).sum(axis=1)).max()
            assert np.abs(a[:, v] - b[:, v]).max() <= 1e-12 * den, (i, v)
        assert abs(dts[i] / d - 1) <= 1e-14, i          # the dt of the last step
    B.close()
