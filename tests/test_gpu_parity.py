"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar: after every step, for every conserved variable q, the normwise relative
error max|q_gpu - q_ref| / max|q_ref| is at most 1e-12 (momenta: the
denominator is the maximum momentum magnitude); the dt each side chooses
agrees to 1e-14 relative; the guard fill is bitwise; event counters match.
Inputs are seeded synthetic states shared by both sides; expected values come
only from the oracle.
"""
import numpy as np
import pytest

import oracle
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

    hydro.lib()  # fails loudly if the library is missing
    return hydro


def ogrid(P):
    return oracle.Grid(P.n, P.nb, P.dx, P.bc, P.gamma, P.small_p, P.ng)


def rel_errors(A, B, n, ng=4):
    """Per-variable normwise relative error of interiors (A: tested, B: reference)."""
    a = ics.interior(A, n, ng)
    b = ics.interior(B, n, ng)
    errs = []
    rho_max = np.abs(b[:, 0]).max()
    mom = np.sqrt((b[:, 1] ** 2 + b[:, 2] ** 2) + b[:, 3] ** 2).max()
    for v in range(5):
        d = np.abs(a[:, v] - b[:, v]).max()
        den = mom if v in (1, 2, 3) else np.abs(b[:, v]).max()
        if den == 0.0:
            den = rho_max
        errs.append(d / den)
    return np.array(errs)


def assert_parity(A, B, n, what=""):
    e = rel_errors(A, B, n)
    assert np.all(e <= TOL), f"{what}: relative errors {e}"
    return e


def step_pair(hy, P, dt):
    """One step from P.U on both sides with the same dt."""
    ref, cnt = oracle.step(ogrid(P), P.U.copy(), dt)
    G = hy.grid_for(P)
    G.step(dt)
    out = G.download()
    return out, ref, cnt, G.counters()


# ---- a1: guard fill -----------------------------------------------------------

@pytest.mark.parametrize("n,nb", [(8, (3, 2, 2)), (16, (2, 1, 3)), (32, (1, 2, 1)), (8, (1, 1, 1))])
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1), (1, 0, 1)])
def test_fill_guards_bitwise(hy, n, nb, bc):
    X, Y, Z = nb[0] * n, nb[1] * n, nb[2] * n
    rng = np.random.default_rng(n + sum(nb))
    G0 = rng.normal(size=(5, Z, Y, X))
    P = ics.Problem("enc", n, nb, (1.0 / X,) * 3, bc, 1.4, ics.to_blocks(G0, n))
    ref = P.U.copy()
    oracle.fill_guards(ogrid(P), ref)
    Gd = hy.grid_for(P)
    out = Gd.fill_guards()
    Gd.stream.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref)
    # the state itself is untouched
    assert np.array_equal(Gd.download(), P.Uc)


# ---- one step from the same state ------------------------------------------------

def _random_problem(shape, n, dx, bc, seed):
    rng = np.random.default_rng(seed)
    X, Y, Z = shape
    G = ics.random_state(rng, (Z, Y, X))
    return ics.Problem("rand", n, (X // n, Y // n, Z // n), dx, bc, 1.4, ics.to_blocks(G, n))


CASES = {
    "sod64": lambda: ics.sod(),
    "sod_y": lambda: ics.sod(N=32, n=8, axis=1),
    "sedov64": lambda: ics.sedov(N=64, n=16),
    "sedov32_n8": lambda: ics.sedov(N=32, n=8),
    "kh_small": lambda: ics.kelvin_helmholtz(shape=(64, 64, 32), n=16),
    "rand_n32_mixed_bc": lambda: _random_problem((64, 32, 32), 32, (0.1, 0.12, 0.08), (1, 0, 1), 21),
    "rand_n8_ragged": lambda: _random_problem((24, 16, 40), 8, (0.05, 0.05, 0.05), (1, 0, 1), 22),
    "rand_n16_single_block": lambda: _random_problem((16, 16, 16), 16, (0.1, 0.1, 0.1), (0, 0, 0), 23),
    "rand_n8_single_block": lambda: _random_problem((8, 8, 8), 8, (0.1, 0.1, 0.1), (0, 0, 0), 24),
    "rand_n32_single_block_outflow": lambda: _random_problem((32, 32, 32), 32, (0.1, 0.1, 0.1), (1, 1, 1), 25),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_one_step_parity(hy, case):
    P = CASES[case]()
    dt = oracle.dt(ogrid(P), P.U, P.cfl)
    out, ref, cnt, gcnt = step_pair(hy, P, dt)
    assert_parity(out, ref, P.n, case)
    assert gcnt.tolist() == cnt.tolist()


def test_uniform_state_preserved_bitwise(hy):
    P = ics.uniform(n=16, nb=(2, 3, 1), bc=(1, 0, 1), dx=(0.1, 0.05, 0.2))
    dt = oracle.dt(ogrid(P), P.U, 0.8)
    out, ref, cnt, gcnt = step_pair(hy, P, dt)
    assert np.array_equal(ics.interior(out, 16), ics.interior(P.U, 16))


def _events_problem():
    """Random-state jump problem (pressure 1e-6 | 1 along x, outflow x) whose
    steps fall back to first order at the jump."""
    n, L = 8, 32
    Z, Y, X = 16, 8, L
    rng = np.random.default_rng(41)
    x = (np.arange(X) + 0.5) / X
    rho = np.exp(0.1 * rng.normal(size=(Z, Y, X)))
    u = 0.6 + 0.05 * rng.normal(size=(Z, Y, X))
    v = 0.1 * rng.normal(size=(Z, Y, X))
    w = np.zeros((Z, Y, X))
    p = np.broadcast_to(np.where(x < 0.5, 1e-6, 1.0)[None, None, :], (Z, Y, X)).copy()
    return ics.from_primitive("events", n, rho, u, v, w, p, 1.4, (1.0 / X,) * 3, (1, 0, 0))


def _plant_low_energy(Uc, rng, k=6):
    """Input construction: k random cells get a total energy of a tenth of
    their kinetic energy (a negative gamma-law pressure, so the floor must act;
    the energy their faces carry out then drives some of them to E <= 0)."""
    nblk, _, n = Uc.shape[:3]
    for _ in range(k):
        b = rng.integers(nblk)
        i, j, l = rng.integers(n, size=3)
        r, mx, my, mz = Uc[b, 0:4, l, j, i]
        Uc[b, 4, l, j, i] = 0.05 * (mx * mx + my * my + mz * mz) / r


def _decision_margins(Uc, gamma, small_p):
    """Distance of each event decision from its threshold, from the state in
    numpy: min |p - small_p| / |E| (the floor) and min |E| / max|E|, min rho
    (the nonphysical check), so that no decision sits within rounding."""
    r, mx, my, mz, E = (Uc[:, i] for i in range(5))
    p = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my + mz * mz) / r)
    return (float((np.abs(p - small_p) / np.abs(E)).min()), float(np.abs(E).min() / np.abs(E).max()),
            float(r.min()))


@pytest.mark.parametrize("plant", [False, True], ids=["jump", "jump_and_low_energy_cells"])
def test_event_counters_match_every_step(hy, plant):
    """Steps whose pressure floor and first-order fallback fire (a pressure
    jump) and, with planted low-energy cells, whose nonphysical check fires
    too: the state agrees to 1e-12 and the three event counters equal the
    oracle's running totals after every step (both sides restart each step
    from the oracle's state)."""
    P = _events_problem()
    g = ogrid(P)
    n = P.n
    Uc = P.Uc.copy()
    prng = np.random.default_rng(7)
    Gd = hy.grid_for(P)
    total = np.zeros(3, dtype=np.int64)
    for s in range(8):
        if plant:
            _plant_low_energy(Uc, prng)
        m_floor, m_energy, rho_min = _decision_margins(Uc, P.gamma, P.small_p)
        assert m_floor > 1e-9 and m_energy > 1e-6 and rho_min > 0.1, (s, m_floor, m_energy, rho_min)
        Gd.upload(Uc)
        U = ics.guard_layout(Uc, n)
        dt = oracle.dt(g, U, 0.8)
        U, c = oracle.step(g, U, dt)
        total += c
        Gd.step(dt)
        assert_parity(Gd.download(), U, n, f"events step {s}")
        assert Gd.counters().tolist() == total.tolist(), (s, Gd.counters(), total)
        Uc = np.ascontiguousarray(ics.interior(U, n))
    assert total[0] > 0 and total[1] > 0
    if plant:
        assert total[2] > 0


# ---- trajectories: each side picks its own dt -------------------------------------

@pytest.mark.parametrize("case,steps", [("sod64", 20), ("sedov64", 20), ("kh_small", 10),
                                        ("rand_n32_mixed_bc", 5)])
@pytest.mark.parametrize("device_dt", [False, True])
def test_trajectory_parity(hy, case, steps, device_dt):
    P = CASES[case]()
    g = ogrid(P)
    U = P.U.copy()
    Gd = hy.grid_for(P)
    for s in range(steps):
        dref = oracle.dt(g, U, P.cfl)
        if device_dt:
            Gd.step_cfl(P.cfl)
            dg = Gd.last_dt()
        else:
            dg = Gd.dt(P.cfl)
            Gd.step(dg)
        assert abs(dg / dref - 1.0) <= DT_TOL, (s, dg, dref)
        U, _ = oracle.step(g, U, dref)
        assert_parity(Gd.download(), U, P.n, f"{case} step {s}")
    assert Gd.counters().tolist() == [0, 0, 0]
    assert abs(Gd.dt(P.cfl) / oracle.dt(g, U, P.cfl) - 1.0) <= DT_TOL


# ---- properties that hold at any size ---------------------------------------------

def test_translation_by_whole_blocks_bitwise(hy):
    n = 16
    P = _random_problem((48, 32, 32), n, (0.1, 0.1, 0.1), (0, 0, 0), 31)
    Gd = hy.grid_for(P)
    dt = 0.5 * Gd.dt(0.8)
    Gd.step(dt)
    R = ics.from_blocks(Gd.download(), n, P.nb)
    G0 = ics.from_blocks(P.U, n, P.nb)
    Gs = np.roll(G0, shift=(n, 2 * n, n), axis=(3, 2, 1))
    P2 = ics.Problem("s", n, P.nb, P.dx, P.bc, 1.4, ics.to_blocks(Gs, n))
    G2 = hy.grid_for(P2)
    G2.step(dt)
    R2 = ics.from_blocks(G2.download(), n, P2.nb)
    assert np.array_equal(R2, np.roll(R, shift=(n, 2 * n, n), axis=(3, 2, 1)))


def test_conservation_on_device(hy):
    n = 32
    P = _random_problem((64, 64, 32), n, (0.1, 0.1, 0.1), (0, 0, 0), 32)
    Gd = hy.grid_for(P)
    before = ics.from_blocks(P.U, n, P.nb).reshape(5, -1)
    for _ in range(3):
        Gd.step_cfl(0.8)
    after = ics.from_blocks(Gd.download(), n, P.nb).reshape(5, -1)
    for v in range(5):
        assert abs(after[v].sum() - before[v].sum()) <= 1e-13 * np.abs(before[v]).sum()


# ---- full-size configurations: sampled blocks --------------------------------------

def _sampled_parity(hy, P, blocks):
    g = ogrid(P)
    dt = oracle.dt(g, P.U, P.cfl)
    Gd = hy.grid_for(P)
    dg = Gd.dt(P.cfl)
    assert abs(dg / dt - 1.0) <= DT_TOL
    Gd.step(dt)
    st = Gd.state
    got = st[blocks].cpu().numpy()
    ref, cnt = oracle.step_blocks(g, P.U, blocks, dt)
    assert_parity(got, ref, P.n, P.name)
    assert Gd.counters().tolist() == [0, 0, 0] and cnt.tolist() == [0, 0, 0]


def test_kh_full_size_sampled_blocks(hy):
    P = ics.kelvin_helmholtz()
    nbx, nby, nbz = P.nb
    pick = [0, nbx - 1, nbx * (nby - 1), P.nblk - 1, nbx * nby * (nbz // 2) + nbx * (nby // 4) + 5,
            nbx * nby * 3 + nbx * (3 * nby // 4) + 17, 12345 % P.nblk, 9876 % P.nblk]
    _sampled_parity(hy, P, sorted(set(pick)))


def test_sedov_full_size_sampled_blocks(hy):
    P = ics.sedov()
    nb = P.nb[0]
    c = nb // 2
    pick = [(c - 1) + nb * ((c - 1) + nb * (c - 1)), c + nb * (c + nb * c), (c - 1) + nb * (c + nb * c),
            0, P.nblk - 1, 1234]
    _sampled_parity(hy, P, sorted(set(pick)))


# ---- full configurations run to their step counts ------------------------------------

def _rel_errors_device(got, ref):
    """rel_errors on device tensors [nblk, 5, n, n, n] (whole grids)."""
    import torch

    rho_max = ref[:, 0].abs().max()
    mom = torch.sqrt((ref[:, 1] ** 2 + ref[:, 2] ** 2) + ref[:, 3] ** 2).max()
    errs = []
    for v in range(5):
        d = (got[:, v] - ref[:, v]).abs().max()
        den = mom if v in (1, 2, 3) else ref[:, v].abs().max()
        if float(den) == 0.0:
            den = rho_max
        errs.append(float(d / den))
    return np.array(errs)


def _full_trajectory(hy, P, steps, planes_list, compare_every=1):
    """Each side runs the configuration for its step count with its own dt
    (device dt on the GPU), on one GPU grid per z-pencil length in
    planes_list (None: the autotuner's choice).  Every block, all five
    variables, agrees to 1e-12 after every compare_every-th step and the
    last one; every step's dt agrees to 1e-14; counters stay zero."""
    import torch

    from paper_2208_11630_amd import tune

    g = ogrid(P)
    grids = []
    for planes in planes_list:
        Gd = hy.grid_for(P)
        if planes is None:
            planes = tune.tune_grid(Gd, P.cfl, use_cache=False)
        else:
            Gd.set_pencil_planes(planes)
        print(f"[parity] {P.name}: GPU grid with {planes}-plane z pencils", flush=True)
        grids.append((planes, Gd))
    U = P.U.copy()
    for s in range(steps):
        for _, Gd in grids:
            Gd.step_cfl(P.cfl)
        d = oracle.dt(g, U, P.cfl)
        U, cnt = oracle.step(g, U, d)
        assert cnt.tolist() == [0, 0, 0]
        for planes, Gd in grids:
            assert abs(Gd.last_dt() / d - 1.0) <= DT_TOL, (planes, s, Gd.last_dt(), d)
        if (s + 1) % compare_every == 0 or s + 1 == steps:
            ref = torch.from_numpy(np.ascontiguousarray(ics.interior(U, P.n))).to(grids[0][1].state.device)
            for planes, Gd in grids:
                Gd.stream.synchronize()
                e = _rel_errors_device(Gd.state, ref)
                assert np.all(e <= TOL), f"{P.name} step {s + 1}, {planes}-plane pencils: relative errors {e}"
            del ref
    for planes, Gd in grids:
        assert Gd.counters().tolist() == [0, 0, 0], planes
        Gd.close()


def test_kh_full_configuration_ten_steps(hy):
    """KH 512x512x256 for its 10 steps, every block after every step: at the
    one-block pencils, at the 64-plane pencils the benchmark times and at
    the autotuner's choice."""
    print("\n[parity] KH 512x512x256, 10 steps", flush=True)
    P = ics.kelvin_helmholtz()
    _full_trajectory(hy, P, 10, [P.n, 64, None])


def test_sedov_full_configuration_hundred_steps(hy):
    """Sedov 256^3 for its 100 steps, every block every 10 steps, at the
    one-block pencils and at the autotuner's choice."""
    print("\n[parity] Sedov 256^3, 100 steps", flush=True)
    P = ics.sedov()
    _full_trajectory(hy, P, 100, [P.n, None], compare_every=10)


@pytest.mark.parametrize("n", [1, 511, 2049, 20481, 3 * 20480 + 7777, 1 << 22])
def test_copy_probe_copies_every_element(n):
    """The bandwidth probe copies exactly n doubles (chunk tails, odd n)."""
    import torch

    from paper_2208_11630_amd import hydro

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    src = torch.arange(n + 64, dtype=torch.float64, device="cuda:0")
    dst = torch.full_like(src, -1.0)
    s = torch.cuda.current_stream()
    hydro.copy_probe(src[:n], dst[:n], s)
    s.synchronize()
    assert torch.equal(dst[:n], src[:n])
    assert bool((dst[n:] == -1.0).all())
