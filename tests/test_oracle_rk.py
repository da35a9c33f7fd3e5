"""Pins of the oracle's SSP Runge-Kutta method-of-lines step (the paper's
other compressible solver, §2.2 Hydrodynamics: second- or third-order SSP
Runge-Kutta time integration).

Each test checks the oracle against something other than itself: exact
preservation of a uniform state, conservation, a special case that reduces
to the textbook scalar method-of-lines scheme, the exact Sod Riemann
solution, and the convergence order on smooth flow.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2208_11630_amd import ics
from tests.ref import exact_riemann as er
from tests.ref import mol1d
from tests.test_oracle_step import _exact_wave, _random_problem, _wave_problem, glob, grid_of


@pytest.mark.parametrize("order", [2, 3])
def test_uniform_state_preserved(order):
    """Fluxes of a uniform state cancel exactly; the Shu-Osher weights of
    order 2 are powers of two (bitwise), those of order 3 round (few ulp)."""
    P = ics.uniform(n=8, nb=(2, 2, 1), bc=(1, 0, 1))
    g = grid_of(P)
    U = P.U.copy()
    Un, cnt = oracle.step_rk(g, U, 1e-3, order)
    a, b = ics.interior(Un, P.n, P.ng), ics.interior(P.U, P.n, P.ng)
    if order == 2:
        assert np.array_equal(a, b)
    else:
        np.testing.assert_allclose(a, b, rtol=4 * np.finfo(float).eps, atol=0)
    assert cnt.tolist() == [0, 0, 0]


@pytest.mark.parametrize("order", [2, 3])
def test_conservation_on_periodic_random_state(order):
    P, _ = _random_problem((16, 8, 8), 8, (1 / 16,) * 3, (0, 0, 0))
    g = grid_of(P)
    U = P.U.copy()
    d = oracle.dt(g, U, 0.8)
    Un, cnt = oracle.step_rk(g, U, d, order)
    s0 = ics.interior(U, P.n, P.ng).sum(axis=(0, 2, 3, 4))
    s1 = ics.interior(Un, P.n, P.ng).sum(axis=(0, 2, 3, 4))
    tot = np.abs(ics.interior(U, P.n, P.ng)).sum(axis=(0, 2, 3, 4))
    assert np.all(np.abs(s1 - s0) <= 1e-13 * tot), (s1 - s0) / tot
    assert cnt.tolist() == [0, 0, 0]


@pytest.mark.parametrize("order", [2, 3])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_pure_contact_is_scalar_method_of_lines(axis, order):
    """Uniform velocity and pressure, rough density: the density follows the
    textbook scalar method-of-lines scheme (van Leer slopes, upwind flux,
    Shu-Osher SSP stages); velocity and pressure stay uniform."""
    L, n = 32, 8
    rng = np.random.default_rng(5)
    q = 1.0 + 0.5 * rng.random(L)
    q[10:14] += 1.0
    a, p0, gam = 0.7, 1.0, 1.4
    shape = [n, n, n]
    shape[axis] = L
    X, Y, Z = shape
    bshape = [1, 1, 1]
    bshape[2 - axis] = L
    rho = np.broadcast_to(q.reshape(bshape), (Z, Y, X)).copy()
    vel = [np.zeros((Z, Y, X)) for _ in range(3)]
    vel[axis][:] = a
    dx = [0.1, 0.1, 0.1]
    P = ics.from_primitive("contact", n, rho, *vel, np.full((Z, Y, X), p0), gam, dx, (0, 0, 0))
    g = grid_of(P)
    U = P.U
    dt = 0.02
    qs = q.copy()
    for _ in range(5):
        U, cnt = oracle.step_rk(g, U, dt, order)
        qs = mol1d.step(qs, a, dt / dx[axis], order)
    G = glob(P, U)
    sl = tuple(slice(None) if aa == 2 - axis else 0 for aa in range(3))
    np.testing.assert_allclose(G[0][sl], qs, rtol=1e-13, atol=0)
    np.testing.assert_allclose(G[1 + axis] / G[0], a, rtol=1e-13)
    pr = (gam - 1) * (G[4] - 0.5 * (G[1] ** 2 + G[2] ** 2 + G[3] ** 2) / G[0])
    np.testing.assert_allclose(pr, p0, rtol=1e-12)


def test_stage_is_forward_euler_of_the_operator():
    """A first stage alone (no base state) is U + dt L(U); with a base state
    U0 and weights (a0, a1) it is a0*U0 + a1*(U + dt L(U)): checked against
    a stage computed without the base and combined here."""
    P, _ = _random_problem((8, 8, 8), 8, (1 / 8,) * 3, (0, 1, 0), seed=21)
    g = grid_of(P)
    U = P.U.copy()
    oracle.fill_guards(g, U)
    d = 0.5 * oracle.dt(g, U, 0.8)
    plain, _ = oracle.stage_block(g, U, 0, d)
    rng = np.random.default_rng(3)
    U0 = U * (1.0 + 0.01 * rng.random(U.shape))
    comb, _ = oracle.stage_block(g, U, 0, d, U0, 0.75, 0.25)
    n, ng = P.n, P.ng
    core = (slice(None), slice(ng, ng + n), slice(ng, ng + n), slice(ng, ng + n))
    expect = 0.75 * U0[0][core] + 0.25 * plain[core]
    np.testing.assert_array_equal(comb[core], expect)


@pytest.mark.parametrize("order", [2, 3])
def test_sod_star_plateau(order):
    """Quasi-1-D Sod to t = 0.2 at 256 cells: the star plateau within 1% of
    the exact Riemann solution and a small L1 density error."""
    L = 256
    P = ics.sod(n=8, shape=(L, 8, 8))
    g = grid_of(P)
    U, t = P.U.copy(), 0.0
    while t < 0.2 - 1e-14:
        d = min(oracle.dt(g, U, 0.8), 0.2 - t)
        U, cnt = oracle.step_rk(g, U, d, order)
        assert cnt.tolist() == [0, 0, 0]
        t += d
    G = glob(P, U)
    rho = G[0, 0, 0]
    x = (np.arange(L) + 0.5) / L
    sel = (x > 0.5 + 0.9275 * t + 0.03) & (x < 0.5 + 1.7522 * t - 0.03)
    assert np.all(np.abs(rho[sel] / 0.265574 - 1) < 0.01)
    sel = (x > 0.5 - 0.0703 * t + 0.03) & (x < 0.5 + 0.9275 * t - 0.03)
    assert np.all(np.abs(rho[sel] / 0.426319 - 1) < 0.01)
    p = 0.4 * (G[4, 0, 0] - 0.5 * G[1, 0, 0] ** 2 / rho)
    sel = (x > 0.5 - 0.0703 * t + 0.03) & (x < 0.5 + 1.7522 * t - 0.03)
    assert np.all(np.abs(p[sel] / 0.303130 - 1) < 0.01)
    ex = er.cell_average(1, 0, 1, 0.125, 0, 0.1, 1.4, 0.5, t, np.arange(L + 1) / L)
    assert np.abs(rho - ex[0]).mean() < 6e-3


@pytest.mark.parametrize("order", [2, 3])
def test_smooth_convergence_order(order):
    """Entropy wave: L1 density error falls at order >= 1.7."""
    errs = []
    T = 0.25
    for L in (32, 64, 128):
        P, x = _wave_problem(L, "entropy", 0)
        g = grid_of(P)
        U, t = P.U.copy(), 0.0
        while t < T - 1e-14:
            d = min(oracle.dt(g, U, 0.8), T - t)
            U, cnt = oracle.step_rk(g, U, d, order)
            t += d
        G = glob(P, U)
        errs.append(np.abs(G[0][0, 0, :] - _exact_wave("entropy", x, t)[0]).mean())
    order_obs = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(order_obs) >= 1.7, (errs, order_obs)


def test_order_must_be_2_or_3():
    P = ics.uniform(n=8, nb=(1, 1, 1))
    with pytest.raises(ValueError):
        oracle.step_rk(grid_of(P), P.U.copy(), 1e-3, 4)
