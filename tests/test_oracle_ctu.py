"""Pins of the oracle's corner-transport-upwind (CTU) step: the unsplit
predictor-corrector solver of §2.2 in its corner-coupled form.

Each test checks the oracle against something other than itself: exact
preservation of a uniform state, conservation, a three-dimensional pure
contact that reduces to the textbook scalar CTU scheme (every transverse and
corner term enters it), agreement with the predictor-corrector step on
one-dimensional data (where every transverse term vanishes), convergence
order on a diagonal smooth wave, and stability at per-direction Courant
number 0.8.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2208_11630_amd import ics
from tests.ref import ctu3d
from tests.test_oracle_step import _random_problem, glob, grid_of


def test_uniform_state_preserved_bitwise():
    P = ics.uniform(n=8, nb=(2, 1, 2), bc=(1, 0, 1))
    g = grid_of(P)
    U = P.U.copy()
    Un, cnt = oracle.step_ctu(g, U, oracle.dt_ctu(g, U, 0.8))
    assert np.array_equal(ics.interior(Un, P.n), ics.interior(P.U, P.n))
    assert cnt.tolist() == [0, 0, 0]


def test_dt_per_direction_closed_form():
    """Uniform state: dt = cfl / max_d (|u_d| + c)/dx_d."""
    P = ics.uniform(n=8, nb=(1, 1, 1), rho=1.3, vel=(0.3, -0.2, 0.1), p=0.7, dx=(0.1, 0.05, 0.2))
    g = grid_of(P)
    c = math.sqrt(1.4 * 0.7 / 1.3)
    expect = 0.8 / max((0.3 + c) / 0.1, (0.2 + c) / 0.05, (0.1 + c) / 0.2)
    assert oracle.dt_ctu(g, P.U, 0.8) == pytest.approx(expect, rel=1e-15)


def test_conservation_on_periodic_random_state():
    P, _ = _random_problem((16, 8, 8), 8, (1 / 16,) * 3, (0, 0, 0), seed=31)
    g = grid_of(P)
    U = P.U.copy()
    Un, cnt = oracle.step_ctu(g, U, oracle.dt_ctu(g, U, 0.8))
    a, b = ics.interior(U, P.n), ics.interior(Un, P.n)
    tot = np.abs(a).sum(axis=(0, 2, 3, 4))
    assert np.all(np.abs(b.sum(axis=(0, 2, 3, 4)) - a.sum(axis=(0, 2, 3, 4))) <= 1e-13 * tot)
    assert cnt[2] == 0


@pytest.mark.parametrize("dx", [(0.1, 0.1, 0.1), (0.1, 0.08, 0.125)])
def test_diagonal_contact_is_scalar_ctu(dx):
    """Uniform velocity (0.7, 0.5, 0.3) and pressure, rough density in 3-D,
    cubic and anisotropic cells: the density follows the scalar
    three-dimensional CTU scheme; velocity and pressure stay uniform."""
    n, L = 8, 16
    rng = np.random.default_rng(8)
    rho = 1.0 + 0.5 * rng.random((L, L, L))
    rho[4:9, 3:7, 6:12] += 1.0
    vel = (0.7, 0.5, 0.3)
    one = np.ones((L, L, L))
    P = ics.from_primitive("contact3d", n, rho, vel[0] * one, vel[1] * one, vel[2] * one, one, 1.4, dx, (0, 0, 0))
    g = grid_of(P)
    U = P.U
    dt = 0.08           # per-direction Courant numbers up to 0.625
    q = rho.copy()
    lam = tuple(dt / h for h in dx)
    for _ in range(4):
        U, cnt = oracle.step_ctu(g, U, dt)
        q = ctu3d.step(q, vel, lam)
        assert cnt.tolist() == [0, 0, 0]
    G = glob(P, U)
    np.testing.assert_allclose(G[0], q, rtol=1e-13, atol=0)
    for d in range(3):
        np.testing.assert_allclose(G[1 + d] / G[0], vel[d], rtol=1e-13)
    pr = 0.4 * (G[4] - 0.5 * (G[1] ** 2 + G[2] ** 2 + G[3] ** 2) / G[0])
    np.testing.assert_allclose(pr, 1.0, rtol=1e-12)


@pytest.mark.parametrize("axis", [0, 2])
def test_one_dimensional_data_matches_predictor_corrector(axis):
    """With variation along one axis only, every transverse slope and flux
    difference vanishes and CTU reduces to the predictor-corrector step."""
    P = ics.sod(N=32, n=8, axis=axis)
    g = grid_of(P)
    dt = 0.5 * oracle.dt(g, P.U, 0.8)
    a, _ = oracle.step_ctu(g, P.U.copy(), dt)
    b, _ = oracle.step(g, P.U.copy(), dt)
    A, B = ics.interior(a, P.n), ics.interior(b, P.n)
    for v in (0, 4, 1 + axis):
        assert np.abs(A[:, v] - B[:, v]).max() <= 1e-14 * np.abs(B[:, v]).max()


def _diagonal_wave(L):
    n = 8
    h = 1.0 / L
    x = (np.arange(L) + 0.5) * h
    X = np.broadcast_to(x[None, None, :], (n, L, L))
    Y = np.broadcast_to(x[None, :, None], (n, L, L))
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * (X + Y))
    one = np.ones((n, L, L))
    P = ics.from_primitive("diag", n, rho, one, one, 0 * one, one, 1.4, (h, h, h), (0, 0, 0))
    return P, X, Y


def test_diagonal_wave_converges_at_second_order():
    errs = []
    T = 0.25
    for L in (16, 32, 64):
        P, X, Y = _diagonal_wave(L)
        g = grid_of(P)
        U, t = P.U.copy(), 0.0
        while t < T - 1e-14:
            d = min(oracle.dt_ctu(g, U, 0.8), T - t)
            U, cnt = oracle.step_ctu(g, U, d)
            t += d
        G = glob(P, U)
        exact = 1.0 + 0.2 * np.sin(2 * np.pi * (X - t + Y - t))
        errs.append(np.abs(G[0] - exact).mean())
    order = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(order) >= 1.7, (errs, order)


def test_stable_at_per_direction_courant_0_8():
    """A random periodic state stays physical for 25 steps at dt from the
    per-direction rule with CFL 0.8, and its total variation of density does
    not grow."""
    P, _ = _random_problem((16, 16, 16), 8, (1 / 16,) * 3, (0, 0, 0), seed=32)
    g = grid_of(P)
    U, dts, cnt = oracle.run(g, P.U.copy(), 25, 0.8, ctu=True)
    assert cnt[2] == 0
    G0, G1 = glob(P, P.U), glob(P, U)
    tv = lambda r: sum(np.abs(np.diff(r, axis=a)).sum() for a in range(3))
    assert tv(G1[0]) < tv(G0[0])


# ---- characteristic tracing of the normal predictor ------------------------

def _random_cell(rng, d):
    """A subsonic or supersonic cell whose wave speeds are clear of zero."""
    while True:
        rho = float(np.exp(rng.normal(0, 0.5)))
        p = float(np.exp(rng.normal(0, 0.5)))
        W = np.array([rho, *rng.normal(0, 1.0, 3), p])
        c = math.sqrt(1.4 * p / rho)
        un = W[1 + d]
        if min(abs(un - c), abs(un), abs(un + c)) > 1e-2:
            return W, c


@pytest.mark.parametrize("d", [0, 1, 2])
def test_trace_faces_match_numpy_eigen_decomposition(d):
    """The traced face states equal the projection computed with numpy's
    eigensolver on the primitive Jacobian (the degenerate entropy/shear
    eigenspace enters through its projector, whatever basis numpy picks)."""
    from tests.ref import char1d

    rng = np.random.default_rng(40 + d)
    for _ in range(200):
        W, c = _random_cell(rng, d)
        S = rng.normal(0, 0.3, 5) * np.abs(W)
        lam = float(rng.uniform(0.05, 0.8)) / (abs(W[1 + d]) + c)
        lo, hi = oracle.trace_faces(W, S, d, lam, 1.4)
        elo, ehi = char1d.traced_faces(W, S, lam, 1.4, d)
        scale = np.abs(W) + np.abs(S)
        assert np.all(np.abs(lo - elo) <= 1e-12 * scale), (W, S, lo, elo)
        assert np.all(np.abs(hi - ehi) <= 1e-12 * scale), (W, S, hi, ehi)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_trace_faces_supersonic_keeps_only_the_upwind_face(d):
    """All waves moving one way: the face they move away from keeps the
    cell-centred state exactly, the other face equals the primitive-form
    half-step face state W - lam/2 A S + S/2 (every wave reaches it)."""
    from tests.ref import char1d

    rng = np.random.default_rng(50 + d)
    for sign in (1.0, -1.0):
        W = np.array([1.3, 0.2, -0.1, 0.3, 0.7])
        c = math.sqrt(1.4 * 0.7 / 1.3)
        W[1 + d] = sign * (c + 0.5)
        S = rng.normal(0, 0.1, 5)
        lam = 0.3 / (abs(W[1 + d]) + c)
        lo, hi = oracle.trace_faces(W, S, d, lam, 1.4)
        half = W - 0.5 * lam * (char1d.jacobian(W, 1.4, d) @ S)
        if sign > 0:
            assert np.array_equal(lo, W)
            np.testing.assert_allclose(hi, half + 0.5 * S, rtol=1e-14, atol=1e-15)
        else:
            assert np.array_equal(hi, W)
            np.testing.assert_allclose(lo, half - 0.5 * S, rtol=1e-14, atol=1e-15)


def test_trace_faces_single_acoustic_wave():
    """A slope along the right-moving acoustic eigenvector of a subsonic
    cell: the low face gets nothing (that wave moves away from it), the high
    face W + (1 - lam (u + c))/2 S: what sets tracing apart from the
    primitive-form half step, whose low face would be W - (1 + lam(u+c))/2 S."""
    rho, u, p = 1.2, 0.3, 0.9
    c = math.sqrt(1.4 * p / rho)
    W = np.array([rho, u, 0.1, -0.2, p])
    eps = 1e-3
    S = eps * np.array([1.0, c / rho, 0.0, 0.0, c * c])
    lam = 0.5 / (u + c)
    lo, hi = oracle.trace_faces(W, S, 0, lam, 1.4)
    np.testing.assert_allclose(lo, W, rtol=0, atol=1e-15)
    np.testing.assert_allclose(hi, W + 0.5 * (1.0 - lam * (u + c)) * S, rtol=1e-14, atol=1e-16)


def test_traced_ctu_uniform_state_and_conservation():
    P = ics.uniform(n=8, nb=(2, 1, 2), bc=(1, 0, 1))
    g = grid_of(P)
    Un, cnt = oracle.step_ctu(g, P.U.copy(), oracle.dt_ctu(g, P.U, 0.8), trace=True)
    assert np.array_equal(ics.interior(Un, P.n), ics.interior(P.U, P.n))
    P, _ = _random_problem((16, 8, 8), 8, (1 / 16,) * 3, (0, 0, 0), seed=33)
    g = grid_of(P)
    U = P.U.copy()
    Un, cnt = oracle.step_ctu(g, U, oracle.dt_ctu(g, U, 0.8), trace=True)
    a, b = ics.interior(U, P.n), ics.interior(Un, P.n)
    tot = np.abs(a).sum(axis=(0, 2, 3, 4))
    assert np.all(np.abs(b.sum(axis=(0, 2, 3, 4)) - a.sum(axis=(0, 2, 3, 4))) <= 1e-13 * tot)
    assert cnt[2] == 0


def test_traced_diagonal_contact_is_scalar_ctu():
    """A pure contact carries one wave per direction (the entropy wave), so
    tracing leaves the scalar three-dimensional CTU scheme in the density."""
    n, L = 8, 16
    dx = (0.1, 0.08, 0.125)
    rng = np.random.default_rng(9)
    rho = 1.0 + 0.5 * rng.random((L, L, L))
    vel = (0.7, 0.5, 0.3)
    one = np.ones((L, L, L))
    P = ics.from_primitive("contact3d", n, rho, vel[0] * one, vel[1] * one, vel[2] * one, one, 1.4, dx, (0, 0, 0))
    g = grid_of(P)
    U, q = P.U, rho.copy()
    lam = tuple(0.08 / h for h in dx)
    for _ in range(3):
        U, cnt = oracle.step_ctu(g, U, 0.08, trace=True)
        q = ctu3d.step(q, vel, lam)
        assert cnt.tolist() == [0, 0, 0]
    np.testing.assert_allclose(glob(P, U)[0], q, rtol=1e-13, atol=0)


@pytest.mark.parametrize("axis,bc", [(0, (1, 0, 0)), (2, (0, 0, 1))])
def test_traced_ctu_on_one_dimensional_data_is_the_1d_traced_scheme(axis, bc):
    """Variation along one axis: every transverse term vanishes and the
    traced CTU step is the one-dimensional traced MUSCL-Hancock step of
    tests/ref/char1d (numpy eigen-decomposition, the oracle's HLLC)."""
    from tests.ref import char1d

    L, n = 32, 8
    x = (np.arange(L) + 0.5) / L
    rng = np.random.default_rng(11)
    rho1 = np.where(x < 0.5, 1.0, 0.125) * (1 + 0.05 * rng.random(L))
    p1 = np.where(x < 0.5, 1.0, 0.1)
    u1 = 0.3 * np.sin(2 * np.pi * x)
    shape = [n, n, n]
    shape[2 - axis] = L

    def field(a):
        s = [1, 1, 1]
        s[2 - axis] = L
        return np.broadcast_to(a.reshape(s), shape).copy()

    z = np.zeros(shape)
    vel = [z, z, z]
    vel[axis] = field(u1)
    dxs = [1.0 / L] * 3
    P = ics.from_primitive("oned", n, field(rho1), vel[0], vel[1], vel[2], field(p1), 1.4, dxs, bc)
    g = grid_of(P)
    U = P.U.copy()
    W = np.stack([rho1, z.reshape(-1)[:L] * 0 + 0, 0 * x, 0 * x, p1])
    W[1] = u1
    hllc = lambda a, b: oracle.hllc(a, b, 0, 1.4)
    for _ in range(3):
        dt = 0.5 * oracle.dt_ctu(g, U, 0.8)
        U, cnt = oracle.step_ctu(g, U, dt, trace=True)
        W = char1d.step(W, dt * L, 1.4, hllc, periodic=bc[axis] == 0)
    G = glob(P, U)
    line = [slice(0, 1)] * 3
    line[2 - axis] = slice(None)
    got = G[(slice(None), *line)].reshape(5, L)
    rho = got[0]
    un = got[1 + axis] / rho
    p = 0.4 * (got[4] - 0.5 * (got[1] ** 2 + got[2] ** 2 + got[3] ** 2) / rho)
    np.testing.assert_allclose(rho, W[0], rtol=1e-13, atol=0)
    np.testing.assert_allclose(un, W[1], rtol=0, atol=1e-13)
    np.testing.assert_allclose(p, W[4], rtol=1e-12, atol=0)


def test_traced_ctu_smooth_acoustic_wave_self_converges_at_second_order():
    """A smooth diagonal sound wave: differences between successive
    resolutions shrink at order >= 1.7."""
    T = 0.2
    sols = []
    for L in (16, 32, 64, 128):
        n = 8
        h = 1.0 / L
        x = (np.arange(L) + 0.5) * h
        X = np.broadcast_to(x[None, None, :], (n, L, L))
        Y = np.broadcast_to(x[None, :, None], (n, L, L))
        s = 1e-2 * np.sin(2 * np.pi * (X + Y))
        rho0, p0 = 1.0, 1.0 / 1.4            # c = 1
        rho = rho0 + s
        un = s / math.sqrt(2.0)              # velocity along (1, 1)/sqrt(2)
        p = p0 + s
        P = ics.from_primitive("acoustic", n, rho, un, un, 0 * s, p, 1.4, (h, h, h), (0, 0, 0))
        g = grid_of(P)
        U, t = P.U.copy(), 0.0
        while t < T - 1e-14:
            d = min(oracle.dt_ctu(g, U, 0.8), T - t)
            U, cnt = oracle.step_ctu(g, U, d, trace=True)
            t += d
        G = glob(P, U)[0][0]
        sols.append(G)
    # restrict each solution to the next coarser grid (2x2 means) and compare
    diffs = []
    for a, b in zip(sols[:-1], sols[1:]):
        bc = 0.25 * (b[0::2, 0::2] + b[1::2, 0::2] + b[0::2, 1::2] + b[1::2, 1::2])
        diffs.append(np.abs(a - bc).mean())
    order = [math.log2(diffs[i] / diffs[i + 1]) for i in range(len(diffs) - 1)]
    assert min(order) >= 1.7, (diffs, order)
