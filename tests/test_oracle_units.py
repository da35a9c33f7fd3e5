"""Pins of the oracle's pieces against facts that do not come from the oracle.

Each check is a closed form, an exact identity of the method, or a textbook
special case; a dropped term, a wrong sign or a swapped operand in the
oracle's limiter, EOS, Euler flux or HLLC fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

import oracle
from tests.ref import exact_riemann as er

G14 = 1.4


# ---- exact Riemann reference pinned to the textbook table -----------------

def _golden_star():
    path = os.path.join(os.path.dirname(__file__), "golden", "riemann_star_states.txt")
    rows = []
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        a, b = line.split("|")
        # tolerance: one unit of the last printed digit of each tabulated value,
        # or 1e-5 relative (test 5's inputs are themselves 6-digit roundings)
        tol = [max(10.0 ** -(len(x.split(".")[1]) if "." in x else 0), 1e-5 * abs(float(x)))
               for x in b.split()]
        rows.append(([float(x) for x in a.split()], [float(x) for x in b.split()], tol))
    return rows


@pytest.mark.parametrize("case", range(5))
def test_exact_riemann_matches_textbook_table(case):
    states, star, tol = _golden_star()[case]
    p, u = er.star_state(*states, G14)
    rl, _, _ = er.sample(*states, G14, np.array([u - 1e-9]))
    rr, _, _ = er.sample(*states, G14, np.array([u + 1e-9]))
    for got, want, t in zip((p, u, rl[0], rr[0]), star, tol):
        assert abs(got - want) <= t, (got, want, t)


# ---- van Leer harmonic limiter ----------------------------------------------

@pytest.mark.parametrize("a", [1e-150, 1e-12, 0.37, 5.0, 3e5])
def test_van_leer_special_cases(a):
    vl = oracle.van_leer
    assert vl(a, a) == a
    assert vl(-a, -a) == -a
    assert vl(a, -a) == 0.0 and vl(-a, 2 * a) == 0.0
    assert vl(0.0, a) == 0.0 and vl(a, 0.0) == 0.0


def test_van_leer_closed_form_and_bounds():
    vl = oracle.van_leer
    assert vl(1.0, 3.0) == 1.5          # 2*1*3/(1+3)
    assert vl(-2.0, -6.0) == -3.0
    rng = np.random.default_rng(7)
    for _ in range(2000):
        a, b = rng.normal(size=2) * 10.0 ** rng.integers(-6, 6, size=2)
        s = vl(a, b)
        assert s == vl(b, a)
        if a * b > 0:
            assert np.sign(s) == np.sign(a)
            assert abs(s) <= 2 * min(abs(a), abs(b)) * (1 + 1e-15)
            assert abs(s) >= min(abs(a), abs(b)) * (1 - 1e-15)   # harmonic mean >= min
        else:
            assert s == 0.0


# ---- EOS ---------------------------------------------------------------------

def test_cons_prim_round_trip_and_floor():
    rng = np.random.default_rng(3)
    for _ in range(500):
        rho = math.exp(rng.normal())
        vel = rng.normal(size=3)
        p = math.exp(rng.normal())
        g = rng.choice([1.4, 5.0 / 3.0, 1.1])
        U = [rho, rho * vel[0], rho * vel[1], rho * vel[2],
             p / (g - 1) + 0.5 * rho * float(vel @ vel)]
        W, floored = oracle.cons_to_prim(U, g)
        assert not floored
        np.testing.assert_allclose(W, [rho, *vel, p], rtol=1e-12, atol=1e-14)
    # internal energy below the floor: pressure clipped to small_p, flagged
    W, floored = oracle.cons_to_prim([1.0, 1.0, 0.0, 0.0, 0.4], 1.4, 1e-10)
    assert floored and W[4] == 1e-10


# ---- Euler flux and HLLC -------------------------------------------------------

def _flux_alt(W, d, g):
    """F = u_n * U + p * (0, e_d, u_n): the conservative flux written in the
    alternative 'advective + pressure' form, independent of the oracle's."""
    rho, u, v, w, p = W
    E = p / (g - 1) + 0.5 * rho * (u * u + v * v + w * w)
    U = np.array([rho, rho * u, rho * v, rho * w, E])
    un = W[1 + d]
    extra = np.zeros(5)
    extra[1 + d] = p
    extra[4] = p * un
    return un * U + extra


def _rand_state(rng, sup=False):
    W = np.array([math.exp(rng.normal()), *rng.normal(size=3), math.exp(rng.normal())])
    return W


@pytest.mark.parametrize("d", [0, 1, 2])
def test_euler_flux_alternative_form(d):
    rng = np.random.default_rng(11 + d)
    for _ in range(200):
        W = _rand_state(rng)
        np.testing.assert_allclose(oracle.euler_flux(W, d, G14), _flux_alt(W, d, G14), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_hllc_consistency(d):
    """F(W, W) = F(W): every wave-speed branch reduces to the physical flux."""
    rng = np.random.default_rng(21 + d)
    for _ in range(300):
        W = _rand_state(rng)
        W[1 + d] *= 3.0   # visit supersonic left/right and subsonic cases
        F = oracle.hllc(W, W, d, G14)
        np.testing.assert_allclose(F, _flux_alt(W, d, G14), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_hllc_supersonic_upwinding_is_exact(d):
    WL = np.array([1.0, 0.1, -0.2, 0.3, 1.0])
    WR = np.array([0.5, -0.3, 0.4, 0.2, 0.6])
    WL[1 + d] = 5.0
    WR[1 + d] = 4.0     # S_L = min(uL - cL, uR - cR) > 0
    assert np.array_equal(oracle.hllc(WL, WR, d, G14), oracle.euler_flux(WL, d, G14))
    WL[1 + d], WR[1 + d] = -5.0, -6.0
    assert np.array_equal(oracle.hllc(WL, WR, d, G14), oracle.euler_flux(WR, d, G14))


@pytest.mark.parametrize("d", [0, 1, 2])
def test_hllc_stationary_contact(d):
    """u = 0, equal pressure, density jump: the flux is pure pressure."""
    WL = np.array([1.0, 0.0, 0.0, 0.0, 0.7])
    WR = np.array([0.1, 0.0, 0.0, 0.0, 0.7])
    F = oracle.hllc(WL, WR, d, G14)
    expect = np.zeros(5)
    expect[1 + d] = 0.7
    np.testing.assert_allclose(F, expect, rtol=0, atol=1e-15)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_hllc_moving_contact_and_shear_exact(d):
    """An isolated contact/shear wave (equal u_n and p, jumps in rho and in the
    tangential velocities) is resolved exactly: the flux is the upwind side's."""
    t1, t2 = [k for k in range(3) if k != d]
    for un in (0.4, -0.4):
        WL = np.zeros(5)
        WR = np.zeros(5)
        WL[0], WR[0] = 1.0, 0.25
        WL[1 + d] = WR[1 + d] = un
        WL[1 + t1], WR[1 + t1] = 0.3, -0.7
        WL[1 + t2], WR[1 + t2] = -0.1, 0.2
        WL[4] = WR[4] = 2.0
        F = oracle.hllc(WL, WR, d, G14)
        up = WL if un > 0 else WR
        np.testing.assert_allclose(F, _flux_alt(up, d, G14), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_hllc_mirror_antisymmetry(d):
    """Reflecting the normal axis (swap L and R, negate u_n) negates the mass and
    energy fluxes and the tangential momentum fluxes, keeps the normal one."""
    rng = np.random.default_rng(31 + d)
    for _ in range(300):
        WL, WR = _rand_state(rng), _rand_state(rng)
        F = oracle.hllc(WL, WR, d, G14)
        mL, mR = WR.copy(), WL.copy()
        mL[1 + d] *= -1
        mR[1 + d] *= -1
        Fm = oracle.hllc(mL, mR, d, G14)
        sign = -np.ones(5)
        sign[1 + d] = 1
        scale = np.abs(F).max() + np.abs(WL).max() + np.abs(WR).max()
        np.testing.assert_allclose(Fm, sign * F, rtol=0, atol=1e-13 * scale)


def _godunov_flux(WL, WR, g):
    r, u, p = er.sample(WL[0], WL[1], WL[4], WR[0], WR[1], WR[4], g, np.array([0.0]))
    vt = WL[2:4] if u[0] > 0 else WR[2:4]
    return _flux_alt(np.array([r[0], u[0], vt[0], vt[1], p[0]]), 0, g)


def test_hllc_converges_to_exact_godunov_flux():
    """For a jump of size eps the HLLC flux differs from the exact Godunov flux
    (exact Riemann solution sampled at x/t = 0) by O(eps^2): consistent to
    second order in the jump, on every wave-pattern case."""
    base = np.array([1.0, 0.2, 0.1, -0.3, 1.0])
    for direction in (np.array([-1.0, -1.0, 0.3, 0.2, -0.5]),   # 2-shock-ish
                      np.array([1.0, 1.0, -0.3, 0.1, 0.5]),     # rarefactions
                      np.array([-0.7, 0.0, 0.5, 0.5, 0.0])):    # contact + shear
        prev = None
        for eps in (1e-1, 1e-2, 1e-3):
            WL, WR = base, base + eps * direction
            err = np.abs(oracle.hllc(WL, WR, 0, G14) - _godunov_flux(WL, WR, G14)).max()
            if prev is not None:
                assert err < 0.05 * prev + 1e-14, (eps, err, prev)
            prev = err
