"""Exact solution of the 1-D Riemann problem for a gamma-law gas.

Written from the standard derivation (Toro, Riemann Solvers and Numerical
Methods for Fluid Dynamics, ch. 4): the star pressure solves
f_L(p) + f_R(p) + (u_R - u_L) = 0 with the shock (Rankine-Hugoniot) and
rarefaction (isentropic) branches of f_K; the solution is then sampled on
x/t.  Independent of the oracle: used to pin it on the Sod problem.
"""
from __future__ import annotations

import math

import numpy as np


def _f(p, rho, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def star_state(rL, uL, pL, rR, uR, pR, g):
    """(p*, u*) by bisection on the monotone pressure function (robust, exact to 1e-15)."""
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    F = lambda p: _f(p, rL, pL, cL, g) + _f(p, rR, pR, cR, g) + (uR - uL)
    lo, hi = 1e-14, max(pL, pR)
    while F(hi) < 0:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if F(mid) > 0:
            hi = mid
        else:
            lo = mid
    p = 0.5 * (lo + hi)
    u = 0.5 * (uL + uR) + 0.5 * (_f(p, rR, pR, cR, g) - _f(p, rL, pL, cL, g))
    return p, u


def sample(rL, uL, pL, rR, uR, pR, g, xi):
    """(rho, u, p) at similarity coordinates xi = (x - x0)/t (array)."""
    ps, us = star_state(rL, uL, pL, rR, uR, pR, g)
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    gm = (g - 1.0) / (g + 1.0)
    for idx, s in np.ndenumerate(xi):
        if s <= us:  # left of contact
            if ps > pL:  # left shock
                SL = uL - cL * math.sqrt((g + 1) / (2 * g) * ps / pL + (g - 1) / (2 * g))
                if s <= SL:
                    r, uu, pp = rL, uL, pL
                else:
                    r = rL * ((ps / pL + gm) / (gm * ps / pL + 1.0))
                    uu, pp = us, ps
            else:  # left rarefaction
                cs = cL * (ps / pL) ** ((g - 1) / (2 * g))
                head, tail = uL - cL, us - cs
                if s <= head:
                    r, uu, pp = rL, uL, pL
                elif s >= tail:
                    r, uu, pp = rL * (ps / pL) ** (1.0 / g), us, ps
                else:
                    r = rL * (2 / (g + 1) + gm / cL * (uL - s)) ** (2 / (g - 1))
                    uu = 2 / (g + 1) * (cL + (g - 1) / 2 * uL + s)
                    pp = pL * (2 / (g + 1) + gm / cL * (uL - s)) ** (2 * g / (g - 1))
        else:
            if ps > pR:  # right shock
                SR = uR + cR * math.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
                if s >= SR:
                    r, uu, pp = rR, uR, pR
                else:
                    r = rR * ((ps / pR + gm) / (gm * ps / pR + 1.0))
                    uu, pp = us, ps
            else:
                cs = cR * (ps / pR) ** ((g - 1) / (2 * g))
                head, tail = uR + cR, us + cs
                if s >= head:
                    r, uu, pp = rR, uR, pR
                elif s <= tail:
                    r, uu, pp = rR * (ps / pR) ** (1.0 / g), us, ps
                else:
                    r = rR * (2 / (g + 1) - gm / cR * (uR - s)) ** (2 / (g - 1))
                    uu = 2 / (g + 1) * (-cR + (g - 1) / 2 * uR + s)
                    pp = pR * (2 / (g + 1) - gm / cR * (uR - s)) ** (2 * g / (g - 1))
        rho[idx], u[idx], p[idx] = r, uu, pp
    return rho, u, p


def cell_average(rL, uL, pL, rR, uR, pR, g, x0, t, edges, sub=64):
    """Cell averages of (rho, rho*u, E) over cells with the given edges (sub-sampled midpoint rule)."""
    edges = np.asarray(edges, dtype=np.float64)
    out = np.zeros((3, len(edges) - 1))
    for c in range(len(edges) - 1):
        xs = edges[c] + (np.arange(sub) + 0.5) / sub * (edges[c + 1] - edges[c])
        r, u, p = sample(rL, uL, pL, rR, uR, pR, g, (xs - x0) / t)
        out[0, c] = r.mean()
        out[1, c] = (r * u).mean()
        out[2, c] = (p / (g - 1) + 0.5 * r * u * u).mean()
    return out
