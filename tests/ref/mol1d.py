"""Scalar 1-D method of lines for linear advection q_t + a q_x = 0 (a > 0),
advanced by the Shu-Osher SSP Runge-Kutta schemes of order 2 and 3.

Written independently of the oracle from the textbook statement (Shu and
Osher 1988; Gottlieb and Shu 1998): van Leer harmonic slopes, the face value
of cell i at i+1/2 is q_i + s_i/2, upwind flux a*q at that face, periodic.
A pure contact of the Euler equations must reproduce it in the density.
"""
import numpy as np

from .muscl1d import van_leer


def rhs(q, a, lam):
    """dt * L(q) for a step with lam = dt/dx."""
    s = van_leer(q - np.roll(q, 1), np.roll(q, -1) - q)
    flux = a * (q + 0.5 * s)
    return -lam * (flux - np.roll(flux, 1))


def step(q, a, lam, order):
    q1 = q + rhs(q, a, lam)
    if order == 2:
        return 0.5 * q + 0.5 * (q1 + rhs(q1, a, lam))
    q2 = 0.75 * q + 0.25 * (q1 + rhs(q1, a, lam))
    return q / 3.0 + 2.0 / 3.0 * (q2 + rhs(q2, a, lam))
