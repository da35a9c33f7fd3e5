"""Scalar 1-D MUSCL-Hancock for linear advection q_t + a q_x = 0 (a > 0).

The textbook scheme (Toro ch. 14 / van Leer 1979), written independently of
the oracle: van Leer harmonic slopes, boundary-extrapolated values evolved by
half a step, upwind flux, conservative update, periodic.  A pure contact of
the Euler equations (uniform velocity and pressure) must reproduce it in the
density.
"""
import numpy as np


def van_leer(a, b):
    out = np.zeros_like(a)
    m = a * b > 0
    out[m] = 2 * a[m] * b[m] / (a[m] + b[m])
    return out


def step(q, a, lam):
    """One step with lam = a*dt/dx... given as dt/dx; a > 0, periodic."""
    dl = q - np.roll(q, 1)
    dr = np.roll(q, -1) - q
    s = van_leer(dl, dr)
    qr = q + 0.5 * s - 0.5 * lam * a * s      # right face value after the half step
    flux = a * qr                              # upwind: flux at i+1/2 from cell i
    return q - lam * (flux - np.roll(flux, 1))
