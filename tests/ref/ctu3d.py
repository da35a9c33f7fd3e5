"""Scalar three-dimensional corner transport upwind (CTU) scheme for linear
advection q_t + a q_x + b q_y + c q_z = 0 with a, b, c > 0, periodic.

Written from the textbook statement of the unsplit CTU method with twelve
upwind fluxes per cell (Colella 1990; Saltzman 1994; Gardiner & Stone
2008), independently of the oracle: van Leer slopes, normal half-step face
values, one-dimensional fluxes, corner values corrected by one transverse
flux difference with weight lam/3, final values corrected by the two cross
corner-flux differences with weight lam/2, conservative update.  Arrays are
indexed [z, y, x].  A pure contact of the Euler equations (uniform velocity
and pressure) must reproduce it in the density.
"""
import numpy as np

from .muscl1d import van_leer

AXIS = {0: 2, 1: 1, 2: 0}          # direction -> array axis
PAIRS = {0: (1, 2), 1: (0, 2), 2: (0, 1)}


def _at(f, d, s):
    """f at the cell s steps along direction d (periodic)."""
    return np.roll(f, -s, axis=AXIS[d])


def step(q, vel, lam):
    """One step; vel = (a, b, c) > 0, lam = (dt/dx, dt/dy, dt/dz)."""
    slope = [van_leer(q - _at(q, d, -1), _at(q, d, 1) - q) for d in range(3)]
    # high-face value of each cell after the normal half step (the upwind side)
    qp = [q + 0.5 * (1.0 - vel[d] * lam[d]) * slope[d] for d in range(3)]
    # flux at the low d-face of each cell comes from the neighbour below
    f1 = [vel[d] * _at(qp[d], d, -1) for d in range(3)]
    corner = {}
    for d in range(3):
        for t in PAIRS[d]:
            qc = qp[d] - (lam[t] / 3.0) * (_at(f1[t], t, 1) - f1[t])
            corner[(d, t)] = vel[d] * _at(qc, d, -1)
    flux = []
    for d in range(3):
        t, u = PAIRS[d]
        qf = qp[d] - 0.5 * (lam[t] * (_at(corner[(t, u)], t, 1) - corner[(t, u)]) +
                            lam[u] * (_at(corner[(u, t)], u, 1) - corner[(u, t)]))
        flux.append(vel[d] * _at(qf, d, -1))
    div = (lam[0] * (_at(flux[0], 0, 1) - flux[0]) + lam[1] * (_at(flux[1], 1, 1) - flux[1])) + \
        lam[2] * (_at(flux[2], 2, 1) - flux[2])
    return q - div
