"""Pins of the oracle's positivity safeguards (first-order fallback, floors).

A steep pressure jump advected at speed u makes the Hancock predictor push a
face pressure below zero; the per-cell fallback to the cell-centred state must
keep the solution finite and positive while conserving mass, momentum and
energy exactly as before (the fallback only changes face states, never the
conservative form).
"""
import numpy as np
import pytest

import oracle
from paper_2208_11630_amd import ics


def _jump_problem(u0, plo, L=32, n=8):
    x = (np.arange(L) + 0.5) / L
    p1 = np.where(x < 0.5, plo, 1.0)
    Z, Y, X = n, n, L
    f = lambda a: np.broadcast_to(a[None, None, :], (Z, Y, X)).copy()
    zero = np.zeros((Z, Y, X))
    return ics.from_primitive("jump", n, f(np.ones(L)), f(np.full(L, u0)), zero, zero, f(p1), 1.4,
                              (1.0 / L,) * 3, (0, 0, 0))


@pytest.mark.parametrize("u0,plo", [(1.0, 1e-6), (2.0, 1e-4)])
def test_fallback_keeps_state_positive_and_conservative(u0, plo):
    P = _jump_problem(u0, plo)
    g = oracle.Grid(P.n, P.nb, P.dx, P.bc, P.gamma)
    U = P.U
    total = np.zeros(3, dtype=np.int64)
    G0 = ics.from_blocks(U, P.n, P.nb)
    for _ in range(30):
        d = oracle.dt(g, U, 0.8)
        assert d > 0
        U, c = oracle.step(g, U, d)
        total += c
    G = ics.from_blocks(U, P.n, P.nb)
    assert total[oracle.CNT_FALLBACK] > 0          # the safeguard was exercised
    assert total[oracle.CNT_NONPHYS] == 0 and total[oracle.CNT_FLOOR] == 0
    assert np.isfinite(G).all()
    p = 0.4 * (G[4] - 0.5 * (G[1] ** 2 + G[2] ** 2 + G[3] ** 2) / G[0])
    assert G[0].min() > 0 and p.min() > 0
    for v in range(5):
        assert abs(G[v].sum() - G0[v].sum()) <= 1e-13 * np.abs(G0[v]).sum() + 1e-300
    assert np.array_equal(G, np.broadcast_to(G[:, :1, :1, :], G.shape))


def test_floor_counts_interior_cells_only():
    """A cell whose internal energy is negative is floored and counted once,
    however many neighbouring blocks also read it as a guard cell."""
    P = ics.uniform(n=8, nb=(2, 2, 2), vel=(0.0, 0.0, 0.0), p=1.0)
    U = P.U
    # interior cell (0, 0, 0) of block 0: kinetic energy larger than E
    ng = 4
    U[0, 1, ng, ng, ng] = 3.0 * U[0, 0, ng, ng, ng]
    g = oracle.Grid(P.n, P.nb, P.dx, P.bc, P.gamma)
    _, cnt = oracle.step(g, U, 1e-4)
    assert cnt[oracle.CNT_FLOOR] == 1
