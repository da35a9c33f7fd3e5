"""One-dimensional MUSCL-Hancock step of the Euler equations with
characteristic tracing (Colella 1990; Stone et al. 2008, the upwind
projection), written independently of the oracle's tracing: the primitive
Jacobian is built as a matrix and decomposed by numpy's eigensolver, each
van Leer primitive slope is split over its eigenvectors, and a face keeps
the waves moving toward it:

    high face: W + sum_{lambda_k > 0} (1 - lam lambda_k)/2 (L S)_k R_k
    low face:  W - sum_{lambda_k < 0} (1 + lam lambda_k)/2 (L S)_k R_k

Fluxes come from a Riemann solver passed in (the tests pass the oracle's
HLLC, which its own pins fix); conservative update.  Arrays are [5, X] of
primitives (rho, u, v, w, p); x is the normal direction.  Boundaries: two
ghost cells per side, periodic or zero-gradient outflow.
"""
import numpy as np

from .muscl1d import van_leer


def jacobian(W, gamma, d=0):
    """Primitive-variable Jacobian A_d of the Euler equations at W."""
    rho, p = W[0], W[4]
    un = W[1 + d]
    A = np.diag([un] * 5).astype(float)
    A[0, 1 + d] = rho
    A[1 + d, 4] = 1.0 / rho
    A[4, 1 + d] = gamma * p
    return A


def traced_faces(W, S, lam, gamma, d=0):
    """(low, high) face states of one cell by the eigen-decomposition."""
    lamk, R = np.linalg.eig(jacobian(W, gamma, d))
    lamk, R = lamk.real, R.real
    beta = np.linalg.solve(R, S)
    hi = W.astype(float).copy()
    lo = W.astype(float).copy()
    for k in range(5):
        if lamk[k] > 0:
            hi = hi + 0.5 * (1.0 - lam * lamk[k]) * beta[k] * R[:, k]
        if lamk[k] < 0:
            lo = lo - 0.5 * (1.0 + lam * lamk[k]) * beta[k] * R[:, k]
    return lo, hi


def to_cons(W, gamma):
    rho, u, v, w, p = W
    return np.array([rho, rho * u, rho * v, rho * w, p / (gamma - 1.0) + 0.5 * rho * ((u * u + v * v) + w * w)])


def to_prim(U, gamma):
    rho = U[0]
    u, v, w = U[1] / rho, U[2] / rho, U[3] / rho
    return np.array([rho, u, v, w, (gamma - 1.0) * (U[4] - 0.5 * rho * ((u * u + v * v) + w * w))])


def step(W, lam, gamma, riemann, periodic=True):
    """One step on primitives W [5, X]; returns the new primitives."""
    X = W.shape[1]
    idx = np.arange(-2, X + 2)
    idx = np.mod(idx, X) if periodic else np.clip(idx, 0, X - 1)
    Wg = W[:, idx]                                   # cells -2 .. X+1
    lo = np.zeros((5, X + 2))
    hi = np.zeros((5, X + 2))
    for i in range(1, X + 3):                        # cells -1 .. X
        S = van_leer(Wg[:, i] - Wg[:, i - 1], Wg[:, i + 1] - Wg[:, i])
        l, h = traced_faces(Wg[:, i], S, lam, gamma)
        if min(l[0], l[4], h[0], h[4]) <= 0:
            l = h = Wg[:, i]
        lo[:, i - 1], hi[:, i - 1] = l, h
    F = np.stack([riemann(hi[:, i], lo[:, i + 1]) for i in range(X + 1)], axis=1)   # faces -1/2 .. X-1/2
    U = np.stack([to_cons(W[:, i], gamma) for i in range(X)], axis=1)
    U = U - lam * (F[:, 1:] - F[:, :-1])
    return np.stack([to_prim(U[:, i], gamma) for i in range(X)], axis=1)
