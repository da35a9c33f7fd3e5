"""Parity of the SSP Runge-Kutta steps (method-of-lines stages) of the HIP
path with the CPU oracle, through the C ABI.

Same bar as the predictor-corrector step: after every step the normwise
relative error per conserved variable is at most 1e-12, the dt each side
chooses agrees to 1e-14, and the event counters (summed over stages) match.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2208_11630_amd import ics
from tests.test_gpu_parity import CASES, DT_TOL, assert_parity, hy, ogrid  # noqa: F401

pytestmark = pytest.mark.gpu

RK_CASES = ["sod64", "sedov32_n8", "kh_small", "rand_n32_mixed_bc", "rand_n8_ragged", "rand_n16_single_block",
            "rand_n8_single_block"]


def rk_grid(hy, P, order):
    G = hy.grid_for(P)
    G.set_scheme(hy.SCHEME_RK2 if order == 2 else hy.SCHEME_RK3)
    return G


@pytest.mark.parametrize("order", [2, 3])
@pytest.mark.parametrize("case", RK_CASES)
def test_one_rk_step_parity(hy, case, order):
    P = CASES[case]()
    dt = oracle.dt(ogrid(P), P.U, P.cfl)
    ref, cnt = oracle.step_rk(ogrid(P), P.U.copy(), dt, order)
    G = rk_grid(hy, P, order)
    before = G.state.data_ptr()
    G.step(dt)
    out = G.download()
    assert G.state.data_ptr() == before  # the state stays in its buffer
    assert_parity(out, ref, P.n, f"{case} rk{order}")
    assert G.counters().tolist() == cnt.tolist()


@pytest.mark.parametrize("order", [2, 3])
@pytest.mark.parametrize("case", ["sod64", "sedov32_n8", "rand_n8_ragged"])
def test_rk_trajectory_with_device_dt(hy, case, order):
    """Each side picks its own dt (device: cfl / reduced signal speed of the
    last stage's result) for several steps."""
    P = CASES[case]()
    g = ogrid(P)
    U = P.U.copy()
    G = rk_grid(hy, P, order)
    for s in range(4):
        d_ref = oracle.dt(g, U, P.cfl)
        G.step_cfl(P.cfl)
        d_gpu = G.last_dt()
        assert abs(d_gpu / d_ref - 1.0) <= DT_TOL, (s, d_gpu, d_ref)
        U, _ = oracle.step_rk(g, U, d_ref, order)
        assert_parity(G.download(), U, P.n, f"{case} rk{order} step {s}")
    assert G.dt(P.cfl) == pytest.approx(oracle.dt(g, U, P.cfl), rel=DT_TOL)


def test_rk2_uniform_state_bitwise(hy):
    P = ics.uniform(n=16, nb=(2, 1, 2), bc=(1, 0, 1))
    G = rk_grid(hy, P, 2)
    for _ in range(3):
        G.step_cfl(0.8)
    assert np.array_equal(G.download(), P.Uc)


@pytest.mark.parametrize("order", [2, 3])
def test_rk_pencils_bitwise_invariant(hy, order):
    P = CASES["rand_n32_mixed_bc"]()
    outs = []
    for nseg in (1, 2, 4):
        G = rk_grid(hy, P, order)
        G.set_pencils(nseg)
        G.step_cfl(0.8)
        G.step_cfl(0.8)
        outs.append(G.download())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_scheme_switch_mid_run(hy):
    """A predictor-corrector step followed by an RK2 and an RK3 step."""
    P = CASES["rand_n16_single_block"]()
    g = ogrid(P)
    U = P.U.copy()
    G = hy.grid_for(P)
    for scheme, order in ((hy.SCHEME_MH, 0), (hy.SCHEME_RK2, 2), (hy.SCHEME_RK3, 3)):
        G.set_scheme(scheme)
        d = oracle.dt(g, U, 0.8)
        G.step(d)
        U, _ = oracle.step_rk(g, U, d, order) if order else oracle.step(g, U, d)
        assert_parity(G.download(), U, P.n, f"scheme {scheme}")


def test_scheme_argument_errors(hy):
    P = CASES["rand_n8_single_block"]()
    G = hy.grid_for(P)
    L = hy.lib()
    assert L.hydro_set_scheme(G.handle, hy.SCHEME_RK3, None) == hy.HYDRO_EINVAL
    assert L.hydro_set_scheme(G.handle, 1, None) == hy.HYDRO_EINVAL
    # the stage buffer may not alias a state buffer
    assert L.hydro_set_scheme(G.handle, hy.SCHEME_RK3, ctypes.c_void_p(G.bufs[1].data_ptr())) == hy.HYDRO_EINVAL
    G.set_scheme(hy.SCHEME_RK2)
    with pytest.raises(hy.HydroError):
        hy.Batch([G])
