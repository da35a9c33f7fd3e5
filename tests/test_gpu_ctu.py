"""Parity of the corner-transport-upwind (CTU) step of the HIP path with the
CPU oracle, through the C ABI.

Same bar as the other schemes: after every step the normwise relative error
per conserved variable is at most 1e-12, the dt each side chooses (here by
the per-direction CFL rule) agrees to 1e-14, and the event counters match.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2208_11630_amd import ics
from tests.test_gpu_parity import CASES, DT_TOL, assert_parity, hy, ogrid  # noqa: F401

pytestmark = pytest.mark.gpu

CTU_CASES = ["sod64", "sod_y", "sedov32_n8", "kh_small", "rand_n32_mixed_bc", "rand_n8_ragged",
             "rand_n16_single_block", "rand_n8_single_block", "rand_n32_single_block_outflow"]


def ctu_grid(hy, P, trace=False):
    G = hy.grid_for(P)
    G.set_scheme(hy.SCHEME_CTU_CHAR if trace else hy.SCHEME_CTU)
    return G


@pytest.mark.parametrize("case", CTU_CASES)
def test_one_ctu_step_parity(hy, case):
    P = CASES[case]()
    dt = oracle.dt_ctu(ogrid(P), P.U, P.cfl)
    ref, cnt = oracle.step_ctu(ogrid(P), P.U.copy(), dt)
    G = ctu_grid(hy, P)
    G.step(dt)
    assert_parity(G.download(), ref, P.n, f"{case} ctu")
    assert G.counters().tolist() == cnt.tolist()


@pytest.mark.parametrize("case", ["sod64", "sedov32_n8", "kh_small", "rand_n8_ragged"])
def test_ctu_trajectory_with_device_dt(hy, case):
    """Each side takes its own dt from the per-direction rule for 4 steps."""
    P = CASES[case]()
    g = ogrid(P)
    U = P.U.copy()
    G = ctu_grid(hy, P)
    for s in range(4):
        d_ref = oracle.dt_ctu(g, U, P.cfl)
        G.step_cfl(P.cfl)
        d_gpu = G.last_dt()
        assert abs(d_gpu / d_ref - 1.0) <= DT_TOL, (s, d_gpu, d_ref)
        U, _ = oracle.step_ctu(g, U, d_ref)
        assert_parity(G.download(), U, P.n, f"{case} ctu step {s}")
    assert G.dt(P.cfl) == pytest.approx(oracle.dt_ctu(g, U, P.cfl), rel=DT_TOL)


def test_ctu_uniform_state_bitwise(hy):
    P = ics.uniform(n=16, nb=(2, 1, 2), bc=(1, 0, 1))
    G = ctu_grid(hy, P)
    for _ in range(3):
        G.step_cfl(0.8)
    assert np.array_equal(G.download(), P.Uc)


def test_ctu_full_kh_sampled_blocks(hy):
    """The full-size Kelvin-Helmholtz grid (32x32x16 blocks of 16^3, 65,536
    column tiles): one step against the oracle on blocks at the domain's
    corners and edges and inside."""
    P = ics.kelvin_helmholtz(shape=(512, 512, 256), n=16)
    G = ctu_grid(hy, P)
    dt = 2.0e-4
    G.step(dt)
    out = G.download()
    g = ogrid(P)
    U = P.U
    blocks = [0, 1, 31, 32, 1023, 1024, 8191, 16383]
    for b in blocks:
        oracle.fill_guards_block(g, U, b)
    tmp = np.zeros((1,) + g.shape()[1:])
    for b in blocks:
        cnt = (ctypes.c_long * 3)(0, 0, 0)
        gc = g.c()
        oracle.lib().oracle_ctu_block(ctypes.byref(gc), oracle._dptr(U), b, oracle._dptr(tmp[0]), dt, cnt)
        ref = ics.interior(tmp, P.n)[0]
        got = out[b]
        for v in range(5):
            den = np.abs(ref[v]).max() if v in (0, 4) else np.sqrt((ref[1:4] ** 2).sum(axis=0)).max()
            assert np.abs(got[v] - ref[v]).max() <= 1e-12 * den, (b, v)


def test_ctu_scheme_switch_resets_the_cfl_rule(hy):
    """After switching between CTU and the predictor-corrector step, hydro_dt
    follows the new scheme's rule."""
    P = CASES["rand_n16_single_block"]()
    G = hy.grid_for(P)
    g = ogrid(P)
    assert G.dt(0.8) == pytest.approx(oracle.dt(g, P.U, 0.8), rel=DT_TOL)
    G.set_scheme(hy.SCHEME_CTU)
    assert G.dt(0.8) == pytest.approx(oracle.dt_ctu(g, P.U, 0.8), rel=DT_TOL)
    G.set_scheme(hy.SCHEME_MH)
    assert G.dt(0.8) == pytest.approx(oracle.dt(g, P.U, 0.8), rel=DT_TOL)


def test_ctu_argument_errors(hy):
    """The CTU schemes need no buffer (a stage pointer is ignored); an
    unknown scheme is refused; a CTU grid cannot join a batch."""
    P = CASES["rand_n8_single_block"]()
    G = hy.grid_for(P)
    L = hy.lib()
    assert L.hydro_set_scheme(G.handle, 7, None) == hy.HYDRO_EINVAL
    assert L.hydro_set_scheme(G.handle, hy.SCHEME_CTU, None) == 0
    assert L.hydro_set_scheme(G.handle, hy.SCHEME_CTU_CHAR, ctypes.c_void_p(G.bufs[1].data_ptr())) == 0
    G.set_scheme(hy.SCHEME_CTU)
    with pytest.raises(hy.HydroError):
        hy.Batch([G])
