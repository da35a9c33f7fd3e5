"""The allocation-free batch step (hydro_batch_step_static) against the
handle-based batch (hydro_batch_create + hydro_batch_step) on the same
inputs: member states bitwise equal (the same kernels and per-grid device
dt), dts and event counters equal; two calls in a row, the second with a
smaller batch, so that the static scratch's leftover tables from the first
call must not leak into the second."""
import numpy as np
import pytest

from paper_2208_11630_amd import ics

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hy():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2208_11630_amd import hydro

    hydro.lib()
    return hydro


def _members(count, seed):
    rng = np.random.default_rng(seed)
    shapes = [(int(rng.integers(1, 7)), [8, 16, 32][i % 3]) for i in range(count)]
    return ics.ensemble(count=count, seed=seed, steps=4, shapes=shapes)


def _with_batch(hy, sims, k, nseg):
    grids = [hy.grid_for(P) for P in sims]
    B = hy.Batch(grids)
    B.set_pencils(*nseg)
    B.step(0.8, k)
    B.synchronize()
    B.close()
    return grids


def _static(hy, sims, k, nseg):
    import torch

    grids = [hy.grid_for(P) for P in sims]
    hy.batch_step_static(grids, 0.8, k, nseg=nseg)
    torch.cuda.synchronize()
    return grids


def _compare(a, b):
    for i, (ga, gb) in enumerate(zip(a, b)):
        assert np.array_equal(ga.download(), gb.download()), f"member {i}"
        assert ga.last_dt() == gb.last_dt(), f"member {i} dt"
        assert np.array_equal(ga.counters(), gb.counters()), f"member {i} counters"


def test_static_batch_matches_batch_on_two_calls(hy):
    big = _members(14, 31)
    small = _members(5, 32)
    print("[no-alloc] call 1: 14 members, 4 steps, pencils (2, 1, 4)", flush=True)
    ref1 = _with_batch(hy, big, 4, (2, 1, 4))
    got1 = _static(hy, big, 4, (2, 1, 4))
    _compare(ref1, got1)
    print("[no-alloc] call 2: 5 members, 3 steps, pencils (1, 1, 1)", flush=True)
    ref2 = _with_batch(hy, small, 3, (1, 1, 1))
    got2 = _static(hy, small, 3, (1, 1, 1))
    _compare(ref2, got2)


def test_static_batch_continues_a_grid_and_rejects_oversize(hy):
    import ctypes

    sims = _members(4, 33)
    ref = [hy.grid_for(P) for P in sims]
    for G in ref:
        for _ in range(3):
            G.step_cfl(0.8)
    got = [hy.grid_for(P) for P in sims]
    for G in got:
        G.step_cfl(0.8)                          # one plain step, then two static ones
    hy.batch_step_static(got, 0.8, 2)
    _compare(ref, got)
    arr = (ctypes.c_void_p * 4097)(*([got[0].handle.value] * 4097))
    rc = hy.lib().hydro_batch_step_static(arr, 4097, None, 0.8, 1, None)
    assert rc == hy.HYDRO_ESIZE


def test_static_batch_argument_errors_leave_the_grids_usable(hy):
    """A grid listed twice, a grid of a batch and a grid on another scheme
    are refused (HYDRO_EINVAL) before any launch; a refused call leaves
    nothing behind, so the same grids then step normally."""
    sims = _members(3, 34)
    ref = [hy.grid_for(P) for P in sims]
    for G in ref:
        G.step_cfl(0.8)
    got = [hy.grid_for(P) for P in sims]
    with pytest.raises(hy.HydroError, match="twice"):
        hy.batch_step_static([got[0], got[1], got[0]], 0.8, 1)
    B = hy.Batch([got[2]])
    with pytest.raises(hy.HydroError, match="batch"):
        hy.batch_step_static(got, 0.8, 1)
    B.close()
    R = hy.grid_for(sims[0])
    R.set_scheme(hy.SCHEME_RK2)
    with pytest.raises(hy.HydroError, match="scheme"):
        hy.batch_step_static([got[1], R], 0.8, 1)
    hy.batch_step_static(got, 0.8, 1)            # the same grids, each once
    _compare(ref, got)
