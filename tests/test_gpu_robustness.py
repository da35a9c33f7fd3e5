"""Checkpoint/resume and failure isolation on the device.

* A run checkpointed after 10 steps and resumed in a new grid reaches the
  state of the uninterrupted 20-step run bit for bit (device dt on both).
* A nonphysical state planted from the host (a negative density) is
  counted and reported (HYDRO_ENONPHYS) without disturbing anything else:
  in a batch, every other member stays bitwise equal to its run alone.
"""
import numpy as np
import pytest

from paper_2208_11630_amd import checkpoint, ics

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hy():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2208_11630_amd import hydro

    hydro.lib()
    return hydro


@pytest.mark.parametrize("scheme", ["mh", "rk2"])
def test_resume_from_checkpoint_is_bitwise(hy, tmp_path, scheme):
    print(f"\n[robust] resume {scheme}", flush=True)
    P = ics.kelvin_helmholtz(shape=(64, 64, 32), n=16)
    sch = {"mh": hy.SCHEME_MH, "rk2": hy.SCHEME_RK2}[scheme]

    def fresh():
        G = hy.grid_for(P)
        if sch != hy.SCHEME_MH:
            G.set_scheme(sch)
        return G

    A = fresh()
    for _ in range(20):
        A.step_cfl(0.8)
    B = fresh()
    for _ in range(10):
        B.step_cfl(0.8)
    checkpoint.save(B, str(tmp_path / "ck"), step=10)
    B.close()
    C, rec = checkpoint.load(str(tmp_path / "ck"))
    assert rec["meta"]["step"] == 10 and rec["grid"]["scheme"] == sch
    for _ in range(10):
        C.step_cfl(0.8)
    assert np.array_equal(C.download(), A.download())
    assert C.last_dt() == A.last_dt()


def _poisoned(P):
    U = P.Uc.copy()
    U[0, 0, 3, 4, 5] = -1.0          # negative density in one cell of block 0
    return ics.Problem(P.name, P.n, P.nb, P.dx, P.bc, P.gamma, U)


def test_nonphysical_state_is_reported(hy):
    P = _poisoned(ics.kelvin_helmholtz(shape=(32, 32, 32), n=16))
    G = hy.grid_for(P)
    G.step(1e-4)
    assert G.counters()[2] > 0
    with pytest.raises(hy.HydroError) as e:
        G.dt(0.8)
    assert e.value.code == hy.HYDRO_ENONPHYS


def test_nonphysical_member_leaves_the_batch_untouched(hy):
    sims = ics.ensemble(count=6, seed=9, steps=4, shapes=[(2, 8), (3, 16), (1, 32), (4, 8), (2, 16), (1, 16)])
    sims[2] = _poisoned(sims[2])
    grids = [hy.grid_for(P) for P in sims]
    B = hy.Batch(grids)
    B.step(0.8, 4)
    B.stream.synchronize()
    out = [G.download() for G in grids]
    B.close()
    for i, P in enumerate(sims):
        if i == 2:
            continue
        G = hy.grid_for(P)
        for _ in range(4):
            G.step_cfl(0.8)
        assert np.array_equal(G.download(), out[i]), i
        assert G.counters().tolist() == grids[i].counters().tolist() == [0, 0, 0]
    assert grids[2].counters()[2] > 0
    with pytest.raises(hy.HydroError) as e:
        grids[2].dt(0.8)
    assert e.value.code == hy.HYDRO_ENONPHYS


def test_amr_resume_from_checkpoint_is_bitwise(hy, tmp_path):
    """A three-level mesh: 2 steps, checkpoint, a new mesh from the files,
    2 more steps equals 4 uninterrupted steps (device dt)."""
    from tests.test_gpu_amr import _tree_case, _tree_gpu

    t, U = _tree_case("n8_three_levels")
    A = _tree_gpu(hy, t, U)
    for _ in range(4):
        A.step_cfl(0.8)
    B = _tree_gpu(hy, t, U)
    for _ in range(2):
        B.step_cfl(0.8)
    checkpoint.save_amr(B, str(tmp_path / "amr"), step=2)
    B.close()
    C, rec = checkpoint.load_amr(str(tmp_path / "amr"))
    assert rec["meta"]["step"] == 2 and C.level_blocks == A.level_blocks
    for _ in range(2):
        C.step_cfl(0.8)
    ra, fa = A.download()
    rc, fc = C.download()
    assert np.array_equal(ra, rc) and np.array_equal(fa, fc)
    assert C.last_dt() == A.last_dt()
