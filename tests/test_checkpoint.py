"""Checkpoint files (host side): the state and the grid description round
trip bit for bit; malformed checkpoints are refused.  No device needed."""
import json
import os

import numpy as np
import pytest

from paper_2208_11630_amd import checkpoint, hydro


class _FakeGrid:
    def __init__(self, nxb, nblk, **kw):
        self.desc = hydro.make_desc(nxb, nblk, **kw)
        self.scheme = hydro.SCHEME_RK2


def test_round_trip_is_bitwise(tmp_path):
    G = _FakeGrid(8, (2, 1, 3), lo=(0.0, -1.0, 0.5), hi=(1.0, 1.0, 2.0), bc=(1, 0, 1), gamma=5 / 3)
    rng = np.random.default_rng(7)
    U = rng.normal(size=(6, 5, 8, 8, 8))
    U[0, 0, 0, 0, 0] = -0.0
    U[1, 2, 3, 4, 5] = 5e-324                       # a subnormal survives
    desc = checkpoint.describe(G)
    checkpoint.write(str(tmp_path / "c"), desc, U, counters=[1, 2, 3], t=0.125, step=10, seed=7)
    g, V, rec = checkpoint.read(str(tmp_path / "c"))
    assert V.tobytes() == U.tobytes()
    assert g == desc and g["scheme"] == hydro.SCHEME_RK2 and g["bc"] == [1, 0, 1]
    assert g["gamma"] == 5 / 3 and g["lo"] == [0.0, -1.0, 0.5]
    assert rec["counters"] == [1, 2, 3] and rec["meta"] == {"t": 0.125, "step": 10, "seed": 7}
    # rewriting replaces the files
    checkpoint.write(str(tmp_path / "c"), desc, 2 * U, step=11)
    assert np.array_equal(checkpoint.read(str(tmp_path / "c"))[1], 2 * U)


def test_malformed_checkpoints_are_refused(tmp_path):
    G = _FakeGrid(8, (2, 1, 1))
    desc = checkpoint.describe(G)
    with pytest.raises(ValueError):
        checkpoint.write(str(tmp_path / "a"), desc, np.zeros((3, 5, 8, 8, 8)))
    checkpoint.write(str(tmp_path / "b"), desc, np.zeros((2, 5, 8, 8, 8)))
    meta = tmp_path / "b" / checkpoint.META
    rec = json.loads(meta.read_text())
    rec["grid"]["nblk"] = [3, 1, 1]
    meta.write_text(json.dumps(rec))
    with pytest.raises(ValueError):
        checkpoint.read(str(tmp_path / "b"))
    rec["grid"]["nblk"] = [2, 1, 1]
    rec["format"] = "something-else"
    meta.write_text(json.dumps(rec))
    with pytest.raises(ValueError):
        checkpoint.read(str(tmp_path / "b"))
    # an object array is never loaded
    rec["format"] = checkpoint.FORMAT
    meta.write_text(json.dumps(rec))
    np.save(str(tmp_path / "b" / checkpoint.STATE), np.array([{"x": 1}], dtype=object), allow_pickle=True)
    with pytest.raises(ValueError):
        checkpoint.read(str(tmp_path / "b"))
    assert not os.path.exists(tmp_path / "b" / (checkpoint.STATE + ".tmp"))
