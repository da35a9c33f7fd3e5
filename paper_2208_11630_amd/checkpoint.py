"""Checkpoint and resume of a grid: the current state as a raw ``.npy`` array
(compact blocked layout, float64) beside a JSON file with the grid
description, the time-integration scheme, the event counters and whatever
the caller adds (time, step number, seed...).  Nothing is pickled; loading
executes nothing from the files.

A resumed grid continues bit for bit: its first step takes the same dt
(the signal speed of the state is recomputed from the same values) and the
same arithmetic as the uninterrupted run.
"""
from __future__ import annotations

import json
import os
from typing import Any, Dict, Tuple

import numpy as np

FORMAT = "hydro-checkpoint-1"
STATE = "state.npy"
META = "meta.json"


def describe(grid) -> Dict[str, Any]:
    """The grid description a checkpoint records (from the handle's descriptor)."""
    d = grid.desc
    return {
        "nxb": int(d.nxb),
        "nblk": [int(x) for x in d.nblk],
        "lo": [float(x) for x in d.lo],
        "hi": [float(x) for x in d.hi],
        "bc": [int(x) for x in d.bc],
        "gamma": float(d.gamma),
        "small_p": float(d.small_p),
        "nguard": int(d.nguard),
        "scheme": int(getattr(grid, "scheme", 0)),
    }


def write(path: str, grid_desc: Dict[str, Any], state: np.ndarray, counters=None, **meta) -> None:
    """Write a checkpoint directory (created if needed; files replaced)."""
    n = grid_desc["nxb"]
    nb = grid_desc["nblk"]
    shape = (nb[0] * nb[1] * nb[2], 5, n, n, n)
    state = np.ascontiguousarray(state, dtype=np.float64)
    if state.shape != shape:
        raise ValueError(f"state has shape {state.shape}, the grid needs {shape}")
    os.makedirs(path, exist_ok=True)
    tmp = os.path.join(path, STATE + ".tmp")
    with open(tmp, "wb") as f:
        np.save(f, state, allow_pickle=False)
    os.replace(tmp, os.path.join(path, STATE))
    rec = {"format": FORMAT, "grid": grid_desc,
           "counters": [int(c) for c in (counters if counters is not None else (0, 0, 0))],
           "meta": meta}
    tmp = os.path.join(path, META + ".tmp")
    with open(tmp, "w") as f:
        json.dump(rec, f, indent=1)
    os.replace(tmp, os.path.join(path, META))


def read(path: str) -> Tuple[Dict[str, Any], np.ndarray, Dict[str, Any]]:
    """(grid description, state, record) of a checkpoint; validates the format
    and the state's shape against the description."""
    with open(os.path.join(path, META)) as f:
        rec = json.load(f)
    if rec.get("format") != FORMAT:
        raise ValueError(f"not a {FORMAT} checkpoint: {rec.get('format')!r}")
    g = rec["grid"]
    state = np.load(os.path.join(path, STATE), allow_pickle=False)
    n, nb = g["nxb"], g["nblk"]
    shape = (nb[0] * nb[1] * nb[2], 5, n, n, n)
    if state.shape != shape or state.dtype != np.float64:
        raise ValueError(f"checkpoint state {state.shape} {state.dtype} does not match the grid {shape}")
    return g, state, rec


def save(grid, path: str, **meta) -> None:
    """Checkpoint a hydro.Grid (waits for its stream)."""
    write(path, describe(grid), grid.download(), grid.counters().tolist(), **meta)


def load(path: str, device: str = "cuda", stream=None):
    """A new hydro.Grid holding the checkpointed state, and the record's
    caller metadata.  The new grid's event counters start at zero (the
    checkpoint keeps the old ones under ``counters``)."""
    from . import hydro

    g, state, rec = read(path)
    G = hydro.Grid(g["nxb"], g["nblk"], g["lo"], g["hi"], g["bc"], g["gamma"], g["small_p"], device=device,
                   stream=stream, nguard=g["nguard"])
    if g.get("scheme", 0) != hydro.SCHEME_MH:
        G.set_scheme(g["scheme"])
    G.upload(state)
    return G, rec


AMR_FORMAT = "hydro-amr-checkpoint-1"


def save_amr(mesh, path: str, **meta) -> None:
    """Checkpoint a hydro.Amr mesh: root state, the state of deeper levels
    (concatenated, as the mesh stores it) and the mesh description with its
    refinement flags (waits for its stream)."""
    Ur, Uf = mesh.download()
    os.makedirs(path, exist_ok=True)
    for name, arr in (("root.npy", Ur), ("fine.npy", Uf)):
        tmp = os.path.join(path, name + ".tmp")
        with open(tmp, "wb") as f:
            np.save(f, np.ascontiguousarray(arr, dtype=np.float64), allow_pickle=False)
        os.replace(tmp, os.path.join(path, name))
    rec = {"format": AMR_FORMAT,
           "mesh": {"nxb": mesh.nxb, "nblk": list(mesh.nblk), "lo": list(mesh.lo), "hi": list(mesh.hi),
                    "bc": list(mesh.bc), "gamma": mesh.gamma, "small_p": mesh.small_p,
                    "refine": [bool(f) for f in mesh.refine], "refine_deep": [bool(f) for f in mesh.refine_deep]},
           "level_blocks": list(mesh.level_blocks), "counters": mesh.counters().tolist(), "meta": meta}
    tmp = os.path.join(path, META + ".tmp")
    with open(tmp, "w") as f:
        json.dump(rec, f)
    os.replace(tmp, os.path.join(path, META))


def read_amr(path: str):
    """(mesh description, root state, deeper-level state, record)."""
    with open(os.path.join(path, META)) as f:
        rec = json.load(f)
    if rec.get("format") != AMR_FORMAT:
        raise ValueError(f"not a {AMR_FORMAT} checkpoint: {rec.get('format')!r}")
    m = rec["mesh"]
    n, nb = m["nxb"], m["nblk"]
    Ur = np.load(os.path.join(path, "root.npy"), allow_pickle=False)
    Uf = np.load(os.path.join(path, "fine.npy"), allow_pickle=False)
    nfine = sum(rec["level_blocks"][1:])
    if Ur.shape != (nb[0] * nb[1] * nb[2], 5, n, n, n) or Ur.dtype != np.float64:
        raise ValueError("root state does not match the mesh")
    if Uf.shape[1:] != (5, n, n, n) or Uf.shape[0] != nfine or Uf.dtype != np.float64:
        raise ValueError("fine state does not match the mesh")
    return m, Ur, Uf, rec


def load_amr(path: str, device: str = "cuda", stream=None):
    """A new hydro.Amr holding the checkpointed mesh and state, and the record."""
    from . import hydro

    m, Ur, Uf, rec = read_amr(path)
    A = hydro.Amr(m["nxb"], m["nblk"], m["refine"], m["lo"], m["hi"], m["bc"], m["gamma"], m["small_p"],
                  device=device, stream=stream, refine_deep=m["refine_deep"])
    A.upload(Ur, Uf if len(Uf) else None)
    return A, rec
