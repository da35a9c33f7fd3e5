"""Benchmark: FP64 cell-updates/s of the unsplit Godunov hydro step on MI355X.

One "step" is one pass of the whole hot path over the grid: the CFL dt formed
on the device from the signal speed the previous step reduced, the fused
guard fill + primitive recovery + PLM/van Leer + Hancock predictor + HLLC
x/y/z + conservative update, and the signal-speed reduction of the new state
(one kernel launch per step).  The default workload is the 512 x 512 x 256
Kelvin-Helmholtz grid (16^3 blocks, 67.1M cells).  Inputs are resident in
HBM before the timed region starts.

Prints one JSON line (see the fields below).  --gpus N > 1 is refused: this
build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
BYTES_PER_CELL = 80.0          # read 5 doubles of U, write 5 doubles of U'


def make_workload(name):
    from paper_2208_11630_amd import ics

    if name == "kh":
        return ics.kelvin_helmholtz(), "kelvin_helmholtz_512x512x256_nxb16"
    if name == "sedov":
        return ics.sedov(), "sedov_256^3_nxb16"
    if name == "sod":
        return ics.sod(), "sod_64^3_nxb16"
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(P, seconds_target=15.0):
    """The oracle (plain FP64 C, OpenMP over blocks) on a bounded sample of the
    same workload: one step of the first nb blocks of the grid, nb doubling
    until one timing takes at least half the target (or covers the grid)."""
    import numpy as np

    import oracle

    g = oracle.Grid(P.n, P.nb, P.dx, P.bc, P.gamma, P.small_p, P.ng)
    dt = oracle.dt(g, P.U, P.cfl) if P.nblk <= 4096 else 1e-4
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    nb = min(64, P.nblk)
    while True:
        blocks = np.arange(nb)
        t1 = time.perf_counter()
        oracle.step_blocks(g, P.U, blocks, dt)
        elapsed = time.perf_counter() - t1
        if elapsed >= seconds_target / 2 or nb == P.nblk:
            break
        nb = min(2 * nb, P.nblk)
    cells = nb * P.n ** 3
    return {"value": cells / elapsed, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"one step of the first {nb} of {P.nblk} blocks ({cells} cells), "
                      f"{elapsed:.2f} s on {cores} host threads"}


def traffic_from_profiles(kernel_tag):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source (else None)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_pmc.json")
    src = os.path.join(ROOT, "paper_2208_11630_amd", "csrc", "hydro_kernels.hip")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("kernel_source_sha256") != h:
        return None
    return rec.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="kh", choices=["kh", "sedov", "sod"])
    ap.add_argument("--cfl", type=float, default=0.8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="also run the streaming copy probe on this many GiB (roofline calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported by this build", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2208_11630_amd import hydro

    hydro.lib()
    torch.cuda.set_device(0)
    P, wname = make_workload(args.workload)
    print(f"[bench] workload {wname}: {P.cells} cells, {P.nblk} blocks", file=sys.stderr, flush=True)
    G = hydro.grid_for(P, device="cuda:0")
    stream = G.stream
    for _ in range(args.warmup):
        G.step_cfl(args.cfl)
    stream.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(args.steps):
        G.step_cfl(args.cfl)
    stop.record(stream)
    stop.synchronize()
    ms = start.elapsed_time(stop)
    ms_step = ms / args.steps
    rate = P.cells * args.steps / (ms * 1e-3)
    cnt = G.counters().tolist()
    print(f"[bench] {args.steps} steps in {ms:.3f} ms ({ms_step:.4f} ms/step), counters {cnt}",
          file=sys.stderr, flush=True)
    achieved = BYTES_PER_CELL * P.cells / (ms_step * 1e-3) / 1e9
    tag = f"step_kernel_nxb{P.n}_{args.workload}"
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_profiles(tag),
            "kernel": tag, "algorithmic_bytes_per_launch": BYTES_PER_CELL * P.cells}
    out = {
        "metric": "FP64 cell-updates/s",
        "value": rate,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wname, "cells": P.cells, "nxb": P.n, "blocks": P.nblk, "cfl": args.cfl,
                   "parallelism": "single-gpu"},
        "roofline": roof,
    }
    if args.copy_probe > 0:
        n = int(args.copy_probe * 2 ** 30) // 8
        src = torch.empty(n, dtype=torch.float64, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        hydro.copy_probe(src, dst, stream)
        stream.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(5):
            hydro.copy_probe(src, dst, stream)
        t1.record(stream)
        t1.synchronize()
        cms = t0.elapsed_time(t1) / 5
        out["copy_probe"] = {"bytes_read": 8 * n, "bytes_written": 8 * n, "ms": cms,
                             "GB/s": 16 * n / (cms * 1e-3) / 1e9}
        del src, dst
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(P, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
