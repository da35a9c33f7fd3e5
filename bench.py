"""Benchmark: FP64 cell-updates/s of the unsplit Godunov hydro step on MI355X.

One "step" is one pass of the whole hot path over the grid: the CFL dt formed
on the device from the signal speed the previous step reduced, the fused
guard fill + primitive recovery + PLM/van Leer + Hancock predictor + HLLC
x/y/z + conservative update, and the signal-speed reduction of the new state
(one kernel launch per step).  The default workload is the 512 x 512 x 256
Kelvin-Helmholtz grid (16^3 blocks, 67.1M cells).  Inputs are resident in
HBM before the timed region starts.

Prints one JSON line (see the fields below).  --gpus N > 1 is refused: the
path runs on one GPU (no multi-GPU exchange is implemented).
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
# SSP Runge-Kutta steps: the first stage reads U and writes U1 (80 B); every
# later stage reads its input and the base state and writes its result (120 B)
RK_BYTES_PER_CELL = {"rk2": 80.0 + 120.0, "rk3": 80.0 + 2 * 120.0}


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
    same workload, on the host cores: one step of the first nb blocks of the
    grid, nb doubling until one timing takes at least half the target (or
    covers the grid), whole-grid steps repeated up to the target; then the
    same on one thread, on a sample of a few seconds."""
    import platform

    import numpy as np

    import oracle

    g = oracle.Grid(P.n, P.nb, P.dx, P.bc, P.gamma, P.small_p, P.ng)
    dt = oracle.dt(g, P.U, P.cfl) if P.nblk <= 4096 else 1e-4
    cores = oracle.lib().oracle_max_threads()

    def timed_sample(target):
        nb = min(64, P.nblk)
        while True:
            blocks = np.arange(nb)
            t1 = time.perf_counter()
            oracle.step_blocks(g, P.U, blocks, dt)
            elapsed = time.perf_counter() - t1
            if elapsed >= target / 2 or nb == P.nblk:
                break
            nb = min(2 * nb, P.nblk)
        reps = 1
        while elapsed < target * 2 / 3 and nb == P.nblk:   # the whole grid: repeat the step
            t1 = time.perf_counter()
            oracle.step_blocks(g, P.U, np.arange(nb), dt)
            elapsed += time.perf_counter() - t1
            reps += 1
        return nb, reps, elapsed

    nb, reps, elapsed = timed_sample(seconds_target)
    cells = nb * P.n ** 3 * reps
    prev = oracle.set_threads(1)
    nb1, reps1, el1 = timed_sample(4.0)
    oracle.set_threads(prev)
    cells1 = nb1 * P.n ** 3 * reps1
    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": cells / elapsed, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{reps} step(s) of the first {nb} of {P.nblk} blocks ({cells} cell updates), "
                      f"{elapsed:.2f} s on {cores} host threads",
            "single_thread": {"value": cells1 / el1, "unit": "cell-updates/s",
                              "sample": f"{reps1} step(s) of the first {nb1} blocks, {el1:.2f} s on 1 thread"},
            "cpu_model": model, "host_cpus": os.cpu_count()}


# FP64 VALU issue: 256 CUs x 4 SIMDs, one wave64 FP64 instruction per SIMD
# every 4 cycles (16 lanes), 2.4 GHz -> 6.144e11 wave instructions/s (with
# 2 flops per FMA lane this is the published 78.6 TFLOP/s); transcendental
# FP64 instructions (rcp, rsq) take four such slots.
VALU_PEAK_SLOTS = 256 * 4 * 2.4e9 / 4


def valu_roofline(kernel_tag, cells_per_s):
    """Issue-slot roofline of the step from the committed instruction counts
    (rocprofv3 SQ counters of the same kernel source), or None."""
    rec = _profile_record(kernel_tag)
    if not rec or "valu_wave_instr_per_dispatch" not in rec:
        return None
    per_cell = rec["valu_wave_instr_per_dispatch"] / rec["cells_per_dispatch"]          # wave instr per cell
    trans = rec["valu_trans_f64_wave_instr_per_dispatch"] / rec["cells_per_dispatch"]
    slots = per_cell + 3.0 * trans
    achieved = cells_per_s * slots
    return {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_SLOTS, "unit": "wave64 VALU issue slots/s",
            "frac": achieved / VALU_PEAK_SLOTS, "valu_instr_per_cell": per_cell * 64,
            "fp64_trans_instr_per_cell": trans * 64}


def _profile_record(kernel_tag):
    import hashlib

    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_pmc.json")
    src = os.path.join(ROOT, "paper_2208_11630_amd", "csrc", "hydro_kernels.hip")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return rec


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


def run_ensemble(args, cpu=True):
    """Batched ensemble: independent periodic simulations with 1-64 blocks of
    8^3, 16^3 or 32^3 cells.  Times the same steps two ways on the same GPU:
    looping the plain per-grid step over the members, and the batch (one
    persistent launch per step, captured as a HIP graph, launch shape from
    the autotuner).  value = batched cell-updates/s."""
    import torch

    from paper_2208_11630_amd import hydro, ics, tune

    sims = ics.ensemble(count=args.members, seed=2, steps=50)
    cells = sum(P.cells for P in sims)
    print(f"[bench] ensemble: {len(sims)} members, {cells} cells", file=sys.stderr, flush=True)
    grids = [hydro.grid_for(P, device="cuda:0") for P in sims]
    st = torch.cuda.current_stream()

    def timed(run, stream, k):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(k):
            run()
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b)

    # looped plain step: one launch per member per step
    def loop_step():
        for G in grids:
            G.step_cfl(args.cfl)
    for _ in range(args.warmup):
        loop_step()
    st.synchronize()
    ms_loop = timed(loop_step, st, args.steps)
    print(f"[bench] looped: {ms_loop / args.steps:.3f} ms/step", file=sys.stderr, flush=True)

    B = hydro.Batch(grids)
    cfg = {"pencils": [1, 1, 1], "per_cu": 2}
    if not args.no_tune:
        cfg = tune.tune_batch(B, args.cfl)
        print(f"[bench] tuned: pencils {cfg['pencils']} workgroups/CU {cfg['per_cu']} tiles {cfg.get('tiles')}",
              file=sys.stderr,
              flush=True)
    B.use_graph(True)
    B.step(args.cfl, 6 * max(1, args.warmup // 6 + 1))
    B.synchronize()
    k = 6 * max(1, round(args.steps / 6))
    ms_batch = timed(lambda: B.step(args.cfl, 6), B.stream, k // 6)
    print(f"[bench] batched: {ms_batch / k:.3f} ms/step", file=sys.stderr, flush=True)
    loop_rate = cells * args.steps / (ms_loop * 1e-3)
    rate = cells * k / (ms_batch * 1e-3)
    ms_step = ms_batch / k
    achieved = BYTES_PER_CELL * cells / (ms_step * 1e-3) / 1e9
    out = {
        "metric": "FP64 cell-updates/s",
        "value": rate,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": k,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batched_ensemble_{len(sims)}_members_nxb8_16_32", "cells": cells,
                   "members": len(sims), "cfl": args.cfl, "launch": "persistent+hipgraph",
                   "pencils": cfg["pencils"], "workgroups_per_cu": cfg["per_cu"],
                   "tiles": cfg.get("tiles", [8, 16, 16]),
                   "parallelism": "single-gpu"},
        "looped_plain_step": {"value": loop_rate, "ms_per_step": ms_loop / args.steps,
                              "launches_per_step": len(sims)},
        "batched_over_looped": rate / loop_rate,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "batch_step_kernel (one launch per block size per step)",
                     "algorithmic_bytes_per_step": BYTES_PER_CELL * cells},
    }
    if cpu and not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        big = max(sims, key=lambda P: P.cells)
        out["cpu_baseline"] = cpu_baseline(big, args.cpu_seconds)
    B.close()
    del B, grids, sims
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def run_amr(args):
    """Block-structured AMR: the Kelvin-Helmholtz shear layer on a 256 x 256
    x 128 root grid of 16^3 blocks, the block rows at the two interfaces
    refined once (fine cells 1/512; workload amr3: the level-1 rows holding
    an interface refined again).  A step: dt from the CFL rule over every
    level formed on the device (the signal speed the previous step
    reduced), views with guards (same level, prolongation), the step of
    every leaf, refluxing and restriction.  value = leaf cell-updates/s.
    One estimate and one regrid are timed after the steps."""
    import numpy as np
    import torch

    from paper_2208_11630_amd import hydro, ics

    n = 16
    if args.workload == "amr3":
        nb, flags, flags1, Ur, Uf, dx, gamma = ics.kelvin_helmholtz_amr3(root=(256, 256, 128), n=n)
        deep = flags1.tolist() + [False] * (8 * int(flags1.sum()))
        nleaf = int((~flags).sum()) + int((~flags1).sum()) + 8 * int(flags1.sum())
        wname = "amr_kelvin_helmholtz_root256x256x128_nxb16_three_levels"
    else:
        nb, flags, Ur, Uf, dx, gamma = ics.kelvin_helmholtz_amr(root=(256, 256, 128), n=n)
        deep = []
        nleaf = int((~flags).sum()) + Uf.shape[0]
        wname = "amr_kelvin_helmholtz_root256x256x128_nxb16_two_levels"
    cells = nleaf * n ** 3
    print(f"[bench] {args.workload}: {flags.size} root blocks, {int(flags.sum())} refined, {nleaf} leaves, "
          f"{cells} leaf cells", file=sys.stderr, flush=True)
    hi = tuple(nb[d] * n * dx[d] for d in range(3))
    A = hydro.Amr(n, nb, flags.tolist(), hi=hi, gamma=gamma, refine_deep=deep)
    A.upload(Ur, Uf)
    del Ur, Uf

    def one():
        A.step_cfl(args.cfl)
    for _ in range(args.warmup):
        one()
    A.stream.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(A.stream)
    for _ in range(args.steps):
        one()
    t1.record(A.stream)
    t1.synchronize()
    ms = t0.elapsed_time(t1)
    ms_step = ms / args.steps
    rate = cells * args.steps / (ms * 1e-3)
    cnt = A.counters().tolist()
    print(f"[bench] {args.steps} steps in {ms:.3f} ms ({ms_step:.4f} ms/step), counters {cnt}", file=sys.stderr,
          flush=True)
    achieved = BYTES_PER_CELL * cells / (ms_step * 1e-3) / 1e9
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
        "config": {"workload": wname, "cells": cells, "levels": len(A.level_blocks),
                   "blocks_per_level": A.level_blocks, "leaf_blocks": nleaf,
                   "cfl": args.cfl, "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "amr_tile_kernel",
                     "algorithmic_bytes_per_step": BYTES_PER_CELL * cells},
    }
    # adaptivity, timed apart from the steps: one estimate (indicator kernel,
    # values read back, the rule on the host) and one regrid to its flags
    # (new mesh: allocation, tables, transfer of the state)
    A.stream.synchronize()
    before = list(A.level_blocks)
    t = time.perf_counter()
    if len(before) > 2:
        flags_new, deep_new, _ = A.estimate_tree(eps=0.01, refine_cutoff=0.8, derefine_cutoff=0.2,
                                                 max_levels=len(before))
    else:
        flags_new, _ = A.estimate(eps=0.01, refine_cutoff=0.8, derefine_cutoff=0.2)
        deep_new = []
    est_ms = (time.perf_counter() - t) * 1e3
    t = time.perf_counter()
    B = A.regrid(flags_new, deep_new)
    B.stream.synchronize()
    regrid_ms = (time.perf_counter() - t) * 1e3
    out["adapt"] = {"estimate_ms": est_ms, "regrid_ms": regrid_ms,
                    "blocks_per_level_before": before, "blocks_per_level_after": list(B.level_blocks),
                    "note": "host wall time; regrid includes allocating the new mesh"}
    print(f"[bench] estimate {est_ms:.2f} ms, regrid {regrid_ms:.2f} ms "
          f"(blocks per level {before} -> {list(B.level_blocks)})", file=sys.stderr, flush=True)
    B.close()
    print(json.dumps(out), flush=True)


def run_served(args):
    """Served stream: many resident cubic simulations (L log-uniform in
    32..256, 16^3 blocks, random initial states), one-step requests with
    uniform targets.  Residency is bounded by an HBM budget (one 40 B/cell
    state buffer per resident simulation, outputs lent per launch; LRU
    eviction to host memory).  Measures the saturated request rate (all
    requests queued at t=0), then sweeps Poisson arrival rates from 10% to
    120% of it, reporting p50/p99 request latency and cell-updates/s; the
    same saturated stream without batching (one simulation per launch) is the
    looped baseline.  value = saturated served cell-updates/s."""
    import numpy as np
    import torch

    from paper_2208_11630_amd import ics, serve

    sizes = ics.served_sizes(args.served_sims, seed=3)
    cells_total = sum(L ** 3 for L in sizes)
    budget = int(args.served_budget_gb * 1e9)
    max_cells = 300_000_000                     # outputs lent per launch: <= 12 GB
    ex = serve.GpuExecutor(sizes, cfl=args.cfl)
    srv = serve.Server(ex, budget - 2 * 40 * max_cells, max_inflight=2, max_cells_per_launch=max_cells)
    print(f"[bench] served: {len(sizes)} simulations, {cells_total} cells ({40 * cells_total / 1e9:.0f} GB "
          f"per copy), budget {budget / 1e9:.0f} GB", file=sys.stderr, flush=True)
    # warm-up: fill the budget with simulations in random order (first touch draws them on the device)
    rng = np.random.default_rng(5)
    srv.stats = serve.Stats()
    for sim in rng.permutation(len(sizes)):
        if srv.used + ex.bytes_of(int(sim)) > srv.budget:
            continue
        srv._admit(int(sim), set())
    torch.cuda.synchronize()
    resident = len(srv.lru)
    # pin host memory for the evicted part of the population up front (server start-up)
    ex.pool.reserve(max(0, 40 * cells_total - srv.budget) + (8 << 30))
    print(f"[bench] warm: {resident} resident, {srv.used / 1e9:.1f} GB", file=sys.stderr, flush=True)

    snapshot = list(srv.lru)   # every measured run starts from the residency after warm-up

    def trace_run(arr, max_cells_launch, inflight):
        srv.restore(snapshot)
        torch.cuda.synchronize()
        srv.max_cells = max_cells_launch
        srv.max_inflight = inflight
        ex.host_s.clear()
        ex.moved.clear()
        st = srv.run(arr)
        torch.cuda.synchronize()
        out = st.summary()
        out["executor_host_s"] = {k: round(v, 4) for k, v in ex.host_s.items()}
        out["host_GB"] = {k: round(v / 1e9, 2) for k, v in ex.moved.items()}
        return out

    def burst(nreq, seed, targets=None):
        r = np.random.default_rng(seed)
        pick = r.integers(0, len(sizes), size=nreq) if targets is None else r.choice(targets, size=nreq)
        return [(0.0, int(x)) for x in pick]

    keys = ("completed", "requests_per_s", "cell_updates_per_s", "p50_ms", "p99_ms", "mean_batch",
            "launches", "evictions", "admissions", "wall_s", "executor_host_s", "host_GB")
    pick = lambda st: {k: st.get(k) for k in keys}

    # host-link ceiling: a request for a simulation that is not resident
    # moves its state host -> device and an evicted one device -> host
    link = host_link(ex, srv, sizes, cells_total)
    print(f"[bench] host link: {link}", file=sys.stderr, flush=True)

    # saturated throughput: the same 2000 requests at t = 0, batched
    # (continuous batching, 2 launches in flight) and looped (one simulation
    # per launch, one launch in flight)
    arr_sat = burst(2000, 7)
    # one untimed pass of the burst first: the pinned staging pool grows and
    # each simulation's grid handle is created on first touch, costs a
    # server in steady state has paid and that would otherwise fall on
    # whichever timed run came first
    trace_run(arr_sat, max_cells, 2)
    sat = trace_run(arr_sat, max_cells, 2)
    print(f"[bench] saturated batched: {pick(sat)}", file=sys.stderr, flush=True)
    sat_loop = trace_run(arr_sat, 1, 1)
    print(f"[bench] saturated looped: {pick(sat_loop)}", file=sys.stderr, flush=True)
    # the burst's own link bound: the bytes its admissions and evictions
    # moved (the larger direction; both run at once) at the measured rate.
    # Requests for one simulation share its admission, so this is below the
    # per-request miss model of `link` for a burst.
    gb = sat["host_GB"]
    sat_link_s = max(gb.get("in", 0.0), gb.get("out", 0.0)) / link["h2d_and_d2h_GB_per_s_each_way"]

    def ramp(burst_rate, fractions, targets, seed):
        """Poisson arrivals at a rising offered rate until the achieved rate
        falls below 90% of the offered one (the server no longer keeps up),
        then the same trace of the highest rate batching kept up with, served
        looped."""
        rows = []
        for frac in fractions:
            arr = serve.poisson_arrivals(frac * burst_rate, args.served_seconds, len(sizes), seed=seed)
            if targets is not None:
                arr = [(t, int(targets[x % len(targets)])) for t, x in arr]
            st = trace_run(arr, max_cells, 2)
            row = {"offered_per_s": len(arr) / args.served_seconds, **pick(st)}
            rows.append(row)
            print(f"[bench] offered {row['offered_per_s']:.0f}/s: {pick(st)}", file=sys.stderr, flush=True)
            if st["requests_per_s"] < 0.9 * row["offered_per_s"]:
                break
        kept = [r for r in rows if r["requests_per_s"] >= 0.9 * r["offered_per_s"]] or rows[:1]
        k = rows.index(kept[-1])
        arr = serve.poisson_arrivals(fractions[k] * burst_rate, args.served_seconds, len(sizes), seed=seed)
        if targets is not None:
            arr = [(t, int(targets[x % len(targets)])) for t, x in arr]
        loop = pick(trace_run(arr, 1, 1))
        print(f"[bench] same trace looped: {loop}", file=sys.stderr, flush=True)
        return rows, {"offered_per_s": kept[-1]["offered_per_s"], "batched": kept[-1],
                      "looped_one_sim_per_launch": loop}

    sweep, same = ramp(sat["requests_per_s"], (0.2, 0.35, 0.5, 0.65, 0.8, 1.0), None, 4)

    # the same comparisons without host traffic: requests for the resident
    # simulations only (targets uniform over the residency after warm-up)
    resident_now = np.array(snapshot)
    arr_res = burst(2000, 9, resident_now)
    res_b = trace_run(arr_res, max_cells, 2)
    res_l = trace_run(arr_res, 1, 1)
    print(f"[bench] resident-only batched: {pick(res_b)}", file=sys.stderr, flush=True)
    print(f"[bench] resident-only looped: {pick(res_l)}", file=sys.stderr, flush=True)
    res_sweep, res_same = ramp(res_b["requests_per_s"], (0.1, 0.2, 0.35, 0.5, 0.65, 0.8, 1.0), resident_now, 6)
    batched_pts = [r for r in sweep if (r.get("mean_batch") or 0) > 1.0]
    out = {
        "metric": "FP64 cell-updates/s; p50/p99 latency of served step requests",
        "value": sat["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": sat["completed"],
        "warmup": resident,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"served_stream_{len(sizes)}_sims_L32-256_nxb16", "cells": cells_total,
                   "budget_GB": budget / 1e9, "resident_after_warmup": resident,
                   "resident_fraction_of_cells": link["resident_fraction_of_cells"], "cfl": args.cfl,
                   "parallelism": "single-gpu"},
        "host_link": link,
        "saturated": {"batched": pick(sat), "looped_one_sim_per_launch": pick(sat_loop),
                      "batched_over_looped": sat["cell_updates_per_s"] / max(sat_loop["cell_updates_per_s"], 1e-30),
                      "link_seconds_of_batched_copies": sat_link_s,
                      "batched_wall_over_link_seconds": sat["wall_s"] / max(sat_link_s, 1e-30),
                      "trace": "the same 2000 requests at t = 0, uniform targets (seed 7)"},
        "latency_sweep": sweep,
        "latency_points_with_mean_batch_above_1": len(batched_pts),
        "same_trace": same,
        "resident_only": {"batched": pick(res_b), "looped_one_sim_per_launch": pick(res_l),
                          "batched_over_looped": res_b["cell_updates_per_s"] /
                          max(res_l["cell_updates_per_s"], 1e-30),
                          "trace": "the same 2000 requests at t = 0 for resident simulations (seed 9)",
                          "latency_sweep": res_sweep,
                          "latency_points_with_mean_batch_above_1":
                              len([r for r in res_sweep if (r.get("mean_batch") or 0) > 1.0]),
                          "same_trace": res_same},
    }
    ex.close()
    del srv, ex
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def host_link(ex, srv, sizes, cells_total):
    """Measured pinned host <-> device copy rates (both directions at once, on
    the executor's two copy streams) and the request rate they allow: with
    uniform targets a request misses the device with probability equal to the
    non-resident fraction of the simulations, and a miss moves one state in
    and one out (40 B per cell each way)."""
    import numpy as np
    import torch

    nbytes = 2 << 30
    h_in = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    h_out = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    d_in = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    d_out = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(2):
        with torch.cuda.stream(ex.copy_stream):
            d_in.copy_(h_in, non_blocking=True)
        with torch.cuda.stream(ex.evict_stream):
            h_out.copy_(d_out, non_blocking=True)
    ex.copy_stream.synchronize()
    ex.evict_stream.synchronize()
    el = time.perf_counter() - t
    del h_in, h_out, d_in, d_out
    gbs = 2 * nbytes / el / 1e9                      # each direction
    resident = set(srv.lru)
    miss = 1.0 - len(resident) / len(sizes)
    mean_cells_missed = float(np.mean([sizes[s] ** 3 for s in range(len(sizes)) if s not in resident] or [0]))
    bytes_per_request = miss * 40.0 * mean_cells_missed  # each way
    mean_cells = cells_total / len(sizes)
    ceiling_req = gbs * 1e9 / bytes_per_request if bytes_per_request > 0 else float("inf")
    return {"h2d_and_d2h_GB_per_s_each_way": gbs, "nonresident_fraction_of_sims": miss,
            "resident_fraction_of_cells": sum(sizes[s] ** 3 for s in resident) / cells_total,
            "ceiling_requests_per_s": ceiling_req, "ceiling_cell_updates_per_s": ceiling_req * mean_cells,
            "note": "uniform targets: a request misses the device with the non-resident fraction of the "
                    "simulations; a miss copies one state in and one out"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="kh", choices=["kh", "sedov", "sod", "ensemble", "served", "amr", "amr3"])
    ap.add_argument("--served-sims", type=int, default=2000)
    ap.add_argument("--served-budget-gb", type=float, default=200.0)
    ap.add_argument("--served-seconds", type=float, default=1.5, help="served: seconds per rate point")
    ap.add_argument("--members", type=int, default=512, help="ensemble: number of simulations")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (default launch shape)")
    ap.add_argument("--cfl", type=float, default=0.8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload: skip the Sod/Sedov, batched-ensemble and served-stream legs")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--scheme", default="mh", choices=["mh", "rk2", "rk3", "ctu", "ctu_char"],
                    help="grid workloads: predictor-corrector step (default) or SSP Runge-Kutta steps")
    ap.add_argument("--copy-probe", type=float, default=1.0,
                    help="streaming copy probe on this many GiB: the achievable HBM bandwidth, reported "
                         "beside the roofline and used to calibrate the traffic counters (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the path has no multi-GPU exchange)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2208_11630_amd import hydro

    hydro.lib()
    torch.cuda.set_device(0)
    if args.workload == "ensemble":
        print(json.dumps(run_ensemble(args)), flush=True)
        return
    if args.workload == "served":
        print(json.dumps(run_served(args)), flush=True)
        return
    if args.workload in ("amr", "amr3"):
        return run_amr(args)
    P, wname = make_workload(args.workload)
    print(f"[bench] workload {wname}: {P.cells} cells, {P.nblk} blocks", file=sys.stderr, flush=True)
    G = hydro.grid_for(P, device="cuda:0")
    if args.scheme != "mh":
        G.set_scheme({"rk2": hydro.SCHEME_RK2, "rk3": hydro.SCHEME_RK3, "ctu": hydro.SCHEME_CTU,
                      "ctu_char": hydro.SCHEME_CTU_CHAR}[args.scheme])
    planes = P.n
    if not args.no_tune and not args.scheme.startswith("ctu"):
        from paper_2208_11630_amd import tune

        planes = tune.tune_grid(G, args.cfl)
        print(f"[bench] tuned: {planes} planes per z pencil, {G.tile}x{G.tile} tiles", file=sys.stderr, flush=True)
    bpc = BYTES_PER_CELL if args.scheme in ("mh", "ctu", "ctu_char") else RK_BYTES_PER_CELL[args.scheme]
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
    achieved = bpc * P.cells / (ms_step * 1e-3) / 1e9
    if args.scheme == "mh":
        tag = f"step_kernel_nxb{P.n}_{args.workload}"
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_profiles(tag),
                "kernel": tag, "algorithmic_bytes_per_launch": BYTES_PER_CELL * P.cells}
        alu = valu_roofline(tag, rate) if args.workload == "kh" else None
    elif args.scheme.startswith("ctu"):  # launches per chunk of blocks: bytes and time per step
        tag = f"ctu_kernel_nxb{P.n}_{args.workload}" + ("_char" if args.scheme == "ctu_char" else "")
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": tag,
                "algorithmic_bytes_per_step": bpc * P.cells}
    else:  # several stage launches per step: bytes and time are per step
        tag = f"stage_kernel_nxb{P.n}_{args.workload}_{args.scheme}"
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": tag,
                "algorithmic_bytes_per_step": bpc * P.cells,
                "launches_per_step": 2 if args.scheme == "rk2" else 3}
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
                   "scheme": {"mh": "predictor-corrector", "rk2": "ssp-rk2", "rk3": "ssp-rk3",
                              "ctu": "corner-transport-upwind",
                              "ctu_char": "corner-transport-upwind-characteristic"}[args.scheme],
                   "pencil_planes": planes, "tile": f"{G.tile}x{G.tile}",
                   "parallelism": "single-gpu"},
        "roofline": roof,
    }
    if args.scheme == "mh" and alu:
        out["alu_roofline"] = alu
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
        gbs = 16 * n / (cms * 1e-3) / 1e9
        out["copy_probe"] = {"bytes_read": 8 * n, "bytes_written": 8 * n, "ms": cms, "GB/s": gbs,
                             "frac_of_peak": gbs / HBM_PEAK_GBS,
                             "step_over_copy": out["roofline"]["achieved"] / gbs}
        del src, dst
    if not args.no_cpu_baseline and args.scheme == "mh":
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(P, args.cpu_seconds)
    if args.workload == "kh" and args.scheme == "mh" and not args.no_extras:
        del G
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        out.update(extras(args))
    print(json.dumps(out), flush=True)


def plain_rate(P, wname, args):
    """Plain-step rate of one configuration (device dt, tuned pencils)."""
    import torch

    from paper_2208_11630_amd import hydro, tune

    G = hydro.grid_for(P, device="cuda:0")
    planes = P.n if args.no_tune else tune.tune_grid(G, args.cfl)
    for _ in range(args.warmup):
        G.step_cfl(args.cfl)
    G.stream.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(G.stream)
    for _ in range(args.steps):
        G.step_cfl(args.cfl)
    b.record(G.stream)
    b.synchronize()
    ms = a.elapsed_time(b) / args.steps
    rate = P.cells / (ms * 1e-3)
    print(f"[bench] {wname}: {ms:.4f} ms/step, {rate:.3e} cell-updates/s", file=sys.stderr, flush=True)
    gbs = BYTES_PER_CELL * rate / 1e9
    return {"cells": P.cells, "ms_per_step": ms, "cell_updates_per_s": rate, "pencil_planes": planes,
            "tile": f"{G.tile}x{G.tile}",
            "algorithmic_GB_per_s": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS,
            "counters": G.counters().tolist()}


def extras(args):
    """The other configurations, measured in the same run: the Sod and Sedov
    grids (plain step), the batched ensemble (batched vs looped on the same
    members) and the served stream (p50/p99 latency under Poisson load,
    batched vs looped on the same traces, host-link ceiling)."""
    import torch

    from paper_2208_11630_amd import ics

    out = {"other_workloads": {}}
    for name, P, w in ((("sod"), ics.sod(), "sod_64^3_nxb16"), ("sedov", ics.sedov(), "sedov_256^3_nxb16")):
        out["other_workloads"][name] = {"workload": w, **plain_rate(P, w, args)}
        if not args.no_cpu_baseline:
            out["other_workloads"][name]["cpu_oracle"] = cpu_baseline(P, 4.0)
        del P
        torch.cuda.empty_cache()
    e = run_ensemble(args, cpu=False)
    out["batched_ensemble"] = {"workload": e["config"]["workload"], "cells": e["config"]["cells"],
                               "batched": {"ms_per_step": e["ms_per_step"], "cell_updates_per_s": e["value"],
                                           "launch": e["config"]["launch"], "pencils": e["config"]["pencils"],
                                           "tiles": e["config"]["tiles"],
                                           "workgroups_per_cu": e["config"]["workgroups_per_cu"]},
                               "looped_plain_step": e["looped_plain_step"],
                               "batched_over_looped": e["batched_over_looped"],
                               "roofline_frac": e["roofline"]["frac"]}
    v = run_served(args)
    out["served_stream"] = {k: v[k] for k in ("config", "host_link", "saturated", "latency_sweep",
                                              "latency_points_with_mean_batch_above_1", "same_trace",
                                              "resident_only")}
    return out


if __name__ == "__main__":
    main()
