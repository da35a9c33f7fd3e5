"""The benchmark's contract on the CPU: it refuses several GPUs before any
device work, the committed counter record is the one of the current kernel
source (so the bench line's HBM traffic is not null), and the oracle leg
returns a well-formed baseline record on a small sample."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr
    assert not r.stdout.strip().startswith("{")


def test_committed_counter_record_matches_the_kernel_source():
    import bench

    rec = bench._profile_record("step_kernel_nxb16_kh")
    assert rec is not None, "profiles/step_kernel_nxb16_kh_pmc.json was taken on another kernel source"
    t = bench.traffic_from_profiles("step_kernel_nxb16_kh")
    algorithmic = bench.BYTES_PER_CELL * rec["cells_per_dispatch"]
    assert algorithmic <= t <= 2.0 * algorithmic
    v = bench.valu_roofline("step_kernel_nxb16_kh", 2.4e10)
    assert v["bound"] == "alu" and 0.0 < v["frac"] < 1.0
    assert v["valu_instr_per_cell"] == pytest.approx(64 * rec["valu_wave_instr_per_dispatch"] / rec["cells_per_dispatch"])


def test_cpu_baseline_record_on_a_small_sample():
    import bench
    from paper_2208_11630_amd import ics

    P = ics.sod(N=32, n=16)
    out = bench.cpu_baseline(P, seconds_target=0.2)
    assert out["kind"] == "oracle" and out["unit"] == "cell-updates/s"
    assert out["value"] > 0 and out["cores"] >= 1
    assert out["single_thread"]["value"] > 0
    assert "blocks" in out["sample"]
    json.dumps(out)
