"""The bench line's helpers without a GPU: the roofline object's fields and arithmetic, the
measured counters valid only at the kernel source they were taken at and for the
workload's own proposal, the workload description, and the refusal of several GPUs."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _m(own=True):
    # 10 launches of 1e9 executed particle-steps in 1 s of filter time each
    return dict(ms_pf=1000.0, executed=1e10, steps=10, own_proposal=own)


def test_roofline_fields_and_arithmetic():
    r = bench.roofline_of("age_seir", _m(), graph=0)
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel", "kernel_ms",
                "executed_particle_steps_per_launch", "algorithmic_ops_per_particle_step",
                "valu_lane_instr_per_particle_step", "valu_issue_frac", "valu_busy", "profile"):
        assert key in r, key
    algo = bench.ALGO_OPS_PER_PSTEP["age_seir"]
    assert r["achieved"] == pytest.approx(algo * 1e9 / 1e12)
    assert r["frac"] == pytest.approx(algo * 1e9 / bench.VALU_PEAK_LANE_OPS)
    assert r["peak"] == pytest.approx(bench.VALU_PEAK_LANE_OPS / 1e12)
    assert r["bound"] == "alu"


def test_measured_counters_follow_the_kernel_source_and_proposal():
    meas = bench.MEASURED["age_seir"]
    r = bench.roofline_of("age_seir", _m(), graph=0)
    valid = bench.kernel_sha() == meas["sha"]
    assert (r["traffic"] == meas["hbm_bytes_per_launch"]) == valid
    assert (r["valu_busy"] is not None) == valid
    assert os.path.exists(os.path.join(ROOT, meas["profile"]))
    # another proposal than the workload's own: the counters do not apply
    r2 = bench.roofline_of("age_seir", _m(own=False), graph=0)
    assert r2["traffic"] is None and r2["valu_busy"] is None and r2["frac"] == r["frac"]
    # a replayed graph has no per-kernel timing
    assert bench.roofline_of("age_seir", _m(), graph=1) is None


def test_committed_profiles_carry_the_measured_hash():
    for name, meas in bench.MEASURED.items():
        text = open(os.path.join(ROOT, meas["profile"])).read()
        assert meas["sha"] in text, name


def test_describe_names_the_proposal():
    w = dict(D=8, prec=0, proposal=1)
    runs = [dict(T=365, nx=2048)]
    d = bench.describe("age_seir", w, runs, 16384)
    assert "N=16384" in d and "Nx=2048" in d and "T=365" in d and "learned proposal" in d
    assert "population" in bench.describe("seir", dict(w, D=4, proposal=3), [dict(T=100, nx=512)], 1024)


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT)
    assert r.returncode == 2 and "one GPU" in r.stderr
