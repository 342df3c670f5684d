"""Host logic of bench.py (no GPU): the multi-GPU refusal and the rule that
reports measured HBM traffic only for the GEMM source and launch mix the
counters were taken on."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_record_applies_only_to_its_source_and_launch_mix():
    bm = _bench()
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    key = "k_gemm_f32@lp_block200_dual"
    assert key in rec
    r = rec[key]
    alg = r["algorithmic_bytes_per_launch"]
    if r["gemm_source_sha256"] == bm.gemm_source_digest():
        assert bm.traffic_of("k_gemm_f32", "lp_block200_dual", alg) == r["bytes_per_launch"]
        assert bm.traffic_of("k_gemm_f32", "lp_block200_dual", alg * 1.004) == r["bytes_per_launch"]
    else:
        assert bm.traffic_of("k_gemm_f32", "lp_block200_dual", alg) is None
    # another launch mix, another workload or kernel: nothing is reported
    assert bm.traffic_of("k_gemm_f32", "lp_block200_dual", alg * 1.01) is None
    assert bm.traffic_of("k_gemm_f32", "lp_block50_dual", alg) is None
    assert bm.traffic_of("k_gemm_f64", "lp_block200_dual", alg) is None
    assert bm.traffic_of("k_gemm_f32", "lp_block200_primal", alg) is None
    # the FP64 GEMM's record, under the same rules
    r64 = rec["k_gemm_f64@lp_block200_dual"]
    alg64 = r64["algorithmic_bytes_per_launch"]
    if r64["gemm_source_sha256"] == bm.gemm_source_digest():
        assert bm.traffic_of("k_gemm_f64", "lp_block200_dual", alg64) == r64["bytes_per_launch"]
    assert bm.traffic_of("k_gemm_f64", "lp_block200_dual", alg64 * 0.99) is None


def test_traffic_record_is_consistent():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for key, r in rec.items():
        assert abs(r["fetch_bytes"] + r["write_bytes"] - r["bytes_per_launch"]) <= 1e-6 * r["bytes_per_launch"]
        # a plain copy calibrates the counters: reads count half, writes in full
        assert abs(r["fetch_scale"] - 2.0) < 0.01 and abs(r["write_scale"] - 1.0) < 0.01
        # traffic can exceed the algorithmic bytes (re-reads) but not fall far below them
        assert r["bytes_per_launch"] >= 0.9 * r["algorithmic_bytes_per_launch"]


def _simulate(bm, requested, t_solve, t_before, budget, compare=True, others=True):
    """Wall time of the bench's step loop with solves of t_solve seconds
    after t_before seconds of set-up and one warmup solve, then the FP64
    solve on the same handle (1.2 t) and the other condensed system (set-up
    plus an FP32 and an FP64 solve, 2.2 t and 3.2 t: the primal system's
    times when the dual one is timed)."""
    now = t_before + t_solve          # set-up, then the (single) warmup
    t_step, done = t_solve, 0
    reserve = (1.5 * t_step if compare else 0.0) + (7.0 * t_step + 15.0 if others else 0.0)
    while done < max(1, requested) and bm.plan_steps(done, now, t_step, reserve, budget):
        now += t_solve
        done += 1
    if compare:
        now += 1.2 * t_solve
    if others:
        now += 10.0 + 2.2 * t_solve + 3.2 * t_solve
    return done, now


def test_driver_command_fits_its_time_limit():
    """--steps 20 --warmup 5 with the dual system's 12 s solve (the primal's
    takes 25 s) and about 60 s of start-up (torch import, generation,
    analysis, CPU baseline): the JSON line comes well before 600 s."""
    bm = _bench()
    for t in (12.0, 25.0, 40.0):
        done, wall = _simulate(bm, 20, t, 60.0, 450.0)
        assert 1 <= done <= 20
        assert wall <= 540.0, (t, wall)
    # a slower solve still runs one timed step
    done, wall = _simulate(bm, 20, 150.0, 60.0, 450.0, others=False)
    assert done == 1
    # small workloads run every requested step
    done, _ = _simulate(bm, 20, 0.02, 10.0, 450.0)
    assert done == 20


def test_first_step_always_runs_and_budget_is_respected():
    bm = _bench()
    assert bm.plan_steps(0, 1e9, 10.0, 0.0, 100.0)
    assert bm.plan_steps(1, 50.0, 10.0, 20.0, 100.0)
    assert not bm.plan_steps(1, 75.0, 10.0, 20.0, 100.0)


def test_cpu_baseline_scaling_and_host_record():
    bm = _bench()
    smp = {"what": "x", "seconds": 10.0, "iterations": 10, "flops": 1e9, "status": "optimal"}
    r = bm.cpu_baseline_scale(smp, 1e12, 20)
    # 1 s per iteration at 1e9 flops -> 1000 s per iteration at 1e12, 20 iterations
    assert abs(1.0 / r["value"] - 20000.0) < 1e-6
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["estimate"] is True
    assert r["host"]["nproc"] >= 1 and isinstance(r["host"]["model"], str)
