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
    key = "k_gemm_f32@lp_block200"
    assert key in rec
    r = rec[key]
    alg = r["algorithmic_bytes_per_launch"]
    if r["gemm_source_sha256"] == bm.gemm_source_digest():
        assert bm.traffic_of("k_gemm_f32", "lp_block200", alg) == r["bytes_per_launch"]
        assert bm.traffic_of("k_gemm_f32", "lp_block200", alg * 1.004) == r["bytes_per_launch"]
    else:
        assert bm.traffic_of("k_gemm_f32", "lp_block200", alg) is None
    # another launch mix, another workload or kernel: nothing is reported
    assert bm.traffic_of("k_gemm_f32", "lp_block200", alg * 1.01) is None
    assert bm.traffic_of("k_gemm_f32", "lp_block50", alg) is None
    assert bm.traffic_of("k_gemm_f64", "lp_block200", alg) is None


def test_traffic_record_is_consistent():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for key, r in rec.items():
        assert abs(r["fetch_bytes"] + r["write_bytes"] - r["bytes_per_launch"]) <= 1e-6 * r["bytes_per_launch"]
        # a plain copy calibrates the counters: reads count half, writes in full
        assert abs(r["fetch_scale"] - 2.0) < 0.01 and abs(r["write_scale"] - 1.0) < 0.01
        # traffic can exceed the algorithmic bytes (re-reads) but not fall far below them
        assert r["bytes_per_launch"] >= 0.9 * r["algorithmic_bytes_per_launch"]
