"""Host logic of bench.py (CPU only): the one-GPU refusal and the roofline
arithmetic of the reported kernel."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_roofline_fields():
    met = {"launches": 4, "total_ms": 2.0, "flops": 4 * 3.0e10, "bytes": 4 * 1.0e9}
    r = bench.roofline(met, "not-the-profiled-workload", "learned")
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    assert abs(r["avg_launch_ms"] - 0.5) < 1e-12
    assert abs(r["achieved"] - 60.0) < 1e-9           # 3e10 flops per 0.5 ms
    assert abs(r["frac"] - 60.0 / 78.6) < 1e-12
    assert abs(r["achieved_algorithmic_GBs"] - 2000.0) < 1e-9
    assert r["traffic"] is None                      # counters were taken on another workload
    assert bench.roofline({"launches": 0, "total_ms": 0.0, "flops": 0.0, "bytes": 0.0}, "x", "learned") is None


def test_traffic_reported_only_for_the_profiled_sources():
    met = {"launches": 1, "total_ms": 1.0, "flops": 1.0e10, "bytes": 1.0e9}
    r = bench.roofline(met, bench.TRAFFIC["workload"], bench.TRAFFIC["form"])
    if bench.TRAFFIC["sha256"] == bench.source_hash():
        assert r["traffic"] == bench.TRAFFIC["bytes_per_launch"]
    else:
        assert r["traffic"] is None
    # the counters belong to one form's dispatches: another form on the same matrix gets none
    other = "plain_fp64" if bench.TRAFFIC["form"] == "learned" else "learned"
    assert bench.roofline(met, bench.TRAFFIC["workload"], other)["traffic"] is None


def test_cpu_baseline_pool_on_a_small_case():
    """The oracle baseline: a spawned pool of worker processes (single-threaded
    BLAS) over a size-stratified sample, extrapolated; every field reported."""
    import workloads as W
    cfg = W.config_c1()
    host = bench.cpu_baseline_host(cfg, cfg.part, reps=1, sample=4)
    out = bench.cpu_baseline_value(host, 17)
    assert out["kind"] == "oracle" and out["cores"] >= 1 and out["value"] > 0
    assert out["setup_s"] > 0 and out["solve_s"] > 0 and out["pcg_iterations_used"] == 17
    assert out["cpu_model"] and out["blas"] and "pool of" in out["sample"]


def test_pack_waves_one_kind_each_within_the_cap():
    sizes = [("a", 300), ("b", 50), ("a", 250), ("a", 600), ("b", 60), ("a", 100), ("b", 500)]
    waves = bench.pack_waves(sizes, ["a", "b"], {"a": 400, "b": 200})
    assert sorted(j for w in waves for j in w) == list(range(len(sizes)))   # every system once
    for w in waves:
        assert len({sizes[j][0] for j in w}) == 1                           # one kind per wave
        assert w == sorted(w)
        total = sum(sizes[j][1] for j in w)
        cap = 400 if sizes[w[0]][0] == "a" else 200
        assert total <= cap or len(w) == 1                                  # a larger system alone
    # first fit by decreasing size: 600 alone, then 300 + 100, then 250
    assert [sorted(sizes[j][1] for j in w) for w in waves if sizes[w[0]][0] == "a"] == [[600], [100, 300], [250]]
