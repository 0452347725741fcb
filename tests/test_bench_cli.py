"""bench.py's command line on the CPU: one GPU only."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    """--gpus N with N > 1 ends with a message and a non-zero status before
    any device work."""
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU only" in (r.stdout + r.stderr)
    assert not r.stdout.strip().startswith("{")       # no result line


def test_counter_lookups_follow_the_committed_profiles():
    """The bench reads counter figures from profiles/kernel_counters.json only
    for the exact machine code (by hash); the batched kernel's profiled-build
    entry is found by block size and variant, every tuner candidate has one,
    and an unknown hash finds nothing."""
    sys.path.insert(0, ROOT)
    import json
    import bench
    d = json.load(open(os.path.join(ROOT, "profiles", "kernel_counters.json")))
    rk4 = [e for e in d["entries"] if e["workload"].startswith("mri_fast_stage rk4 64^3")][0]
    assert bench.counter_flops_per_unit(rk4["kernel_code_hash"]) == rk4["counter_fp64_flops_per_unit"]
    assert bench.counter_flops_per_unit("0" * 16) is None
    variants = {"built-in": {}, "one wave per SIMD": {"waves_per_simd": 1},
                "polynomial exponential": {"exp_table": 0},
                "scheduling window 1": {"sched_window": 1},
                "scheduling window 4": {"sched_window": 4}}
    for block in (64, 128, 256):
        for name, choice in variants.items():
            e = bench.batch_counters_profiled_build(block, dict(choice))
            assert e is not None and e["tile"][0] == block and e["variant"] == name
            assert e["counter_fp64_flops_per_unit"] > 0
