"""The benchmark's host-side parts: more than one GPU is refused with a
message (the library runs on one GPU; sharding is designed, not built),
before anything touches a device; the batched oracle baseline's process
pool agrees with its serial run and with the oracle."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_help_lists_the_measurements():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--no-batched", "--no-served", "--no-heavy",
                 "--no-correlated", "--no-closed", "--copy-probe", "--path", "--workload"):
        assert flag in r.stdout, flag


def test_batched_cpu_baseline_pool_equals_serial():
    """The batched workload's oracle baseline (host only): the process pool
    and the serial run agree, on a small batch."""
    import argparse
    import numpy as np
    import bench
    from paper_1703_06680_amd import workloads as W
    r = bench.cpu_batched_baseline(argparse.Namespace(batch_count=24), W, np)
    assert r["instances"] == [0, 8, 16] and len(r["counts"]) == 3
    assert r["one_core"]["cores"] == 1 and r["all_cores"]["cores"] >= 1
    insts = W.batched_instances(24, d=2, seed=0)
    from oracle import oracle as O
    for b, k in zip(r["instances"], r["counts"]):
        t = insts[b]
        assert k == O.default().sbm(t.upd_lo, t.upd_hi, t.sub_lo, t.sub_hi, pairs=False,
                                    per_update=False)[0]
