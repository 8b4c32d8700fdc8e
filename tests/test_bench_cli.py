"""The benchmark's command line on the CPU: it refuses more than one GPU with a message
(before touching a device) and lists its workloads."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    res = _bench("--gpus", "2")
    assert res.returncode == 2
    line = json.loads(res.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_workloads_listed():
    res = _bench("--help")
    assert res.returncode == 0
    for name in ["paper_scale", "plain_fp64", "precision", "batched", "served", "table1",
                 "rows_first"]:
        assert name in res.stdout
