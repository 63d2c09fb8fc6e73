"""The benchmark's command-line contract on a machine without a GPU: more
than one GPU is refused with a JSON message and exit status 2, and the
oracle baseline (the `cpu_baseline` leg) prints one JSON object with the
fields the benchmark line carries."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, timeout=300):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=timeout, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_cpu_baseline_line():
    r = _bench("--cpu-only", "--dcut", "4")
    assert r.returncode == 0, r.stderr
    b = json.loads(r.stdout.strip().splitlines()[-1])
    assert b["kind"] == "oracle" and b["unit"] == "RG-steps/s"
    assert b["value"] > 0 and b["cores"] >= 1 and b["extrapolated"] is True
    assert b["one_core"]["cores"] == 1 and b["one_core"]["value"] > 0
    assert "D=4" in b["sample"]
