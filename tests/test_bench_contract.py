"""bench.py's command line contract, checked without a GPU: more than one GPU
is refused with a message (this build runs on one), and the helpers that do
not touch the device behave."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_cpu_model_is_a_string_or_none():
    sys.path.insert(0, ROOT)
    import bench
    m = bench.cpu_model()
    assert m is None or (isinstance(m, str) and m)
