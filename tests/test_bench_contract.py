"""The benchmark's command-line contract that needs no GPU: several GPUs
are refused with a one-line JSON message and exit status 2."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_world_size_above_one_is_refused():
    env = dict(os.environ, WORLD_SIZE="2")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")], capture_output=True,
                       text=True, timeout=120, cwd=ROOT, env=env)
    assert r.returncode == 2


def test_golden_error_helper():
    """The benchmark's accuracy check on the oracle golden: zero error and no
    index mismatch for the golden's own values, and a planted power error and
    a planted index outside the near-tie set are reported."""
    import numpy as np
    import bench
    g = bench.load_golden()
    if g is None:
        return
    pm = np.zeros((g["k"].max() + 1, g["r"].max() + 1), np.float64)
    af = np.zeros(pm.shape, np.int32)
    pm[g["k"], g["r"]] = g["p"]
    af[g["k"], g["r"]] = g["f"]
    e, bad = bench.golden_error(pm, af, g)
    assert e == 0.0 and bad == 0
    pm[g["k"][5], g["r"][5]] += 3e-3 * g["pmax"]
    af[g["k"][7], g["r"][7]] = g["f"][7] + 5000
    e, bad = bench.golden_error(pm, af, g)
    assert abs(e - 3e-3) < 1e-9 and bad == 1
