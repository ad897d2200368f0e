"""CPU-side checks of bench.py: the multi-GPU request is refused with a
message, and the oracle-only timing of the 32^3 configuration runs on the
host (no GPU) and reports the oracle's own V-cycle count."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_more_than_one_gpu_is_refused():
    cp = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=300)
    assert cp.returncode != 0
    assert "exactly one GPU" in cp.stderr


def test_oracle_timing_of_the_32_cube_configuration():
    env = dict(os.environ, OMP_NUM_THREADS="2")
    cp = subprocess.run([sys.executable, BENCH, "--configs-oracle", "cfg1"], capture_output=True, text=True,
                        timeout=600, env=env, check=True)
    res = json.loads(cp.stdout.strip().splitlines()[-1])["cfg1"]
    assert res["threads"] == 2 and res["forward_s"] > 0
    assert res["one_thread"]["threads"] == 1
    # 10 outer steps of the 32^3 Zel'dovich input, as the GPU solve takes them
    assert res["vcycles_total"] == res["one_thread"]["vcycles_total"] == 79
