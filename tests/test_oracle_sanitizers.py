"""The oracle built with AddressSanitizer and UBSan (every report fatal) runs
small forward solves in every mode, both reverse modes and the stage routines
cleanly, in a child process on the CPU (the ASan runtime has to be preloaded
there)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
sys.path.insert(0, %r)
import numpy as np
import oracle
from paper_1611_09638_amd import inputs
rho = inputs.lognormal_density(16, 125.0, 1.5, 7)
cfg = oracle.Config(max_outer=3, record_tape=1, tol=1e-12)
phi, d, st = oracle.solve(rho, 125.0, cfg)
g = oracle.backward(np.random.default_rng(1).normal(size=rho.shape), None, 125.0,
                    oracle.Config(max_outer=3, tol=1e-12))
pos = inputs.zeldovich_particles(16, 125.0, 0.8, 2)
grid = oracle.cic_particles(pos, 16, 125.0)
phi2, d2, st2 = oracle.solve(grid, 125.0, oracle.Config(max_outer=2, coarse_n=4))
a = oracle.normalize(rho)
r = np.random.default_rng(2).normal(size=rho.shape)
r -= r.mean()
z = oracle.vcycle(a, r)
# particles at their Lagrangian positions, with the exact-Jacobian solve and
# the mass update, and the reverse mode of the particle deposit
pos = inputs.zeldovich_particles(16, 32.0, 1.0, 3)
pcfg = dict(max_outer=2, tol=1e-12, particle_deposit=1)
oracle.solve_particles(pos, 16, 32.0, oracle.Config(record_tape=1, **pcfg))
gp = oracle.backward_particles(np.random.default_rng(3).normal(size=(16, 16, 16)), None, 32.0,
                               oracle.Config(**pcfg))
oracle.solve_particles(pos, 16, 32.0, oracle.Config(max_outer=2, particle_deposit=1, full_operator=1))
oracle.solve(rho, 125.0, oracle.Config(max_outer=2, mass_update=1, full_operator=1))
idx = np.array([0, 7, 4095])
fo = oracle.full_operator_at(phi / (125.0 / 16) ** 2, a, r, idx)
print("ok", st["outer_steps"], st2["outer_steps"], float(np.linalg.norm(g)), float(np.linalg.norm(z)),
      float(np.linalg.norm(gp)), float(np.linalg.norm(fo)))
""" % ROOT


def test_oracle_under_sanitizers(tmp_path):
    import oracle
    so = oracle.build_sanitized(str(tmp_path / "librecon_oracle_san.so"))
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan):
        pytest.skip("gcc has no ASan runtime")
    preload = asan + (":" + os.environ["LD_PRELOAD"] if os.environ.get("LD_PRELOAD") else "")
    env = dict(os.environ, RECON_ORACLE_LIB=so, LD_PRELOAD=preload, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    out = subprocess.run([sys.executable, "-c", SCRIPT], env=env, capture_output=True, text=True, timeout=900)
    assert out.returncode == 0, out.stderr[-4000:]
    assert "AddressSanitizer" not in out.stderr and "runtime error" not in out.stderr, out.stderr[-4000:]
    assert out.stdout.startswith("ok 3 2"), out.stdout
