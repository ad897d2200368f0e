"""Write lognormal128_oracle_grad.json: the FP64 oracle's gradient of the
filtered-power loss for the 128^3 lognormal workload at 64 seeded voxels.

Calls only oracle/ and the seeded input generators.  Loss (unnormalised
forward DFT over all N^3 modes): L = sum_k W(k) |delta_r(k)|^2 with
W(k) = exp(-k^2 R^2), R = 10 Mpc/h, k = 2 pi fftfreq(N, box/N), so that
dL/d delta_r = 2 N^3 Re(ifftn(W fftn(delta_r))).  Run from the repository
root: python tests/golden/make_lognormal128_grad.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1611_09638_amd import inputs  # noqa: E402

R_SMOOTH = 10.0
N_VOX = 64
VOX_SEED = 44


def window(n, box):
    k = 2 * np.pi * np.fft.fftfreq(n, box / n)
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    return np.exp(-k2 * R_SMOOTH ** 2)


def loss_grad(delta, W):
    n = delta.shape[0]
    return 2.0 * n ** 3 * np.real(np.fft.ifftn(W * np.fft.fftn(delta)))


def main():
    w = inputs.WORKLOADS["lognormal128"]
    n, box = w["n"], w["box"]
    rho = inputs.lognormal_density(n, box, w["sigma_g"], w["seed"])
    cfg = oracle.Config(tol=1e-13, max_vcycles=400, record_tape=1)
    t0 = time.time()
    oracle.build(force=False)
    phi, delta, st = oracle.solve(rho, box, cfg)
    t1 = time.time()
    W = window(n, box)
    g = oracle.backward(loss_grad(delta, W), None, box, cfg)
    t2 = time.time()
    vox = np.random.default_rng(VOX_SEED).choice(n ** 3, N_VOX, replace=False)
    out = {
        "workload": "lognormal128", "n": n, "box": box, "sigma_g": w["sigma_g"], "seed": w["seed"],
        "R": R_SMOOTH, "vox_seed": VOX_SEED, "tol": cfg.tol, "max_outer": cfg.max_outer,
        "alpha": st["alpha"], "vcycles": st["vcycles"],
        "voxels": [int(v) for v in vox], "grad": [float(g.ravel()[v]) for v in vox],
        "grad_l2": float(np.linalg.norm(g)), "delta_l2": float(np.linalg.norm(delta)),
        "oracle_seconds": {"forward": round(t1 - t0, 1), "backward": round(t2 - t1, 1)},
        "generator": "tests/golden/make_lognormal128_grad.py (FP64 oracle, C + OpenMP)",
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lognormal128_oracle_grad.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, out["oracle_seconds"], flush=True)


if __name__ == "__main__":
    main()
