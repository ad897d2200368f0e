"""The paper's measure of reconstruction quality (Sec. III) on stand-in data:
a Zel'dovich input (128^3 particles, 300 Mpc/h, rms displacement 1.5 cells),
whose linear density -div Psi is known exactly, reconstructed on the GPU
(mixed precision).  Against the nonlinear (CIC) density, the reconstruction
must raise the cross-correlation r(k) with the linear field in every shell,
strongly where the nonlinear field has decorrelated, and raise the
propagator C(k)."""
import numpy as np
import pytest

from paper_1611_09638_amd import diagnostics as dg
from paper_1611_09638_amd import inputs

pytestmark = pytest.mark.gpu


def test_reconstruction_recovers_the_linear_field():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_09638_amd import binding
    n, box = 128, 300.0
    psi = inputs.zeldovich_displacement(n, box, 1.5, 21)
    delta_L = dg.linear_density(psi)
    pos = torch.from_numpy(inputs.particles_from_displacement(psi, box)).cuda()
    rec = binding.Recon(n, binding.Config(precision=binding.MIXED))
    delta_nl = rec.cic(pos, box).cpu().numpy() - 1.0
    _, dr, st = rec.solve_particles(pos, box, want_phi=False)
    assert st["outer_steps"] == 10 and st["rms_sigma"][-1] < 0.05 * st["rms_sigma"][0]
    a = dg.propagator(delta_nl, delta_L, box, 16)
    b = dg.propagator(dr.cpu().numpy(), delta_L, box, 16)
    assert np.all(b["r"] >= a["r"] - 1e-3)
    assert np.all(b["C"] >= a["C"] - 1e-3)
    lost = a["r"] < 0.8
    assert lost.any() and np.all(b["r"][lost] - a["r"][lost] > 0.15)
    # where the nonlinear field keeps half its correlation, the reconstruction keeps 0.9
    assert np.all(b["r"][a["r"] >= 0.5] > 0.9)
