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


def _limiter_activity(phi, xi_m, v_m):
    """Nodes of the mesh of phi (grid units) with sqrt g = det e above v_m and
    with lambda_0 below xi_m, from numpy's determinant and eigenvalues of the
    compact-Hessian triad (independent of both solvers)."""
    e = np.empty(phi.shape + (3, 3))
    r = lambda f, a, d: np.roll(f, -d, axis=a)  # noqa: E731
    for a in range(3):
        e[..., a, a] = 1.0 + r(phi, a, 1) - 2 * phi + r(phi, a, -1)
        for b in range(a + 1, 3):
            e[..., a, b] = e[..., b, a] = 0.25 * (r(r(phi, a, 1), b, 1) - r(r(phi, a, 1), b, -1)
                                                  - r(r(phi, a, -1), b, 1) + r(r(phi, a, -1), b, -1))
    return int((np.linalg.det(e) > v_m).sum()), int((np.linalg.eigvalsh(e)[..., 0] < xi_m).sum())


@pytest.mark.parametrize("xi_m,v_m", [(0.2, 5.0), (0.05, 20.0)])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_limiter_constants_of_the_sweeps_against_oracle(orc, xi_m, v_m, precision):
    """App. B's limiter sweeps (xi_m in 1/5..1/20, v_m in 5..20) at their
    extreme settings, on a strongly nonlinear Zel'dovich input (64^3, cells of
    2.34 Mpc/h, rms displacement 3.5 cells): the GPU reconstruction against the
    oracle's with the same constants -- identical step sizes, phi and delta_r
    within 1e-6.  At xi_m = 1/5, v_m = 5 both limiters act on the final mesh."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_09638_amd import binding
    n, box = 64, 150.0
    pos = inputs.zeldovich_particles(n, box, 3.5, 31)
    rho = orc.cic_particles(pos, n, box)
    phi_o, d_o, st_o = orc.solve(rho, box, orc.Config(xi_m=xi_m, v_m=v_m))
    if v_m == 5.0:
        expand, compress = _limiter_activity(phi_o / (box / n) ** 2, xi_m, v_m)
        assert expand > 0 and compress > 0
    rec = binding.Recon(n, binding.Config(xi_m=xi_m, v_m=v_m, precision=precision))
    phi, d, st = rec.solve_particles(torch.from_numpy(pos).cuda(), box)
    phi, d = phi.cpu().numpy(), d.cpu().numpy()
    assert st["alpha"] == st_o["alpha"]
    assert np.linalg.norm(phi - phi_o) <= 1e-6 * np.linalg.norm(phi_o)
    assert np.linalg.norm(d - d_o) <= 1e-6 * np.linalg.norm(d_o)
    np.testing.assert_allclose(st["rms_sigma"], st_o["rms_sigma"], rtol=1e-6)
    if precision == 0:
        assert st["vcycles"] == st_o["vcycles"]
