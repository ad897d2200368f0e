"""The exact-Jacobian linear solve (App. A, Eq. elliptic_diff without the
x ~ xi approximation) on the GPU, through the C ABI, against the FP64 oracle:

* the solve div(a e^-1 grad u) = b alone (recon_stage_mg_solve_full): the same
  Krylov iterates, so the same iteration count in FP64, and the solution to the
  solve's tolerance, checked also by re-applying the oracle's full operator;
* full reconstructions with full_operator = 1, alone and with the mass update:
  identical step sizes, phi and delta_r within 1e-6 of the oracle.

Inputs are lognormal densities (sigma_g 1.0, and 0.5 with the mass update) at
a cell of 15.6 Mpc/h."""
import functools

import numpy as np
import pytest

from paper_1611_09638_amd import inputs

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def solve_inputs(n, seed):
    rng = np.random.default_rng(seed)
    a = np.exp(0.6 * rng.normal(size=(n, n, n))) + 0.05
    g = inputs.gaussian_field(n, 250.0 * n / 32, seed + 1)
    phi = 0.3 * g / np.abs(g).max()
    b = rng.normal(size=(n, n, n))
    return a, phi, b - b.mean()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("n,cn", [(32, 8), (48, 6), (64, 8)])
def test_full_solve_against_oracle(torch_cuda, orc, n, cn, precision):
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    a, phi, b = solve_inputs(n, 900 + n)
    assert orc.is_pd(phi)
    tol = 1e-11
    u_o, cyc_o, r_o = orc.mg_solve_full(a, phi, b, orc.Config(coarse_n=cn, tol=tol))
    rec = binding.Recon(n, binding.Config(coarse_n=cn, precision=precision, full_operator=1))
    u, cyc, r = rec.mg_solve_full(dev(torch, a), dev(torch, phi), dev(torch, b), tol=tol)
    u = host(u)
    assert r <= tol
    assert rel(orc.full_operator(phi, a, u), b) <= 2 * tol
    assert abs(u.mean()) < 1e-13 * np.abs(u).max()
    assert rel(u, u_o) < 1e-8
    if precision == 0:
        assert cyc == cyc_o
    # phi = 0: the x ~ xi solve of the same context
    u0, _, _ = rec.mg_solve_full(dev(torch, a), dev(torch, np.zeros_like(phi)), dev(torch, b), tol=tol)
    u1, _, _ = rec.mg_solve(dev(torch, a), dev(torch, b), tol=tol)
    assert rel(host(u0), host(u1)) < 1e-8


@functools.lru_cache(maxsize=None)
def oracle_solve(n, box, sigma, seed, cn, mass_update):
    import oracle
    rho = inputs.lognormal_density(n, box, sigma, seed)
    return rho, oracle.solve(rho, box, oracle.Config(coarse_n=cn, full_operator=1, mass_update=mass_update))


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("n,sigma,mass_update", [(32, 1.0, 0), (64, 1.0, 0), (32, 0.5, 1), (48, 0.5, 1)])
def test_full_operator_reconstruction_against_oracle(torch_cuda, n, sigma, mass_update, precision):
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    box = 500.0 * n / 32
    cn = 6 if n == 48 else 8
    rho, (phi_o, dr_o, st_o) = oracle_solve(n, box, sigma, 7, cn, mass_update)
    rec = binding.Recon(n, binding.Config(coarse_n=cn, precision=precision, full_operator=1,
                                          mass_update=mass_update))
    phi, dr, st = rec.solve(dev(torch, rho), box)
    assert st["alpha"] == st_o["alpha"]
    assert rel(host(phi), phi_o) < 1e-6
    assert rel(host(dr), dr_o) < 1e-6
    assert np.allclose(st["kappa"], st_o["kappa"], rtol=1e-7, atol=0)
    if mass_update:  # carried mass: conserved exactly
        assert all(abs(k - 1.0) < 1e-12 for k in st["kappa"])
    assert st["min_det"] > 0 and st["min_lambda0"] > 0
    if precision == 0:
        assert st["vcycles"] == st_o["vcycles"]


def test_full_operator_improves_on_x_approx_xi(torch_cuda):
    """On a 64^3 sigma_g = 1 lognormal the exact-Jacobian mode leaves less mass
    deviation after ten steps than the x ~ xi mode (both on the GPU)."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    n, box = 64, 1000.0
    rho = dev(torch, inputs.lognormal_density(n, box, 1.0, 7))
    _, _, st0 = binding.Recon(n, binding.Config(precision=1)).solve(rho, box)
    _, _, st1 = binding.Recon(n, binding.Config(precision=1, full_operator=1)).solve(rho, box)
    assert st1["rms_sigma"][-1] < st0["rms_sigma"][-1]


def test_full_operator_config_errors(torch_cuda):
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    with pytest.raises(binding.ReconError):
        binding.Recon(32, binding.Config(full_operator=1, record_tape=1))
    rec = binding.Recon(32, binding.Config())
    f = torch.ones((32, 32, 32), dtype=torch.float64, device="cuda")
    with pytest.raises(binding.ReconError):
        rec.mg_solve_full(f, f, f)
