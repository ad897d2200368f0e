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


A_MIN = 1e-3  # the default face floor, on the exact-Jacobian solve's diagonal fluxes too


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
    assert rel(orc.full_operator(phi, a, u, A_MIN), b) <= 2 * tol
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


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_full_operator_with_plain_vcycle_iteration(torch_cuda, orc, precision):
    """solver = V-cycle iteration u += V(b - L_K u) on the exact Jacobian."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    n, box = 32, 500.0
    rho = inputs.lognormal_density(n, box, 1.0, 7)
    phi_o, dr_o, st_o = orc.solve(rho, box, orc.Config(full_operator=1, solver=1, max_vcycles=300))
    rec = binding.Recon(n, binding.Config(precision=precision, full_operator=1, solver=1, max_vcycles=300))
    phi, dr, st = rec.solve(dev(torch, rho), box)
    assert st["alpha"] == st_o["alpha"]
    assert rel(host(phi), phi_o) < 1e-6
    assert rel(host(dr), dr_o) < 1e-6
    if precision == 0:
        assert st["vcycles"] == st_o["vcycles"]


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_full_operator_with_particle_deposit(torch_cuda, orc, precision):
    """Particles deposited at their Lagrangian positions and the exact-Jacobian
    solve together (32^3 Zel'dovich particles, rms 1.2 cells, where the exact
    Jacobian halves the mass deviation left after ten steps)."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    n, box = 32, 250.0
    pos = inputs.zeldovich_particles(n, box, 1.2, 7)
    cfg = dict(particle_deposit=1, full_operator=1)
    phi_o, dr_o, st_o = orc.solve_particles(pos, n, box, orc.Config(**cfg))
    rec = binding.Recon(n, binding.Config(precision=precision, **cfg))
    phi, dr, st = rec.solve_particles(dev(torch, pos), box)
    assert st["alpha"] == st_o["alpha"]
    assert rel(host(phi), phi_o) < 1e-6
    assert rel(host(dr), dr_o) < 1e-6
    assert st["rms_sigma"][-1] < 0.6 * orc.solve_particles(pos, n, box, orc.Config(particle_deposit=1))[2]["rms_sigma"][-1]
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


@pytest.mark.parametrize("n", [64, 128])
def test_full_residual_variants(torch_cuda, orc, n):
    """r = b - L_K u with r.r and its FP32 copy: the per-node gather and the
    streaming pass (several tiles and i-chunks, periodic wrap) against the
    oracle's operator."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    rec = binding.Recon(n, binding.Config(full_operator=1))
    a, phi, b = solve_inputs(n, 960 + n)
    u = np.random.default_rng(970 + n).normal(size=(n, n, n))
    ref = b - orc.full_operator(phi, a, u, A_MIN)
    args = [dev(torch, x) for x in (phi, a, u, b)]
    for variant in (1, 2):
        r, r32, rr = rec.full_residual(*args, variant=variant, fp32_copy=True)
        r = host(r)
        assert rel(r, ref) < 1e-13
        assert abs(rr - (r * r).sum()) < 1e-12 * rr
        assert np.array_equal(host(r32), r.astype(np.float32))


@pytest.mark.parametrize("n", [64, 128])
def test_full_direction_variants(torch_cuda, orc, n):
    """p_new = z + beta p_old, q = L_K p_new, p_new.q, and the deferred
    u += alpha_u p_old: both variants against the oracle's operator, FP64
    and FP32 directions."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    rec = binding.Recon(n, binding.Config(full_operator=1))
    a, phi, _ = solve_inputs(n, 980 + n)
    rng = np.random.default_rng(990 + n)
    z, p_old, u = (rng.normal(size=(n, n, n)) for _ in range(3))
    beta, alpha_u = 0.37, -0.81
    dphi, da = dev(torch, phi), dev(torch, a)
    for variant in (1, 2):
        # first step: p = z
        pn, q, pq = rec.full_direction(dphi, da, dev(torch, z), None, 0.0, first=True, variant=variant)
        assert np.array_equal(host(pn), z)
        q = host(q)
        assert rel(q, orc.full_operator(phi, a, z, A_MIN)) < 1e-13
        assert abs(pq - (z * q).sum()) < 1e-11 * abs(pq)
        # later step with the deferred solution update
        ud = dev(torch, u)
        pn, q, pq = rec.full_direction(dphi, da, dev(torch, z), dev(torch, p_old), beta, variant=variant,
                                       u=ud, alpha_u=alpha_u)
        pn, q = host(pn), host(q)
        assert rel(pn, z + beta * p_old) < 1e-15
        assert rel(q, orc.full_operator(phi, a, pn, A_MIN)) < 1e-13
        assert abs(pq - (pn * q).sum()) < 1e-11 * abs(pq)
        assert rel(host(ud), u + alpha_u * p_old) < 1e-15
    # FP32 z and directions (streaming only): p_new rounded as formed, q of the rounded values
    z32, p32 = z.astype(np.float32), p_old.astype(np.float32)
    pn, q, pq = rec.full_direction(dphi, da, dev(torch, z32), dev(torch, p32), beta, variant=2,
                                   p_dtype=torch.float32)
    pn, q = host(pn), host(q)
    assert pn.dtype == np.float32
    want = (z32.astype(np.float64) + beta * p32.astype(np.float64)).astype(np.float32)
    assert np.abs(pn.astype(np.float64) - want).max() <= 1.2e-7 * np.abs(want).max()
    assert rel(q, orc.full_operator(phi, a, pn.astype(np.float64), A_MIN)) < 1e-13


def test_full_solve_streaming_256(torch_cuda, orc):
    """At 256^3 the solve runs the streaming kernels: its solution satisfies the
    oracle's full operator equation to the solve's tolerance."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    n = 256
    a, phi, b = solve_inputs(n, 1000)
    assert orc.is_pd(phi)
    tol = 1e-10
    for precision in (0, 1):
        rec = binding.Recon(n, binding.Config(precision=precision, full_operator=1))
        u, cyc, r = rec.mg_solve_full(dev(torch, a), dev(torch, phi), dev(torch, b), tol=tol)
        u = host(u)
        assert r <= tol and cyc < 40
        assert rel(orc.full_operator(phi, a, u, A_MIN), b) <= 1.5 * tol
        del rec


def test_full_operator_floor_active(torch_cuda, orc):
    """A sigma_g = 2 lognormal whose mass falls below a_min: both kernels of the
    exact operator against the oracle's floored operator, and the first
    solve equal to the x ~ xi one (same operator at phi = 0); full
    reconstructions against the oracle, FP64 and mixed."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    n, box = 64, 250.0
    rho = inputs.lognormal_density(n, box, 2.0, 9)
    M = rho / rho.mean()
    assert M.min() < A_MIN
    rng = np.random.default_rng(64)
    g = inputs.gaussian_field(n, box, 65)
    phi = 0.3 * g / np.abs(g).max()
    u, b = rng.normal(size=(n, n, n)), rng.normal(size=(n, n, n))
    ref = b - orc.full_operator(phi, M, u, A_MIN)
    assert rel(ref, b - orc.full_operator(phi, M, u)) > 1e-8  # the floor is active
    rec = binding.Recon(n, binding.Config(full_operator=1))
    for variant in (1, 2):
        r, _, _ = rec.full_residual(dev(torch, phi), dev(torch, M), dev(torch, u), dev(torch, b), variant=variant)
        assert rel(host(r), ref) < 1e-13
    for precision in (0, 1):
        cfg = dict(max_vcycles=300, precision=precision)
        phi_o, dr_o, st_o = orc.solve(rho, box, orc.Config(full_operator=1, max_outer=4, max_vcycles=300))
        r1 = binding.Recon(n, binding.Config(full_operator=1, max_outer=4, **cfg))
        ph, dr, st = r1.solve(dev(torch, rho), box)
        assert st["alpha"] == st_o["alpha"]
        assert rel(host(ph), phi_o) < 1e-6 and rel(host(dr), dr_o) < 1e-6
        _, _, s0 = binding.Recon(n, binding.Config(max_outer=1, **cfg)).solve(dev(torch, rho), box)
        assert st["vcycles"][0] == s0["vcycles"][0]


def test_full_operator_config_errors(torch_cuda):
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    with pytest.raises(binding.ReconError):
        binding.Recon(32, binding.Config(full_operator=1, record_tape=1))
    rec = binding.Recon(32, binding.Config())
    f = torch.ones((32, 32, 32), dtype=torch.float64, device="cuda")
    with pytest.raises(binding.ReconError):
        rec.mg_solve_full(f, f, f)
    with pytest.raises(binding.ReconError):
        rec.full_residual(f, f, f, f)
    rec = binding.Recon(48, binding.Config(coarse_n=6, full_operator=1))
    g = torch.ones((48, 48, 48), dtype=torch.float64, device="cuda")
    with pytest.raises(binding.ReconError):  # streaming needs multiples of 64
        rec.full_residual(g, g, g, g, variant=2)
    z32 = torch.ones((48, 48, 48), dtype=torch.float32, device="cuda")
    with pytest.raises(binding.ReconError):  # FP32 directions need the streaming kernel
        rec.full_direction(g, g, z32, z32, 0.5, variant=1, p_dtype=torch.float32)
    with pytest.raises(binding.ReconError):  # u may not alias p_old or z
        rec.full_direction(g, g, g, g, 0.5, variant=1, u=g)


def test_full_operator_kernels_at_512(torch_cuda, orc):
    """The streaming exact-Jacobian kernels at 512^3, in the launch shape the
    solve uses there (8 x 64 tiles, 256-plane i-chunks), against the oracle's
    operator formed at 4096 sampled nodes (and the faces and corners of the
    periodic box): the residual with its norm, the direction pass in FP64
    and with FP32 directions, with the deferred solution update, and the mass
    update's unfloored application."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    n = 512
    w = inputs.WORKLOADS["lognormal512_mild"]
    rng = np.random.default_rng(5120)
    M = inputs.lognormal_density(n, w["box"], w["sigma_g"], w["seed"])
    M /= M.mean()
    g = inputs.gaussian_field(n, w["box"], 5121)
    phi = 0.3 * g / np.abs(g).max()
    del g
    idx = np.concatenate([[0, n - 1, n * n - 1, n ** 3 - 1, n ** 3 - n * n, (n // 2) * (n * n + n + 1)],
                          rng.choice(n ** 3, 4096, replace=False)])
    rec = binding.Recon(n, binding.Config(precision=binding.MIXED, full_operator=1))
    dphi, dM = dev(torch, phi), dev(torch, M)
    # residual r = b - L_K u with r.r and its FP32 copy
    u = rng.standard_normal((n, n, n))
    b = rng.standard_normal((n, n, n))
    r, r32, rr = rec.full_residual(dphi, dM, dev(torch, u), dev(torch, b), variant=2, fp32_copy=True)
    r = host(r)
    ref = b.ravel()[idx] - orc.full_operator_at(phi, M, u, idx, A_MIN)
    assert np.abs(r.ravel()[idx] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert abs(rr - float(np.dot(r.ravel(), r.ravel()))) <= 1e-10 * rr
    assert np.array_equal(host(r32).ravel()[idx], r.ravel()[idx].astype(np.float32))
    del r, r32, b
    # FP64 direction with the deferred update
    z = rng.standard_normal((n, n, n))
    p_old = rng.standard_normal((n, n, n))
    beta, alpha_u = 0.41, 0.73
    ud = dev(torch, u)
    pn, q, pq = rec.full_direction(dphi, dM, dev(torch, z), dev(torch, p_old), beta, variant=2, u=ud,
                                   alpha_u=alpha_u)
    pn, q = host(pn), host(q)
    p_ref = z + beta * p_old
    assert np.abs(pn - p_ref).max() <= 1e-15 * np.abs(p_ref).max()
    ref = orc.full_operator_at(phi, M, p_ref, idx, A_MIN)
    assert np.abs(q.ravel()[idx] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert abs(pq - float(np.dot(pn.ravel(), q.ravel()))) <= 1e-10 * abs(pq)
    assert np.abs(host(ud).ravel()[idx] - (u + alpha_u * p_old).ravel()[idx]).max() <= 1e-15 * np.abs(u).max() * 4
    del pn, q, ud
    # FP32 z and directions, as the mixed solve runs them
    z32, p32 = z.astype(np.float32), p_old.astype(np.float32)
    del z, p_old
    pn, q, pq = rec.full_direction(dphi, dM, dev(torch, z32), dev(torch, p32), beta, variant=2,
                                   p_dtype=torch.float32)
    pn = host(pn)
    p_ref = (z32.astype(np.float64) + beta * p32.astype(np.float64)).astype(np.float32)
    assert np.abs(pn.astype(np.float64) - p_ref).max() <= 1.2e-7 * np.abs(p_ref).max()
    ref = orc.full_operator_at(phi, M, pn.astype(np.float64), idx, A_MIN)
    assert np.abs(host(q).ravel()[idx] - ref).max() <= 1e-12 * np.abs(ref).max()
    del pn, q
    # the mass update's exact change (no floor), in its streaming pass
    f = rng.standard_normal((n, n, n))
    D = host(rec.mass_change(dphi, dM, dev(torch, f)))
    ref = orc.full_operator_at(phi, M, f, idx)
    assert np.abs(D.ravel()[idx] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert abs(D.sum()) < 1e-11 * np.abs(D).sum()
