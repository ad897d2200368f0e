"""Particles deposited at their Lagrangian positions on the deformed mesh (the
literal "CIC on the deformed mesh" for particle input), on the GPU through
the C ABI, against the FP64 oracle: the Newton inversion of the continuous
map x = xi + trilinear(D_c phi), the xi-space CIC deposit, and full
reconstructions in that mode (identical steps, phi and delta_r within 1e-6,
mass exact)."""
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


def periodic_gap(a, b, n):
    d = a - b
    return np.abs(d - n * np.round(d / n)).max()


@pytest.mark.parametrize("n", [32, 48])
def test_inversion_and_deposit_against_oracle(torch_cuda, orc, n):
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    rec = binding.Recon(n, binding.Config(coarse_n=8 if n == 32 else 6))
    box = 250.0 * n / 32
    g = inputs.gaussian_field(n, box, 800 + n)
    phi = 0.4 * g / np.abs(g).max()
    assert orc.is_pd(phi)
    rng = np.random.default_rng(810 + n)
    pos = (rng.random((20000, 3)) * box).astype(np.float32)
    y = pos.astype(np.float64) * (n / box)
    xi_o = orc.invert_map(phi, y)
    xi, bad = rec.invert_map(dev(torch, phi), dev(torch, pos), box)
    assert bad == 0
    xi = xi.cpu().numpy()
    assert periodic_gap(xi, xi_o, n) < 1e-10
    assert xi.min() >= 0.0 and xi.max() < n
    M = rec.deposit_xi(dev(torch, xi)).cpu().numpy()
    M_o = orc.deposit_xi(xi, n)
    assert rel(M, M_o) < 1e-13
    assert abs(M.sum() - n ** 3) < 1e-9 * n ** 3
    # warm start from the solution: nothing to do, same answer
    xi2, bad = rec.invert_map(dev(torch, phi), dev(torch, pos), box, xi0=dev(torch, xi))
    assert bad == 0 and periodic_gap(xi2.cpu().numpy(), xi, n) < 1e-11
    # particles at the deformed-mesh nodes (float32 positions) deposit a uniform M
    nodes = np.stack(np.meshgrid(*(np.arange(n, dtype=float),) * 3, indexing="ij"), -1).reshape(-1, 3)
    shifts = np.stack([0.5 * (np.roll(phi, -1, a) - np.roll(phi, 1, a)) for a in range(3)], -1).reshape(-1, 3)
    pn = (np.mod(nodes + shifts, n) * (box / n)).astype(np.float32)
    pn[pn >= np.float32(box)] = 0.0
    xn, bad = rec.invert_map(dev(torch, phi), dev(torch, pn), box)
    assert bad == 0
    assert periodic_gap(xn.cpu().numpy(), nodes, n) < 1e-4
    Mn = rec.deposit_xi(xn).cpu().numpy()
    assert np.abs(Mn - 1.0).max() < 1e-3


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("n,box,rms", [(32, 250.0, 0.8), (64, 250.0, 1.2)])
def test_particle_deposit_solve_against_oracle(torch_cuda, orc, n, box, rms, precision):
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    pos = inputs.zeldovich_particles(n, box, rms, 820 + n)
    phi_o, dr_o, st_o = orc.solve_particles(pos, n, box, orc.Config(particle_deposit=1))
    rec = binding.Recon(n, binding.Config(precision=precision, particle_deposit=1))
    phi, dr, st = rec.solve_particles(dev(torch, pos), box)
    assert st["alpha"] == st_o["alpha"]
    assert rel(phi.cpu().numpy(), phi_o) < 1e-6
    assert rel(dr.cpu().numpy(), dr_o) < 1e-6
    assert all(abs(k - 1.0) < 1e-12 for k in st["kappa"])
    assert st["rms_sigma"][-1] < 0.3 * st["rms_sigma"][0]


def test_particle_deposit_needs_particles(torch_cuda):
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    rec = binding.Recon(32, binding.Config(particle_deposit=1))
    with pytest.raises(binding.ReconError):
        rec.solve(torch.ones((32, 32, 32), dtype=torch.float64, device="cuda"), 250.0)
    with pytest.raises(binding.ReconError):
        binding.Recon(32, binding.Config(particle_deposit=1, mass_update=1))


PCASES = [
    # n, box, rms displacement (cells), seed, precision, every k-th particle, extra config
    (16, 32.0, 1.0, 3, 0, 1, {}),
    (32, 250.0, 1.2, 5, 0, 1, {}),
    (32, 250.0, 1.2, 5, 1, 1, {}),
    (32, 250.0, 1.0, 6, 0, 3, {}),
    (48, 375.0, 1.0, 7, 1, 1, {"coarse_n": 6}),
    # FP32 tape: the backward linearises about phi rebuilt from the rounded u_i
    (32, 250.0, 1.2, 5, 1, 1, {"tape_fp32": 1}),
    # n^3 particles out of lattice order: the block-summed scatters fall back to memory
    (32, 250.0, 1.2, 5, 0, 1, {"shuffle": 1}),
]


@pytest.mark.parametrize("case", PCASES, ids=["16", "32", "32-mixed", "32-subsampled", "48-mixed", "32-fp32-tape", "32-shuffled"])
def test_particle_gradient_matches_oracle(torch_cuda, orc, case):
    """dL/d(positions) of a recorded particle-deposit forward, through the C
    ABI, against the oracle's reverse mode (itself pinned to finite
    differences)."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    n, box, rms, seed, prec, every, extra = case
    pos = np.ascontiguousarray(inputs.zeldovich_particles(n, box, rms, seed)[::every])
    extra = dict(extra)
    tape32 = extra.pop("tape_fp32", 0)
    if extra.pop("shuffle", 0):
        pos = np.ascontiguousarray(pos[np.random.default_rng(seed).permutation(len(pos))])
    base = dict(max_outer=3, tol=1e-13, max_vcycles=300, particle_deposit=1, **extra)
    rng = np.random.default_rng(seed)
    gd = rng.normal(size=(n, n, n))
    gp = rng.normal(size=(n, n, n)) * 1e-3
    _, _, st_o = orc.solve_particles(pos, n, box, orc.Config(record_tape=1, **base))
    g_o = orc.backward_particles(gd, gp, box, orc.Config(**base))
    rec = binding.Recon(n, binding.Config(record_tape=1, tape_fp32=tape32, precision=prec, **base))
    pd = dev(torch, pos)
    _, _, st = rec.solve_particles(pd, box)
    assert st["alpha"] == st_o["alpha"]
    g = rec.backward_particles(pd, dev(torch, gd), dev(torch, gp)).cpu().numpy()
    assert g.shape == pos.shape
    assert rel(g, g_o) < (1e-5 if tape32 else 1e-8), rel(g, g_o)
    # a second backward of the same tape gives the same gradient: its Newton
    # inversions start from other positions (the first step's, left by the
    # first backward) and stop within 1e-12 cells, and the atomic sums run in
    # another order
    g2 = rec.backward_particles(pd, dev(torch, gd), dev(torch, gp)).cpu().numpy()
    assert rel(g2, g) < 1e-10


def test_particle_backward_errors(torch_cuda):
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    n, box = 16, 32.0
    pos = dev(torch, inputs.zeldovich_particles(n, box, 1.0, 3))
    g = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    rec = binding.Recon(n, binding.Config(record_tape=1, particle_deposit=1, max_outer=2))
    with pytest.raises(binding.ReconError):  # no tape yet
        rec.backward_particles(pos, g)
    rec.solve_particles(pos, box)
    with pytest.raises(binding.ReconError):  # a particle tape has no density gradient
        rec.backward(g)
    with pytest.raises(binding.ReconError):  # other particles
        rec.backward_particles(pos[:-1].contiguous(), g)
    # the deposit keeps Lagrangian positions for at most n^3 particles
    many = torch.cat([pos, pos[:1]]).contiguous()
    with pytest.raises(binding.ReconError):
        binding.Recon(n, binding.Config(particle_deposit=1, max_outer=1)).solve_particles(many, box)
    dens = binding.Recon(n, binding.Config(record_tape=1, max_outer=2))
    dens.solve(1.0 + 0.1 * torch.rand((n, n, n), dtype=torch.float64, device="cuda"), box)
    with pytest.raises(binding.ReconError):  # a density tape has no particle gradient
        dens.backward_particles(pos, g)


def test_autograd_function_for_particles(torch_cuda):
    """ReconstructParticles.apply: the gradient reaching pos through autograd
    is recon_backward_particles's."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    n, box = 16, 32.0
    pos = dev(torch, inputs.zeldovich_particles(n, box, 1.0, 3)).requires_grad_(True)
    rec = binding.Recon(n, binding.Config(record_tape=1, particle_deposit=1, max_outer=3, tol=1e-13))
    w = torch.from_numpy(np.random.default_rng(4).normal(size=(n, n, n))).cuda()
    delta, phi = binding.ReconstructParticles.apply(pos, rec, box)
    loss = (w * delta).sum() + 1e-3 * (w * phi).sum()
    loss.backward()
    g_ref = rec.backward_particles(pos.detach(), w, 1e-3 * w)
    assert pos.grad.dtype == torch.float32
    assert torch.allclose(pos.grad.double(), g_ref, rtol=1e-6, atol=1e-7 * float(g_ref.abs().max()))


def test_inversion_and_deposit_at_512(torch_cuda, orc):
    """134M Zel'dovich particles at 512^3 (rms displacement 1.5 cells) on a
    deformed mesh, in the launch shape of the solve: every particle located
    (cold start from its Eulerian position), the Lagrangian positions against
    the oracle's own inversion, and the xi-space deposit against the oracle's
    deposit of its own positions."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    n, box = 512, 1000.0
    pos = inputs.zeldovich_particles(n, box, 1.5, 5130)
    g = inputs.gaussian_field(n, box, 5131)
    phi = 0.4 * g / np.abs(g).max()
    del g
    assert orc.is_pd(phi)
    rec = binding.Recon(n, binding.Config(precision=binding.MIXED, particle_deposit=1))
    xi, bad = rec.invert_map(dev(torch, phi), dev(torch, pos), box)
    assert bad == 0
    M = host(rec.deposit_xi(xi))
    xi = host(xi)
    del rec
    y = pos.astype(np.float64) * (n / box)
    del pos
    xi_o = orc.invert_map(phi, y)
    assert periodic_gap(xi, xi_o, n) < 1e-9
    del xi, y
    M_o = orc.deposit_xi(xi_o, n)
    assert rel(M, M_o) < 1e-12
    assert abs(M.sum() - n ** 3) < 1e-9 * n ** 3 and M.min() >= 0.0


def test_block_summed_deposit_any_order(torch_cuda, orc):
    """n^3 particles: the deposit summed per lattice block in LDS gives the
    oracle's deposit whether the particles are in lattice order (all through
    the windows) or shuffled (mostly straight to memory)."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    n, box = 32, 250.0
    pos = inputs.zeldovich_particles(n, box, 1.2, 7)
    g = inputs.gaussian_field(n, box, 3)
    phi = 0.4 * g / np.abs(g).max()
    xi = orc.invert_map(phi, pos.astype(np.float64) * (n / box))
    M_o = orc.deposit_xi(xi, n)
    rec = binding.Recon(n, binding.Config(particle_deposit=1))
    perm = np.random.default_rng(11).permutation(len(xi))
    for x in (xi, xi[perm]):
        M = host(rec.deposit_xi(dev(torch, x)))
        assert rel(M, M_o) < 1e-13
        assert abs(M.sum() - n ** 3) < 1e-9 * n ** 3
