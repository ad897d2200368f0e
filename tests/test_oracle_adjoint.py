"""Pins of the oracle's reverse mode (the hand-written adjoint of the whole
reconstruction) against central finite differences of the oracle's own
forward, with every discrete decision (step sizes, limiter masks) unchanged
between the perturbed runs.  The finite differences difference the fields
before the (linear) loss, which avoids cancellation in L+ - L-.  CPU only."""
import numpy as np
import pytest

from paper_1611_09638_amd import inputs

N, BOX = 16, 125.0


def fd_check(orc, rho, base, voxels, tol, with_phi=True, seed=3):
    rng = np.random.default_rng(seed)
    gd = rng.normal(size=rho.shape)
    gp = rng.normal(size=rho.shape) * 1e-3 if with_phi else None
    phi, d, st = orc.solve(rho, BOX, orc.Config(record_tape=1, **base))
    g = orc.backward(gd, gp, BOX, orc.Config(**base))
    for idx in voxels:
        eps = 1e-6 * rho[idx]
        rp, rm = rho.copy(), rho.copy()
        rp[idx] += eps
        rm[idx] -= eps
        pp, dp, sp = orc.solve(rp, BOX, orc.Config(**base))
        pm, dm, sm = orc.solve(rm, BOX, orc.Config(**base))
        assert sp["alpha"] == st["alpha"] == sm["alpha"]
        fd = np.vdot(gd, dp - dm) / (2 * eps)
        if gp is not None:
            fd += np.vdot(gp, pp - pm) / (2 * eps)
        assert abs(fd - g[idx]) <= tol * abs(fd), (idx, g[idx], fd)
    return st, g


VOX = [(0, 0, 0), (3, 7, 11), (15, 2, 9), (8, 8, 8)]


def test_adjoint_compression_limiter_active(orc):
    rho = inputs.lognormal_density(N, BOX, 1.0, 7)
    st, g = fd_check(orc, rho, dict(max_outer=3, tol=1e-13, max_vcycles=200), VOX, 2e-5)
    assert st["min_lambda0"] < 0.1  # lambda_0 < xi_m somewhere: the eigenvector path is exercised


def test_adjoint_expansion_limiter_and_floor_active(orc):
    """v_m lowered so that the expansion limiter masks about 40% of the nodes;
    sigma_g = 2 puts mass below the coefficient floor a_min."""
    rho = inputs.lognormal_density(N, BOX, 2.0, 9)
    assert (rho / rho.mean()).min() < 1e-3
    fd_check(orc, rho, dict(max_outer=3, tol=1e-13, max_vcycles=300, v_m=1.05), VOX, 1e-4, with_phi=False, seed=4)


def test_adjoint_plain_vcycle_solver_and_zeldovich_input(orc):
    pos = inputs.zeldovich_particles(N, BOX, 0.8, 1)
    rho = orc.cic_particles(pos, N, BOX)
    fd_check(orc, rho, dict(max_outer=4, tol=1e-13, max_vcycles=300, solver=1), VOX[:3], 2e-5)


def test_adjoint_directional_derivative_over_all_voxels(orc):
    """<dL/drho, v> against (L(rho + eps v) - L(rho - eps v)) / 2 eps for a
    random direction v touching every voxel."""
    rho = inputs.lognormal_density(N, BOX, 1.2, 12)
    base = dict(max_outer=3, tol=1e-13, max_vcycles=200)
    rng = np.random.default_rng(12)
    gd = rng.normal(size=rho.shape)
    v = rng.normal(size=rho.shape) * rho
    phi, d, st = orc.solve(rho, BOX, orc.Config(record_tape=1, **base))
    g = orc.backward(gd, None, BOX, orc.Config(**base))
    eps = 1e-7
    _, dp, sp = orc.solve(rho + eps * v, BOX, orc.Config(**base))
    _, dm, sm = orc.solve(rho - eps * v, BOX, orc.Config(**base))
    assert sp["alpha"] == st["alpha"] == sm["alpha"]
    fd = np.vdot(gd, dp - dm) / (2 * eps)
    assert abs(fd - np.vdot(g, v)) <= 1e-5 * abs(fd)


def test_gradient_is_invariant_to_density_normalisation(orc):
    """The reconstruction sees only rho / mean(rho): the gradient is orthogonal
    to rho (scaling rho leaves the output unchanged) and scales as 1/c."""
    rho = inputs.lognormal_density(N, BOX, 1.0, 5)
    base = dict(max_outer=2, tol=1e-12, record_tape=1)
    gd = np.random.default_rng(5).normal(size=rho.shape)
    orc.solve(rho, BOX, orc.Config(**base))
    g1 = orc.backward(gd, None, BOX, orc.Config(**base))
    assert abs(np.vdot(g1, rho)) < 1e-10 * np.abs(g1).sum() * rho.mean()
    orc.solve(3.0 * rho, BOX, orc.Config(**base))
    g3 = orc.backward(gd, None, BOX, orc.Config(**base))
    np.testing.assert_allclose(g3, g1 / 3.0, rtol=1e-9, atol=1e-14)


def test_min_eigenvector_matches_lapack(orc):
    rng = np.random.default_rng(8)
    for _ in range(300):
        a = rng.normal(size=(3, 3))
        e = np.eye(3) + 0.4 * (a + a.T)
        lam, v = orc.eig_min_vec(e)
        w, V = np.linalg.eigh(e)
        assert abs(lam - w[0]) < 1e-12
        assert abs(abs(np.dot(v, V[:, 0])) - 1.0) < 1e-10
        np.testing.assert_allclose(e @ v, lam * v, atol=1e-11)


def test_backward_needs_a_tape(orc):
    orc.lib().orc_tape_clear()
    with pytest.raises(orc.OracleError) as e:
        orc.backward(np.zeros((8, 8, 8)), None, 10.0)
    assert e.value.code == -5


# ------------------- particles deposited at their Lagrangian positions

PBOX = 32.0  # positions below 32: a shift of 2^-10 is exact in float32


def particle_fd(orc, pos, base, gd, gp, idx, a, eps=2.0 ** -10):
    pp, pm = pos.copy(), pos.copy()
    pp[idx, a] += np.float32(eps)
    pm[idx, a] -= np.float32(eps)
    step = (float(pp[idx, a]) - float(pm[idx, a])) / 2
    php, dp, sp = orc.solve_particles(pp, N, PBOX, orc.Config(**base))
    phm, dm, sm = orc.solve_particles(pm, N, PBOX, orc.Config(**base))
    fd = np.vdot(gd, dp - dm) / (2 * step)
    if gp is not None:
        fd += np.vdot(gp, php - phm) / (2 * step)
    return fd, sp["alpha"], sm["alpha"]


@pytest.mark.parametrize("rms,seed", [(0.8, 1), (1.4, 2)])
def test_particle_adjoint_against_finite_differences(orc, rms, seed):
    """dL/d(position) through the inversion of the map and the xi-space
    deposit, for single particle coordinates, with the step sizes unchanged."""
    pos = inputs.zeldovich_particles(N, PBOX, rms, seed)
    base = dict(max_outer=3, tol=1e-13, max_vcycles=200, particle_deposit=1)
    rng = np.random.default_rng(20 + seed)
    gd = rng.normal(size=(N, N, N))
    gp = rng.normal(size=(N, N, N)) * 1e-3
    _, _, st = orc.solve_particles(pos, N, PBOX, orc.Config(record_tape=1, **base))
    g = orc.backward_particles(gd, gp, PBOX, orc.Config(**base))
    assert g.shape == pos.shape
    scale = np.abs(g).max()
    for idx in rng.choice(len(pos), 5, replace=False):
        for a in range(3):
            fd, ap, am = particle_fd(orc, pos, base, gd, gp, idx, a)
            assert ap == st["alpha"] == am
            assert abs(fd - g[idx, a]) <= 1e-5 * max(abs(fd), 0.05 * scale), (idx, a, fd, g[idx, a])


def test_particle_adjoint_directional_derivative(orc):
    """<dL/dpos, v> for a random direction v moving every particle, against
    central differences of the forward.  The CIC weights have a kink where a
    Lagrangian position crosses a cell face, and a crossing costs an error of
    the size of that particle's whole term; the amplitude (2^-18 of a box of
    32, about 2e-6 cells, so that most coordinates move by one or two float32
    units) keeps every particle inside its cells, and the sum over all
    particles must agree to rounding."""
    pos = inputs.zeldovich_particles(N, PBOX, 1.0, 3)
    base = dict(max_outer=3, tol=1e-13, max_vcycles=200, particle_deposit=1)
    rng = np.random.default_rng(31)
    gd = rng.normal(size=(N, N, N))
    _, _, st = orc.solve_particles(pos, N, PBOX, orc.Config(record_tape=1, **base))
    g = orc.backward_particles(gd, None, PBOX, orc.Config(**base))
    for seed in (1, 2):
        v = np.random.default_rng(seed).normal(size=pos.shape) * 2.0 ** -18
        pp = (pos + v).astype(np.float32)
        pm = (pos - v).astype(np.float32)
        _, dp, sp = orc.solve_particles(pp, N, PBOX, orc.Config(**base))
        _, dm, sm = orc.solve_particles(pm, N, PBOX, orc.Config(**base))
        assert sp["alpha"] == st["alpha"] == sm["alpha"]
        fd = np.vdot(gd, dp - dm)
        an = np.vdot(g, pp.astype(np.float64) - pm.astype(np.float64))
        assert abs(fd - an) <= 1e-6 * abs(fd)


def test_particle_backward_needs_a_particle_tape(orc):
    rho = inputs.lognormal_density(N, BOX, 0.5, 1)
    orc.solve(rho, BOX, orc.Config(record_tape=1, max_outer=1))
    with pytest.raises(orc.OracleError):
        orc.backward_particles(np.zeros((N, N, N)), None, PBOX)
