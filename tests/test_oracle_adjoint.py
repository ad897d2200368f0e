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
