"""The quality diagnostics of Sec. III (propagator, mode coupling, cross-
correlation) against closed forms: a field with itself, its negative and a
multiple; the normalisation by Parseval on a plane wave and white noise; and
the linear density of an analytic displacement."""
import numpy as np

from paper_1611_09638_amd import diagnostics as dg


def test_correlation_of_a_field_with_itself_and_multiples():
    n, box = 32, 200.0
    rng = np.random.default_rng(3)
    a = rng.normal(size=(n, n, n))
    p = dg.propagator(a, a, box, 8)
    assert np.allclose(p["r"], 1.0, atol=1e-12) and np.allclose(p["C"], 1.0, atol=1e-12)
    assert np.allclose(p["P_N"], 0.0, atol=1e-9 * p["P_L"].max())
    q = dg.propagator(-2.5 * a, a, box, 8)
    assert np.allclose(q["r"], -1.0, atol=1e-12) and np.allclose(q["C"], -2.5, atol=1e-12)
    # independent noise added: C unchanged in expectation, P_N = noise power
    b = rng.normal(size=(n, n, n))
    s = dg.propagator(a + b, a, box, 8)
    assert np.all(np.abs(s["C"][1:] - 1.0) < 0.1)
    assert np.all(np.abs(s["r"][1:] - 1 / np.sqrt(2)) < 0.07)


def test_power_normalisation():
    """A plane wave of amplitude A has variance A^2 / 2, all of it in the shell
    of its wavenumber; white noise of variance s^2 has flat power s^2 V / N."""
    n, box = 32, 100.0
    x = np.arange(n)
    a = 1.7 * np.cos(2 * np.pi * 3 * x / n)[:, None, None] * np.ones((1, n, n))
    k, pab, paa, pbb, modes = dg.binned_spectra(a, a, box, 16)
    total = np.nansum(paa * modes) / box ** 3
    assert abs(total - 1.7 ** 2 / 2) < 1e-12
    k0 = 2 * np.pi * 3 / box
    hit = np.nonzero(paa > 1e-12 * np.nanmax(paa))[0]
    edges = np.linspace(0.0, np.pi * n / box, 17)
    assert len(hit) == 1 and edges[hit[0]] <= k0 < edges[hit[0] + 1]
    rng = np.random.default_rng(4)
    w = 0.8 * rng.normal(size=(n, n, n))
    k, pab, paa, pbb, modes = dg.binned_spectra(w, w, box, 8)
    flat = 0.8 ** 2 * box ** 3 / n ** 3
    assert np.all(np.abs(paa[1:] / flat - 1) < 0.15)


def test_linear_density_of_an_analytic_displacement():
    """Psi = grad f for f = cos(2 pi (x + 2y)/n) / (2 pi / n)^2 (cells): the
    linear density -div Psi = -lap f = 5 cos(2 pi (x + 2y)/n)."""
    n = 32
    g = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    arg = 2 * np.pi * (g[0] + 2 * g[1]) / n
    kk = 2 * np.pi / n
    psi = np.stack([-np.sin(arg) / kk, -2 * np.sin(arg) / kk, np.zeros_like(arg)])
    assert np.abs(dg.linear_density(psi) - 5 * np.cos(arg)).max() < 1e-12
