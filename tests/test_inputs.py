"""The seeded input generators: statistics they promise, and the threaded
transforms used from 1024^3 up agreeing with numpy's."""
import numpy as np

from paper_1611_09638_amd import inputs


def test_threaded_transforms_match_numpy(monkeypatch):
    ref = inputs.zeldovich_displacement(16, 100.0, 1.5, 3)
    g_ref = inputs.gaussian_field(16, 100.0, 3)
    monkeypatch.setattr(inputs, "BIG", 8)
    psi = inputs.zeldovich_displacement(16, 100.0, 1.5, 3)
    g = inputs.gaussian_field(16, 100.0, 3)
    assert np.abs(g - g_ref).max() <= 1e-14 * np.abs(g_ref).max()
    assert np.abs(psi - ref).max() <= 1e-14 * np.abs(ref).max()


def test_generator_statistics():
    g = inputs.gaussian_field(32, 250.0, 1)
    assert abs(g.mean()) < 1e-15
    rho = inputs.lognormal_density(32, 250.0, 1.5, 2)
    assert abs(rho.mean() - 1.0) < 1e-14 and rho.min() > 0
    psi = inputs.zeldovich_displacement(32, 250.0, 0.8, 1)
    assert abs(np.sqrt(np.mean(np.sum(psi * psi, axis=0))) - 0.8) < 1e-12
    # Psi is a gradient field: its Fourier curl vanishes away from the
    # Nyquist planes (where a real field cannot hold i k delta)
    k = np.fft.fftfreq(32)
    P = [np.fft.fftn(p) for p in psi]
    curl_z = k[:, None, None] * P[1] - k[None, :, None] * P[0]
    inner = np.ones((32, 32, 32), bool)
    inner[16] = inner[:, 16] = inner[:, :, 16] = False
    assert np.abs(curl_z[inner]).max() < 1e-10 * np.abs(P[0]).max()
    pos = inputs.zeldovich_particles(32, 250.0, 0.8, 1)
    assert pos.shape == (32 ** 3, 3) and pos.dtype == np.float32
    assert pos.min() >= 0 and pos.max() < 250.0
