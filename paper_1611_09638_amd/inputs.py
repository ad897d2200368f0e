"""Seeded synthetic inputs for the reconstruction.

This module holds only input generation: Gaussian random fields with the
stated spectral shape, lognormal densities, and Zel'dovich-displaced particle
positions.  It contains none of the reconstruction's arithmetic and is the only
code shared by the FP64 oracle's tests and the HIP path's tests and benchmark.

The paper reconstructs density grids made from N-body snapshots (Sec. III:
2048^3 particles in 600 Mpc/h gridded to 512^3; App. B: 1024^3 particles in
300 Mpc/h).  Those snapshots are not available, so seeded synthetic fields of
the same kind stand in for them:

* Gaussian field g: white N(0,1) noise from ``numpy.random.Generator(PCG64(seed))``
  of shape (n, n, n), multiplied in Fourier space by sqrt(P(k)) with
  P(k) = k / (1 + (k/0.02)^2)^2 (k in h/Mpc, k = 2 pi fftfreq(n, box/n)),
  P(0) = 0, transformed back and de-meaned.
* Lognormal density: g rescaled to sample standard deviation sigma_g,
  1 + delta = exp(g - sigma_g^2 / 2), then normalised to mean 1.
* Zel'dovich particles: one particle per lattice site q, displaced by
  Psi = IFFT(i k / k^2 * delta_hat), rescaled so that sqrt(<|Psi|^2>) equals the
  requested rms displacement in cells, positions wrapped into [0, box).

All arrays are C-order [i][j][k] (k fastest); positions are float32 (x, y, z)
in Mpc/h with x along the first array index.

Transforms are numpy's below 1024^3 and scipy's multithreaded ones from
1024^3 up (the same transforms; only the rounding of the input may differ).
"""
from __future__ import annotations

import os

import numpy as np

BIG = 1024  # grids of this edge and larger use threaded transforms


def _rfftn(x):
    if x.shape[0] >= BIG:
        import scipy.fft
        return scipy.fft.rfftn(x, workers=min(os.cpu_count() or 1, 16))
    return np.fft.rfftn(x)


def _irfftn(x, n):
    if n >= BIG:
        import scipy.fft
        return scipy.fft.irfftn(x, s=(n, n, n), axes=(0, 1, 2), workers=min(os.cpu_count() or 1, 16))
    return np.fft.irfftn(x, s=(n, n, n), axes=(0, 1, 2))

K_PEAK = 0.02  # h/Mpc, the turnover scale of the synthetic spectrum


def power_spectrum(k: np.ndarray) -> np.ndarray:
    """P(k) proportional to k / (1 + (k/0.02)^2)^2, with P(0) = 0."""
    k = np.asarray(k, dtype=np.float64)
    return k / (1.0 + (k / K_PEAK) ** 2) ** 2


def _kgrid(n: int, box: float):
    d = box / n
    kx = 2.0 * np.pi * np.fft.fftfreq(n, d=d)
    kz = 2.0 * np.pi * np.fft.rfftfreq(n, d=d)
    return kx, kz


def gaussian_field(n: int, box: float, seed: int) -> np.ndarray:
    """Zero-mean Gaussian random field with the synthetic spectrum shape (float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    white = rng.standard_normal((n, n, n))
    wk = _rfftn(white)
    del white
    kx, kz = _kgrid(n, box)
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    amp = np.sqrt(power_spectrum(np.sqrt(k2)))
    del k2
    wk *= amp
    del amp
    g = _irfftn(wk, n)
    del wk
    g -= g.mean()
    return g


def lognormal_density(n: int, box: float, sigma_g: float, seed: int) -> np.ndarray:
    """Lognormal density 1 + delta = exp(g - sigma_g^2/2), normalised to mean 1."""
    g = gaussian_field(n, box, seed)
    g *= sigma_g / g.std()
    g -= 0.5 * sigma_g * sigma_g
    np.exp(g, out=g)
    g /= g.mean()
    return g


def zeldovich_displacement(n: int, box: float, rms_cells: float, seed: int) -> np.ndarray:
    """Displacement Psi (shape (3, n, n, n), in cells) with sqrt(<|Psi|^2>) = rms_cells."""
    return displacement_from_field(gaussian_field(n, box, seed), box, rms_cells)


def displacement_from_field(g: np.ndarray, box: float, rms_cells: float) -> np.ndarray:
    """Psi = IFFT(i k / k^2 FFT(g)) rescaled to sqrt(<|Psi|^2>) = rms_cells (consumes g)."""
    n = g.shape[0]
    gk = _rfftn(g)
    del g
    kx, kz = _kgrid(n, box)
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    k2[0, 0, 0] = 1.0
    psi = np.empty((3, n, n, n), dtype=np.float64)
    comps = (kx[:, None, None], kx[None, :, None], kz[None, None, :])
    for a in range(3):
        psi[a] = _irfftn(1j * comps[a] / k2 * gk, n)
    rms = np.sqrt(np.mean(np.sum(psi * psi, axis=0)))
    psi *= rms_cells / rms
    return psi


def particles_from_displacement(psi: np.ndarray, box: float) -> np.ndarray:
    """Lattice sites q displaced by psi (cells), wrapped into [0, box); float32 [n^3, 3] in Mpc/h."""
    n = psi.shape[1]
    q = np.arange(n, dtype=np.float64)
    pos = np.empty((n, n, n, 3), dtype=np.float64)
    pos[..., 0] = q[:, None, None] + psi[0]
    pos[..., 1] = q[None, :, None] + psi[1]
    pos[..., 2] = q[None, None, :] + psi[2]
    pos *= box / n
    np.mod(pos, box, out=pos)
    out = pos.reshape(-1, 3).astype(np.float32)
    # float32 rounding can turn a value just below box into exactly box
    out[out >= np.float32(box)] = 0.0
    return out


def zeldovich_particles(n: int, box: float, rms_cells: float, seed: int) -> np.ndarray:
    """n^3 lattice particles displaced by a Zel'dovich field; float32 [n^3, 3] in Mpc/h."""
    return particles_from_displacement(zeldovich_displacement(n, box, rms_cells, seed), box)


# Workloads used by the tests and the benchmark: (n, box, kind, parameter, seed).
WORKLOADS = {
    "zeldovich32": dict(n=32, box=250.0, kind="particles", rms_cells=0.8, seed=1),
    "lognormal256": dict(n=256, box=1000.0, kind="lognormal", sigma_g=1.5, seed=2),
    "lognormal512": dict(n=512, box=1000.0, kind="lognormal", sigma_g=2.0, seed=3),
    "lognormal128": dict(n=128, box=500.0, kind="lognormal", sigma_g=1.5, seed=4),
    "zeldovich1024": dict(n=1024, box=2000.0, kind="particles", rms_cells=1.5, seed=5),
    # cells of 2.34 Mpc/h: the reconstruction takes full steps from the fourth on
    "zeldovich256": dict(n=256, box=600.0, kind="particles", rms_cells=1.5, seed=31),
    # milder field (cells of 15.6 Mpc/h): the paper's mass update converges on it
    "lognormal512_mild": dict(n=512, box=8000.0, kind="lognormal", sigma_g=0.5, seed=6),
}


def make_workload(name: str):
    """Return (kind, array, n, box) for a named workload."""
    w = WORKLOADS[name]
    if w["kind"] == "lognormal":
        return "density", lognormal_density(w["n"], w["box"], w["sigma_g"], w["seed"]), w["n"], w["box"]
    return "particles", zeldovich_particles(w["n"], w["box"], w["rms_cells"], w["seed"]), w["n"], w["box"]
