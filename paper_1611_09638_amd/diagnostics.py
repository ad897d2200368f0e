"""Quality diagnostics of a reconstruction against a known linear field (Sec. III).

For a density field delta and the linear field delta_L:

* the propagator C(k) = P_{delta delta_L}(k) / P_{delta_L}(k);
* the mode-coupling power P_N(k) = P_delta(k) - C(k)^2 P_{delta_L}(k);
* the cross-correlation coefficient
  r(k) = P_{delta delta_L} / sqrt(P_delta P_{delta_L}) = 1 / sqrt(1 + P_N / (C^2 P_L)).

On synthetic Zel'dovich inputs the linear field is known exactly: the linear
density of the displacement, delta_L = -div Psi.

This is host-side analysis of outputs (numpy FFTs on the host); it is not
part of the reconstruction, which runs in the HIP library.
"""
import numpy as np


def _kmag(n: int, box: float):
    kx = 2.0 * np.pi * np.fft.fftfreq(n, d=box / n)
    kz = 2.0 * np.pi * np.fft.rfftfreq(n, d=box / n)
    return np.sqrt(kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2)


def _half_weights(n: int):
    """Modes each stored rFFT coefficient stands for (its conjugate twin too,
    except on the k_z = 0 and Nyquist planes; n even)."""
    w = np.full(n // 2 + 1, 2.0)
    w[0] = 1.0
    w[-1] = 1.0
    return w[None, None, :]


def linear_density(psi: np.ndarray) -> np.ndarray:
    """delta_L = -div Psi for a displacement Psi[3, n, n, n] in cells
    (spectral divergence; exact for the band-limited Zel'dovich field)."""
    n = psi.shape[1]
    kc = 2.0 * np.pi * np.fft.fftfreq(n)
    kcz = 2.0 * np.pi * np.fft.rfftfreq(n)
    comps = (kc[:, None, None], kc[None, :, None], kcz[None, None, :])
    div = sum(1j * comps[a] * np.fft.rfftn(psi[a]) for a in range(3))
    return -np.fft.irfftn(div, s=(n, n, n), axes=(0, 1, 2))


def binned_spectra(a: np.ndarray, b: np.ndarray, box: float, nbins: int = 16):
    """Auto and cross power in nbins linear shells from 0 to the Nyquist
    wavenumber: (k_mean, P_ab, P_aa, P_bb, modes), P in (length)^3 with
    P(k) = V |delta_k|^2 / N^2 (V = box^3, N = n^3), so that the power summed
    over modes and divided by V is the variance."""
    n = a.shape[0]
    A = np.fft.rfftn(a)
    B = np.fft.rfftn(b)
    k = _kmag(n, box)
    w = np.broadcast_to(_half_weights(n), k.shape)
    edges = np.linspace(0.0, np.pi * n / box, nbins + 1)
    idx = np.digitize(k, edges) - 1
    norm = box ** 3 / float(n) ** 6
    out = np.zeros((5, nbins))
    for i in range(nbins):
        m = (idx == i) & (k > 0)
        wm = w[m]
        W = wm.sum()
        if W == 0:
            out[:, i] = np.nan
            continue
        out[0, i] = (wm * k[m]).sum() / W
        out[1, i] = norm * (wm * (A[m] * np.conj(B[m])).real).sum() / W
        out[2, i] = norm * (wm * np.abs(A[m]) ** 2).sum() / W
        out[3, i] = norm * (wm * np.abs(B[m]) ** 2).sum() / W
        out[4, i] = W
    return out


def propagator(delta: np.ndarray, delta_L: np.ndarray, box: float, nbins: int = 16) -> dict:
    """k, C(k), r(k), P_N(k), P_L(k) and the mode count per shell (Sec. III)."""
    k, pab, paa, pll, modes = binned_spectra(delta, delta_L, box, nbins)
    C = pab / pll
    return dict(k=k, C=C, r=pab / np.sqrt(paa * pll), P_N=paa - C ** 2 * pll, P_L=pll, modes=modes)
