"""FP64 oracle of the standard periodic FFT potential solver -- TEST
INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU leg).

The usual approach the paper compares against (Sec. 1; results in Sec. 3.1,
Tables 1 and 4): truncate the problem to the periodic box [-L, L)^2 of the grid
and apply the multiplier of eq. (4) to the discrete Fourier coefficients,

    Phi_hat(k_m) = -kx^2 / |k|^2 rho_hat(k_m),   k_m = m / (N h), m in FFT order,

with Phi_hat(0) = 0 (the mean of the periodic potential is not determined; the
zero mode is dropped).  numpy's FFT serves as the DFT.
"""
from __future__ import annotations

import numpy as np

__all__ = ["periodic_multiplier", "phi_periodic"]


def periodic_multiplier(n: int, h: float, component: str = "xx") -> np.ndarray:
    """-kx^2/|k|^2 (or -ky^2/|k|^2) on the n x n Fourier grid of the box, 0 at k = 0;
    axis 1 is x."""
    k = np.fft.fftfreq(n, d=h)
    kx2 = (k ** 2)[None, :]
    ky2 = (k ** 2)[:, None]
    k2 = kx2 + ky2
    num = kx2 if component == "xx" else ky2
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(k2 > 0.0, -num / k2, 0.0)


def phi_periodic(rho: np.ndarray, h: float, component: str = "xx") -> np.ndarray:
    """Phi of the standard periodic FFT solver for the n x n density rho."""
    rho = np.asarray(rho, dtype=np.float64)
    mult = periodic_multiplier(rho.shape[0], h, component)
    return np.fft.ifft2(np.fft.fft2(rho) * mult).real
