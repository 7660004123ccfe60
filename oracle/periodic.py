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
    """-kx^2/|k|^2 (or -ky^2/|k|^2, or -kx ky/|k|^2) on the n x n Fourier grid of
    the box, 0 at k = 0; axis 1 is x.  The mixed multiplier is odd in each of kx,
    ky; on the Nyquist lines (index n/2) one DFT bin stands for +k and -k, and
    the bin takes the mean of the multiplier over them, 0 (also at the corner)."""
    k = np.fft.fftfreq(n, d=h)
    kx = k[None, :]
    ky = k[:, None]
    k2 = kx * kx + ky * ky
    num = {"xx": kx * kx + 0.0 * ky, "yy": ky * ky + 0.0 * kx, "xy": kx * ky}[component]
    with np.errstate(divide="ignore", invalid="ignore"):
        mult = np.where(k2 > 0.0, -num / k2, 0.0)
    if component == "xy":
        mult[n // 2, :] = 0.0
        mult[:, n // 2] = 0.0
    return mult


def phi_periodic(rho: np.ndarray, h: float, component: str = "xx") -> np.ndarray:
    """Phi of the standard periodic FFT solver for the n x n density rho."""
    rho = np.asarray(rho, dtype=np.float64)
    mult = periodic_multiplier(rho.shape[0], h, component)
    return np.fft.ifft2(np.fft.fft2(rho) * mult).real
