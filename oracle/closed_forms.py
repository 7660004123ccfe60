"""Closed-form potentials used to pin the oracle -- TEST INFRASTRUCTURE ONLY.

Each function gives the exact whole-space potential of eq. 4 (Sec. 1) for a
density with a known answer, independent of any discretisation:

  * isotropic Gaussian (Sec. 3.1, Example 1, generalised to any width),
  * Arkadiev's algebraically decaying density (Sec. 3.1, Example 2),
  * an axis-aligned anisotropic Gaussian through a one-dimensional integral
    (derived below), which by superposition gives the potential of |u|^2 for
    any Gaussian-mixture wave function,
  * the low-frequency part I2 of a point source (a Hankel-transform identity),
  * the 2-D Coulomb potential (multiplier 1/|k|, the Remark of Sec. 2.1) of an
    isotropic Gaussian (a Bessel-function closed form) and of an axis-aligned
    Gaussian (a one-dimensional integral), hence of any Gaussian mixture.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "phi_isotropic_gaussian",
    "phi_arkadiev",
    "phi_axis_gaussian",
    "mixture_terms",
    "phi_mixture",
    "rho_mixture_from_terms",
    "i2_point_source",
    "coulomb_isotropic_gaussian",
    "coulomb_axis_gaussian",
    "coulomb_mixture",
]


def _one_minus_one_plus_q_exp(q: np.ndarray) -> np.ndarray:
    """1 - (1 + q) e^{-q}, accurate for small q via its Taylor series
    sum_{n>=2} (-1)^n (n-1) q^n / n!."""
    q = np.asarray(q, dtype=np.float64)
    out = np.empty_like(q)
    small = q < 0.5
    big = ~small
    out[big] = -np.expm1(-q[big]) - q[big] * np.exp(-q[big])
    qs = q[small]
    term_sum = np.zeros_like(qs)
    power = qs * qs
    fact = 2.0
    for k in range(2, 30):
        if k > 2:
            power = power * qs
            fact = fact * k
        term_sum += ((-1) ** k) * (k - 1) * power / fact
    out[small] = term_sum
    return out


def phi_isotropic_gaussian(x: np.ndarray, y: np.ndarray, amplitude: float = 1.0,
                           a: float = 1.0) -> np.ndarray:
    """Phi for rho = amplitude e^{-a r^2}:

        Phi = amplitude [ -e^{-a r^2}/2 + (x^2 - y^2)/(2 a r^4) (1 - (1 + a r^2) e^{-a r^2}) ]

    With amplitude = pi, a = pi^2 this is the formula of Sec. 3.1, Example 1.
    (-kx^2/|k|^2 = -1/2 - cos(2 phi_k)/2; the cos 2 phi_k part inverts through a
    J_2 Hankel transform of the Gaussian.)  The limit at r = 0 is -amplitude/2."""
    r2 = x * x + y * y
    q = a * r2
    bracket = _one_minus_one_plus_q_exp(q)
    with np.errstate(invalid="ignore", divide="ignore"):
        aniso = np.where(r2 > 0.0, (x * x - y * y) / (2.0 * a * r2 * r2) * bracket, 0.0)
    return amplitude * (-0.5 * np.exp(-q) + aniso)


def phi_xy_isotropic_gaussian(x: np.ndarray, y: np.ndarray, amplitude: float = 1.0,
                              a: float = 1.0) -> np.ndarray:
    """Phi_xy (multiplier -kx ky/|k|^2) for rho = amplitude e^{-a r^2}:

        Phi_xy = amplitude x y (1 - (1 + a r^2) e^{-a r^2}) / (a r^4),  0 at r = 0.

    -kx ky/|k|^2 = -sin(2 phi_k)/2 is the cos(2 phi_k) part of -kx^2/|k|^2 turned
    by 45 degrees, and the transform of an isotropic density commutes with
    rotations, so the (x^2 - y^2) term of phi_isotropic_gaussian becomes 2 x y."""
    r2 = x * x + y * y
    q = a * r2
    bracket = _one_minus_one_plus_q_exp(q)
    with np.errstate(invalid="ignore", divide="ignore"):
        return amplitude * np.where(r2 > 0.0, x * y * bracket / (a * r2 * r2), 0.0)


def phi_arkadiev(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Sec. 3.1, Example 2: Phi = -2 (y^2 - (x+1)^2 + 1) / ((x+1)^2 + y^2 + 1)^2."""
    s = (x + 1.0) ** 2 + y * y + 1.0
    return -2.0 * (y * y - (x + 1.0) ** 2 + 1.0) / (s * s)


def phi_axis_gaussian(xr: np.ndarray, yr: np.ndarray, a: float, b: float,
                      component: str = "xx", step: float = 0.125,
                      umin: float = -48.0, umax: float = 48.0) -> np.ndarray:
    """Exact potential of G = exp(-X^2/a^2 - Y^2/b^2) (X, Y relative to its centre).

    From 1/|k|^2 = pi int_0^inf e^{-pi s |k|^2} ds and the Gaussian transform
    G_hat = pi a b e^{-pi^2 (a^2 kx^2 + b^2 ky^2)}, with v = s/pi:

        Phi_xx = -a b int_0^inf e^{-X^2/(a^2+v) - Y^2/(b^2+v)}
                 / sqrt((a^2+v)(b^2+v)) [1/(2(a^2+v)) - X^2/(a^2+v)^2] dv

    ("yy": swap the roles of (X, a) and (Y, b) in the bracket).  In general the
    multiplier -k_i k_j/|k|^2 maps through k_i k_j <-> -(1/(4 pi^2)) d_i d_j of
    e^{-X^2/A^2 - Y^2/B^2} to the bracket delta_ij/(2 A_i^2) - X_i X_j/(A_i^2 A_j^2),
    so "xy" has the bracket -X Y/((a^2+v)(b^2+v)).  The integral is
    taken with v = e^u and the trapezoidal rule on u in [umin, umax]: the
    integrand decays exponentially in both directions of u, so the rule
    converges geometrically (a step of 1/8 is converged to rounding).  The
    step is a power of two and umin an integer, so every node u_i is exact:
    rounded, unevenly spaced nodes would cost accuracy at the 1e-13 level."""
    xr = np.asarray(xr, dtype=np.float64)
    yr = np.asarray(yr, dtype=np.float64)
    u = umin + step * np.arange(int(round((umax - umin) / step)) + 1)
    v = np.exp(u)
    shape = xr.shape
    xf = xr.reshape(-1, 1)
    yf = yr.reshape(-1, 1)
    av = a * a + v[None, :]
    bv = b * b + v[None, :]
    expo = np.exp(-xf * xf / av - yf * yf / bv)
    if component == "xx":
        bracket = 1.0 / (2.0 * av) - xf * xf / (av * av)
    elif component == "yy":
        bracket = 1.0 / (2.0 * bv) - yf * yf / (bv * bv)
    elif component == "xy":
        bracket = -xf * yf / (av * bv)
    else:
        raise ValueError(f"unknown component {component}")
    integrand = expo / np.sqrt(av * bv) * bracket * v[None, :]   # dv = v du
    total = step * integrand.sum(axis=1)
    return (-a * b * total).reshape(shape)


def mixture_terms(cx, cy, wx, wy, phase):
    """|u|^2 for u = sum_i exp(-((x-cx_i)/wx_i)^2 - ((y-cy_i)/wy_i)^2 + i phase_i)
    as a real combination of axis-aligned Gaussians.

    g_i conj(g_j) per axis: (x-c_i)^2/w_i^2 + (x-c_j)^2/w_j^2
      = (x-m)^2/s^2 + (c_i-c_j)^2/(w_i^2+w_j^2),  1/s^2 = 1/w_i^2 + 1/w_j^2,
        m = s^2 (c_i/w_i^2 + c_j/w_j^2);
    pairs i<j appear twice with total factor 2 cos(phase_i - phase_j).
    Returns a list of (weight, mx, my, sx, sy)."""
    terms = []
    count = len(cx)
    for i in range(count):
        for j in range(i, count):
            sx2 = 1.0 / (1.0 / wx[i] ** 2 + 1.0 / wx[j] ** 2)
            sy2 = 1.0 / (1.0 / wy[i] ** 2 + 1.0 / wy[j] ** 2)
            mx = sx2 * (cx[i] / wx[i] ** 2 + cx[j] / wx[j] ** 2)
            my = sy2 * (cy[i] / wy[i] ** 2 + cy[j] / wy[j] ** 2)
            amp = math.exp(-(cx[i] - cx[j]) ** 2 / (wx[i] ** 2 + wx[j] ** 2)
                           - (cy[i] - cy[j]) ** 2 / (wy[i] ** 2 + wy[j] ** 2))
            weight = amp if i == j else 2.0 * math.cos(phase[i] - phase[j]) * amp
            terms.append((weight, mx, my, math.sqrt(sx2), math.sqrt(sy2)))
    return terms


def rho_mixture_from_terms(terms, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """sum of weight exp(-(x-mx)^2/sx^2 - (y-my)^2/sy^2) (checks the expansion)."""
    out = np.zeros(np.broadcast(x, y).shape)
    for weight, mx, my, sx, sy in terms:
        out += weight * np.exp(-((x - mx) / sx) ** 2 - ((y - my) / sy) ** 2)
    return out


def phi_mixture(terms, x: np.ndarray, y: np.ndarray, component: str = "xx") -> np.ndarray:
    """Exact potential of a Gaussian-mixture density by superposition."""
    out = np.zeros(np.broadcast(x, y).shape)
    for weight, mx, my, sx, sy in terms:
        out += weight * phi_axis_gaussian(x - mx, y - my, sx, sy, component)
    return out


def i2_point_source(x: np.ndarray, y: np.ndarray, sigma: float) -> np.ndarray:
    """Whole-plane value of -int cos^2(phi_k) e^{-|k|^2/sigma^2} e^{2 pi i k.x} dk.

    This is I2 of Sec. 2.1 (eq. 10 written in polar form, eq. 11) for a density
    with rho_hat = 1, with the disk radius taken to infinity.  With
    cos^2 = (1 + cos 2 phi)/2, E = pi^2 sigma^2 r^2 and the Hankel integrals
      int_0^inf e^{-k^2/s^2} J0(2 pi k r) k dk = s^2 e^{-E}/2,
      int_0^inf e^{-k^2/s^2} J2(2 pi k r) k dk = (1 - e^{-E})/(2 pi^2 r^2) - s^2 e^{-E}/2,
    and int_0^{2pi} cos(2 phi) e^{i z cos(phi - theta)} dphi = -2 pi J2(z) cos(2 theta):
      I2 = -(pi sigma^2/2) e^{-E}
           + pi cos(2 theta) [(1 - e^{-E})/(2 pi^2 r^2) - sigma^2 e^{-E}/2]."""
    r2 = x * x + y * y
    e_arg = math.pi ** 2 * sigma ** 2 * r2
    iso = -0.5 * math.pi * sigma ** 2 * np.exp(-e_arg)
    with np.errstate(invalid="ignore", divide="ignore"):
        cos2 = np.where(r2 > 0.0, (x * x - y * y) / r2, 0.0)
        first = np.where(r2 > 0.0, -np.expm1(-e_arg) / (2.0 * math.pi ** 2 * r2),
                         0.5 * sigma ** 2)
    aniso = math.pi * cos2 * (first - 0.5 * sigma ** 2 * np.exp(-e_arg))
    return iso + aniso


def coulomb_isotropic_gaussian(x: np.ndarray, y: np.ndarray, amplitude: float = 1.0,
                               a: float = 1.0) -> np.ndarray:
    """2-D Coulomb potential Phi = int rho(y) / |x - y| dy (Fourier multiplier
    1/|k| in the 2 pi convention of eq. 5) of rho = amplitude e^{-a r^2}:

        Phi = amplitude pi^{3/2} / sqrt(a) e^{-a r^2/2} I_0(a r^2/2).

    In polar coordinates the angular integral of 1/|x - y| against the radial
    density gives a Bessel function: with s = |y|, int_0^{2 pi} e^{2 r s cos t} dt
    = 2 pi I_0(2 r s) after completing |x - y|^2 through the Gaussian's
    Laplace representation 1/|z| = pi^{-1/2} int_0^inf t^{-1/2} e^{-t z^2} dt;
    the value at r = 0 is amplitude pi^{3/2}/sqrt(a).  scipy's exponentially
    scaled i0e(z) = e^{-z} I_0(z) serves as the Bessel function."""
    from scipy.special import i0e
    r2 = x * x + y * y
    return amplitude * math.pi ** 1.5 / math.sqrt(a) * i0e(0.5 * a * r2)


def coulomb_axis_gaussian(xr: np.ndarray, yr: np.ndarray, a: float, b: float,
                          step: float = 0.125, umin: float = -40.0, umax: float = 40.0) -> np.ndarray:
    """2-D Coulomb potential of G = exp(-X^2/a^2 - Y^2/b^2) (X, Y relative to its
    centre).  From 1/|z| = pi^{-1/2} int_0^inf t^{-1/2} e^{-t |z|^2} dt, the
    Gaussian convolution per axis int e^{-y^2/a^2} e^{-t (X-y)^2} dy =
    a sqrt(pi/(1 + a^2 t)) e^{-t X^2/(1 + a^2 t)}, and t = s^2:

        Phi = 2 sqrt(pi) a b int_0^inf e^{-s^2 X^2/(1+a^2 s^2) - s^2 Y^2/(1+b^2 s^2)}
              / sqrt((1 + a^2 s^2)(1 + b^2 s^2)) ds.

    The integral is taken with s = e^u and the trapezoidal rule on u (the
    integrand times s decays exponentially in both directions of u, so the rule
    converges geometrically; exact power-of-two step and integer ends)."""
    xr = np.asarray(xr, dtype=np.float64)
    yr = np.asarray(yr, dtype=np.float64)
    u = umin + step * np.arange(int(round((umax - umin) / step)) + 1)
    s = np.exp(u)
    s2 = (s * s)[None, :]
    shape = xr.shape
    xf = xr.reshape(-1, 1)
    yf = yr.reshape(-1, 1)
    da = 1.0 + a * a * s2
    db = 1.0 + b * b * s2
    integrand = np.exp(-s2 * xf * xf / da - s2 * yf * yf / db) / np.sqrt(da * db) * s[None, :]   # ds = s du
    total = step * integrand.sum(axis=1)
    return (2.0 * math.sqrt(math.pi) * a * b * total).reshape(shape)


def coulomb_mixture(terms, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """2-D Coulomb potential of a Gaussian-mixture density (mixture_terms) by
    superposition."""
    out = np.zeros(np.broadcast(x, y).shape)
    for weight, mx, my, sx, sy in terms:
        out += weight * coulomb_axis_gaussian(x - mx, y - my, sx, sy)
    return out
