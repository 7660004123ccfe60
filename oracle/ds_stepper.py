"""FP64 oracle of the split-step time integration of the DS system -- TEST
INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU leg).

The DS system (Sec. 1, eqs. 1-2), in the 2 pi Fourier convention of eq. 5:

    i u_t = -u_xx + alpha u_yy - 2 beta |u|^2 u - 4 beta Phi u,
    -Laplace(Phi) = d_xx |u|^2,  i.e.  Phi_hat = -kx^2/|k|^2 rho_hat,  rho = |u|^2,

on a periodic box (Sec. 2.3).  The time-splitting method (Sec. 2.3) splits the
right-hand side into

    A: i v_t = (-d_xx + alpha d_yy) v      exact in Fourier space:
       v_hat(t + s) = v_hat(t) exp(-i 4 pi^2 (kx^2 - alpha ky^2) s);
    B: i w_t = (-2 beta |w|^2 - 4 beta Phi) w   |w| is constant in time, so with
       Phi frozen at the density of the substep's input (Sec. 2.3)
       w(t + s) = w(t) exp(i s (2 beta rho + 4 beta Phi)).
The coefficients of rho and Phi in the phase, c_local = 2 beta and
c_potential = 4 beta for eq. 1, can be set apart: the E-E system of Sec. 3.3,
i u_t = -(u_xx + u_yy) + chi |u|^2 u + gamma Phi u, has alpha = -1,
c_local = -chi, c_potential = -gamma.

One step of length tau is a composition of these flows (Sec. 2.3):
  "strang"    e^{A tau/2} e^{B tau} e^{A tau/2}, second order;
  "yoshida4"  e^{A a1 tau} e^{B b1 tau} e^{A a2 tau} e^{B b2 tau} e^{A a3 tau}
              e^{B b3 tau} e^{A a4 tau} with b1 = b3 = 1/(2 - 2^(1/3)),
              b2 = -2^(1/3) b3, a1 = a4 = b3/2, a2 = a3 = (b3 + b2)/2 (the
              fourth-order composition the paper uses for its experiments).
Phi comes from the split quadrature of split_solver.phi ("split"), so the
oracle stepper is exactly what the GPU stepper computes with direct sums in
place of NUFFTs, or from the standard periodic FFT solver ("periodic", the
paper's baseline).

Gradients of a real loss J(u) of the complex field u are represented as the
complex field g = dJ/dRe(u) + i dJ/dIm(u), so that the first-order change is
dJ = Re sum(conj(g) du).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .periodic import phi_periodic
from .split_solver import SplitParams, phi, phi_transpose

__all__ = [
    "DSParams",
    "linear_flow",
    "nonlinear_phase",
    "nonlinear_flow",
    "strang_step",
    "composition",
    "step",
    "evolve",
    "loss_l4",
    "loss_l4_gradient",
    "nonlinear_flow_adjoint",
]


@dataclasses.dataclass(frozen=True)
class DSParams:
    """Grid (n points of spacing h on [-L, L)^2, L = n h / 2), coefficients
    alpha, beta of eq. 1, time step tau, polar node counts of the Phi solve,
    the composition ("strang" or "yoshida4") and the potential solver ("split"
    or "periodic")."""
    n: int
    h: float
    alpha: float = 1.0
    beta: float = 1.0
    tau: float = 1e-3
    n_r: int = 64
    n_theta: int = 128
    scheme: str = "strang"
    potential: str = "split"
    c_local: float | None = None        # default 2 beta
    c_potential: float | None = None    # default 4 beta

    def coefficients(self) -> tuple[float, float]:
        cl = 2.0 * self.beta if self.c_local is None else self.c_local
        cp = 4.0 * self.beta if self.c_potential is None else self.c_potential
        return cl, cp

    def split(self) -> SplitParams:
        return SplitParams(n=self.n, h=self.h, n_r=self.n_r, n_theta=self.n_theta)


def _wavenumbers(p: DSParams) -> np.ndarray:
    """k = m / (n h), m in FFT order: the Fourier modes of the periodic box."""
    return np.fft.fftfreq(p.n, d=p.h)


def linear_flow(u: np.ndarray, p: DSParams, t: float) -> np.ndarray:
    """Exact flow of i v_t = (-d_xx + alpha d_yy) v over time t (Sec. 2.3,
    first substep), via the discrete Fourier transform of the periodic box;
    axis 1 is x, axis 0 is y."""
    k = _wavenumbers(p)
    kx2 = (k ** 2)[None, :]
    ky2 = (k ** 2)[:, None]
    mult = np.exp(-1j * 4.0 * math.pi ** 2 * (kx2 - p.alpha * ky2) * t)
    return np.fft.ifft2(np.fft.fft2(u) * mult)


def potential(rho: np.ndarray, p: DSParams) -> np.ndarray:
    """Phi[rho] by the stepper's potential solver."""
    if p.potential == "periodic":
        return phi_periodic(rho, p.h)
    return phi(rho, p.split())


def potential_transpose(g: np.ndarray, p: DSParams) -> np.ndarray:
    """The transpose of the potential operator (the periodic one is symmetric)."""
    if p.potential == "periodic":
        return phi_periodic(g, p.h)
    return phi_transpose(g, p.split())


def nonlinear_phase(v: np.ndarray, p: DSParams, t: float) -> np.ndarray:
    """t (c_local rho + c_potential Phi[rho]) with rho = |v|^2 (Sec. 2.3, second
    substep; c_local = 2 beta, c_potential = 4 beta for eq. 1)."""
    rho = np.abs(v) ** 2
    cl, cp = p.coefficients()
    return t * (cl * rho + cp * potential(rho, p))


def nonlinear_flow(v: np.ndarray, p: DSParams, t: float) -> np.ndarray:
    """Exact pointwise flow of the second substep over time t."""
    return v * np.exp(1j * nonlinear_phase(v, p, t))


def composition(scheme: str):
    """(linear times, nonlinear times) of one step as fractions of tau:
    e^{A c_0 tau} e^{B d_0 tau} e^{A c_1 tau} ... e^{B d_{K-1} tau} e^{A c_K tau}."""
    if scheme == "strang":
        return [0.5, 0.5], [1.0]
    if scheme == "yoshida4":
        b1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
        b2 = -(2.0 ** (1.0 / 3.0)) * b1
        a1 = 0.5 * b1
        a2 = 0.5 * (b1 + b2)
        return [a1, a2, a2, a1], [b1, b2, b1]
    raise ValueError(f"unknown scheme {scheme}")


def step(u: np.ndarray, p: DSParams) -> np.ndarray:
    """One step of the scheme's composition."""
    lin, nonlin = composition(p.scheme)
    u = linear_flow(u, p, lin[0] * p.tau)
    for d, c in zip(nonlin, lin[1:]):
        u = nonlinear_flow(u, p, d * p.tau)
        u = linear_flow(u, p, c * p.tau)
    return u


def strang_step(u: np.ndarray, p: DSParams) -> np.ndarray:
    """e^{A tau/2} e^{B tau} e^{A tau/2} u."""
    v = linear_flow(u, p, 0.5 * p.tau)
    w = nonlinear_flow(v, p, p.tau)
    return linear_flow(w, p, 0.5 * p.tau)


def evolve(u0: np.ndarray, p: DSParams, steps: int) -> np.ndarray:
    u = np.asarray(u0, dtype=np.complex128)
    for _ in range(steps):
        u = strang_step(u, p) if p.scheme == "strang" else step(u, p)
    return u


def loss_l4(u: np.ndarray, p: DSParams) -> float:
    """J(u) = h^2 sum |u|^4 (the quadrature of the L4 norm to the fourth power)."""
    return float(p.h ** 2 * np.sum(np.abs(u) ** 4))


def nonlinear_flow_adjoint(g: np.ndarray, v: np.ndarray, p: DSParams, t: float) -> np.ndarray:
    """Gradient with respect to the input v of the second substep, given the
    gradient g with respect to its output w = v e^{i phi(v)},
    phi = t (c_l rho + c_p A rho), rho = |v|^2, A the Phi operator.

    dw = e^{i phi} dv + i w dphi, so Re sum conj(g) dw = Re sum conj(g e^{-i phi}) dv
    + sum s dphi with s = Re(conj(g) i w) = -Im(conj(g) w); sum s dphi =
    sum r drho with r = t (c_l s + c_p A^T s); drho = 2 Re(conj(v) dv), so
    the gradient is g e^{-i phi} + 2 r v."""
    ph = nonlinear_phase(v, p, t)
    w = v * np.exp(1j * ph)
    s = -np.imag(np.conj(g) * w)
    cl, cp = p.coefficients()
    r = t * (cl * s + cp * potential_transpose(s, p))
    return g * np.exp(-1j * ph) + 2.0 * r * v


def loss_l4_gradient(u0: np.ndarray, p: DSParams, steps: int) -> tuple[float, np.ndarray]:
    """J(evolve(u0)) and its gradient with respect to u0, by the reverse pass
    through every substep with all intermediate states kept.  The linear
    substep is unitary with a unit-modulus Fourier multiplier, so its adjoint
    is the same flow backwards in time."""
    lin, nonlin = composition(p.scheme)
    u = np.asarray(u0, dtype=np.complex128)
    vs = []
    for _ in range(steps):
        u = linear_flow(u, p, lin[0] * p.tau)
        for d, c in zip(nonlin, lin[1:]):
            vs.append(u)
            u = linear_flow(nonlinear_flow(u, p, d * p.tau), p, c * p.tau)
    loss = loss_l4(u, p)
    g = 4.0 * p.h ** 2 * np.abs(u) ** 2 * u        # dJ/dRe u + i dJ/dIm u
    k = len(vs)
    for _ in range(steps):
        for d, c in zip(reversed(nonlin), reversed(lin[1:])):
            k -= 1
            g = linear_flow(g, p, -c * p.tau)
            g = nonlinear_flow_adjoint(g, vs[k], p, d * p.tau)
        g = linear_flow(g, p, -lin[0] * p.tau)
    return loss, g
