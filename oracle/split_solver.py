"""Plain FP64 oracle for the split potential solve -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the CPU-baseline leg of the benchmark may use
this module.  The GPU library never imports, links or calls it.

What it computes (Mauser, Stimming, Zhang, "A novel nonlocal potential solver
based on nonuniform FFT ..."):

    Phi(x) = int -kx^2/|k|^2 rho_hat(k) e^{2 pi i k.x} dk            (Sec. 1, eq. 4)
    rho_hat(k) = int rho(x) e^{-2 pi i k.x} dx                       (Sec. 1, eq. 5)

split with the partition p(k) = exp(-|k|^2 / sigma^2) into

    I1 = high-frequency part, integrand continuous and zero at k = 0,
         evaluated with the trapezoidal rule on a zero-padded box     (Sec. 2.1, eq. 9)
    I2 = low-frequency part on the disk |k| <= c, polar coordinates,
         radial Gauss rule x azimuthal trapezoid rule                 (Sec. 2.1, eqs. 10-12)

The oracle evaluates every discrete sum exactly as it is defined: I1 through
the 2-D DFT of the zero-padded density (numpy.fft serves as the DFT, a library
step), rho_hat at the polar nodes and the I2 sum as direct nonuniform DFT sums
(Sec. 2.1: the direct evaluation costs O(N N_r N_theta)), written as separable
matrix products.  No NUFFT appears here: the GPU path's NUFFTs approximate
exactly these direct sums.

Readings of points the paper leaves open (each is listed in the design notes):
  * 2 pi convention of eqs. 4-5 throughout; the Fourier grid of I1 is
    k_m = m / (M h), m in FFT order (-M/2 .. M/2-1), on the padded box of
    side M = kappa N (or any M >= 2N given as pad_side; kappa = M / N).
  * the grid holds N points x_n = -L + n h, n = 0..N-1 (periodic box).
  * g1(0) = 0, its limit (Sec. 2.1: the I1 integrand vanishes at the origin).
  * sigma = sqrt(lambda) / (2 pi (kappa-1) L), lambda = ln(1/eps_s): the
    periodic images of the I1 kernel on the padded box are suppressed to
    eps_s (Sec. 2.1 only fixes sigma = O(1/P)); c = sqrt(lambda) sigma, so that
    p(c) = eps_s (Sec. 2.1: c is a multiple of sigma).
  * radial rule: Gauss-Legendre on [0, c] with the polar Jacobian r folded into
    the weight (the paper names a Gauss-Jacobi rule; both integrate the same
    smooth radial integrand); azimuthal rule: trapezoid theta_j = 2 pi j/N_theta.
  * I2 is complex in eq. 12; its real part is taken (the imaginary part is
    zero by the k -> -k symmetry of the node set when N_theta is even).
  * the 2-D Coulomb multiplier 1/|k| (the Remark of Sec. 2.1): the paper's
    Gaussian partition leaves a cone in the I1 integrand at k = 0 (its error is
    pinned as a measured reading); the partition erfc(|k|/sigma) keeps the I1
    integrand erf(|k|/sigma)/|k| smooth and the polar one erfc(r/sigma) smooth in
    r, as Sec. 2.1 asks of the two parts.  The radial rule is Gauss-Legendre:
    1/|k| cancels the Jacobian r.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "SplitParams",
    "split_constants",
    "grid_points",
    "highfreq_multiplier",
    "i1_padded_fft",
    "i1_padded_dft_matrix",
    "polar_nodes_weights",
    "polar_rule",
    "type2_direct",
    "type1_direct",
    "i2_direct",
    "phi",
    "phi_parts",
    "phi_transpose",
]


@dataclasses.dataclass(frozen=True)
class SplitParams:
    """Discretisation of one potential solve.

    n        grid points per side (even), spacing h, box [-L, L)^2 with L = n h / 2
    n_r      radial Gauss nodes;  n_theta  azimuthal trapezoid nodes
    kappa    zero-padding factor of the I1 box (Sec. 2.1: kappa >= 2)
    pad_side side M of the zero-padded I1 box in grid points (None: kappa n).
             Sec. 2.1 pads the box by a factor kappa >= 2; any M >= 2n is such
             a box, with kappa = M / n, which also fixes the default sigma
    sigma    partition width; cutoff  disk radius c (None -> default reading)
    eps_split   target size of the neglected tails (defines the defaults)
    component   "xx": multiplier -kx^2/|k|^2 (the DS potential, eq. 4);
                "yy": -ky^2/|k|^2 (its companion; the two sum to -1);
                "xy": -kx ky/|k|^2 (the mixed one; with the other two the whole
                tensor -k_i k_j/|k|^2, another potential the Remark of Sec. 2.1
                covers: bounded, even and of degree 0, so the split carries over
                with only the multiplier's values changed);
                "coulomb": 1/|k|, the 2-D Coulomb potential int rho(y)/|x-y| dy
                (the Remark of Sec. 2.1: any multiplier with a known transform)
    partition   the partition function p(k) of Sec. 2.1 (eq. 8): "gauss" is the
                paper's e^{-|k|^2/sigma^2}; "erfc" is erfc(|k|/sigma), for
                "coulomb" only.  Sec. 2.1 asks that the I1 integrand be smooth
                in Cartesian and the I2 integrand in polar coordinates.  With
                1/|k| the Gaussian p leaves (1 - p)/|k| ~ |k|/sigma^2 at k = 0, a
                cone the padded trapezoidal rule resolves only to an error that
                falls like 1/((kappa-1) L); erf(|k|/sigma)/|k| is an even entire
                function of |k| (smooth at 0), and p(r) r / r = erfc(r/sigma) is
                smooth in r, so both parts keep spectral accuracy.  None: "gauss"
    """
    n: int
    h: float
    n_r: int
    n_theta: int
    kappa: int = 2
    sigma: float | None = None
    cutoff: float | None = None
    eps_split: float = 1e-16
    component: str = "xx"
    radial: str = "legendre"    # or "jacobi": Gauss-Jacobi(0, 1), the weight r built in
    pad_side: int | None = None
    partition: str | None = None

    @property
    def partition_kind(self) -> str:
        kind = "gauss" if self.partition is None else self.partition
        if kind not in ("gauss", "erfc"):
            raise ValueError(f"unknown partition {kind!r}")
        if kind == "erfc" and self.component != "coulomb":
            raise ValueError("the erfc partition is for the Coulomb multiplier 1/|k| only")
        return kind

    @property
    def half_width(self) -> float:
        return 0.5 * self.n * self.h

    @property
    def padded_side(self) -> int:
        """Side M of the zero-padded I1 box (Sec. 2.1 asks for kappa >= 2)."""
        m = self.kappa * self.n if self.pad_side is None else int(self.pad_side)
        if m < 2 * self.n:
            raise ValueError(f"the padded box must be at least twice the grid (kappa >= 2): {m} < 2 * {self.n}")
        return m

    @property
    def kappa_eff(self) -> float:
        """The padding factor of the box actually used, M / n."""
        return self.padded_side / self.n


def split_constants(p: SplitParams) -> tuple[float, float]:
    """(sigma, c) following the reading of Sec. 2.1 stated in the module doc."""
    lam = math.log(1.0 / p.eps_split)
    sigma = p.sigma
    if sigma is None:
        sigma = math.sqrt(lam) / (2.0 * math.pi * (p.kappa_eff - 1) * p.half_width)
    c = p.cutoff
    if c is None:
        c = math.sqrt(lam) * sigma
    return sigma, c


def grid_points(p: SplitParams) -> np.ndarray:
    """x_n = -L + n h, n = 0..N-1 (Sec. 2.1 and Sec. 3)."""
    return -p.half_width + p.h * np.arange(p.n, dtype=np.float64)


def highfreq_multiplier(kx: np.ndarray, ky: np.ndarray, sigma: float,
                        component: str = "xx", partition: str = "gauss") -> np.ndarray:
    """g1(k) = -(k_a^2/|k|^2) (1 - exp(-|k|^2/sigma^2)), g1(0) = 0.

    The integrand of I1 (Sec. 2.1, eq. 9) divided by rho_hat.  1 - e^{-s} is
    formed as -expm1(-s) so that it keeps full relative accuracy near k = 0.
    "coulomb": (1 - p(k))/|k|, i.e. (1 - e^{-|k|^2/sigma^2})/|k| (0 at k = 0) or,
    with the erfc partition, erf(|k|/sigma)/|k| (2/(sigma sqrt(pi)) at k = 0)."""
    k2 = kx * kx + ky * ky
    if component == "coulomb":
        from scipy.special import erf
        kk = np.sqrt(k2)
        out = np.zeros_like(k2)
        nz = k2 > 0.0
        if partition == "erfc":
            out[nz] = erf(kk[nz] / sigma) / kk[nz]
            out[~nz] = 2.0 / (sigma * math.sqrt(math.pi))
        else:
            out[nz] = (-np.expm1(-k2[nz] / sigma ** 2)) / kk[nz]
        return out
    num = {"xx": kx * kx, "yy": ky * ky, "xy": kx * ky}[component]
    out = np.zeros_like(k2)
    nz = k2 > 0.0
    out[nz] = -(num[nz] / k2[nz]) * (-np.expm1(-k2[nz] / sigma ** 2))
    return out


def _padded_frequencies(p: SplitParams) -> tuple[np.ndarray, np.ndarray]:
    m_side = p.padded_side
    k = np.fft.fftfreq(m_side, d=p.h)           # k_m = m / (M h)
    ky, kx = np.meshgrid(k, k, indexing="ij")
    return kx, ky


def padded_multiplier(p: SplitParams) -> np.ndarray:
    """g1 on the padded DFT grid.  The mixed multiplier is odd in each of kx,
    ky, and on the Nyquist lines (index M / 2) one DFT bin stands for +k
    and -k; the bin takes the mean of the multiplier over them, which is 0 (also
    at the corner, where numpy's negative representatives alone would give
    -1/2)."""
    sigma, _ = split_constants(p)
    kx, ky = _padded_frequencies(p)
    g1 = highfreq_multiplier(kx, ky, sigma, p.component, p.partition_kind)
    if p.component == "xy":
        nyq = p.padded_side // 2
        g1[nyq, :] = 0.0
        g1[:, nyq] = 0.0
    return g1


def i1_padded_fft(rho: np.ndarray, p: SplitParams) -> np.ndarray:
    """I1 on the grid (Sec. 2.1, eq. 9 by the trapezoidal rule on the padded box).

    rho_hat(k_m) ~ h^2 sum_n rho_n e^{-2 pi i k_m.x_n} (trapezoid on B_p), the k
    integral ~ (Delta k)^2 sum_m with Delta k = 1/(M h) (M = kappa N the padded
    side); the phases only involve x_n - x_n', so the density sits at the corner
    of the padded array:
        I1_n = Re[M^-2 sum_m g1(k_m) S_m e^{+2 pi i m.n/M}],
        S_m  = sum_n P_n e^{-2 pi i m.n/M},  P = zero-padded rho."""
    m_side = p.padded_side
    padded = np.zeros((m_side, m_side), dtype=np.float64)
    padded[: p.n, : p.n] = rho
    s_hat = np.fft.fft2(padded)                      # S_m (unnormalised DFT)
    g1 = padded_multiplier(p)
    full = np.fft.ifft2(g1 * s_hat)                  # includes M^-2
    return full[: p.n, : p.n].real.copy()


def i1_padded_dft_matrix(rho: np.ndarray, p: SplitParams) -> np.ndarray:
    """Same sum as i1_padded_fft written with explicit DFT matrices (small N only)."""
    m_side = p.padded_side
    m = np.arange(m_side)
    n = np.arange(p.n)
    fwd = np.exp(-2j * np.pi * np.outer(m, n) / m_side)    # [m][n]
    s_hat = fwd @ rho @ fwd.T                               # S[m_y][m_x]
    g1 = padded_multiplier(p)
    inv = np.exp(+2j * np.pi * np.outer(n, m) / m_side)    # [n][m]
    return (inv @ (g1 * s_hat) @ inv.T).real / m_side ** 2


def polar_nodes_weights(p: SplitParams):
    """Radial nodes/weights on [0, c] for int_0^c f(r) r dr and the azimuthal
    trapezoid nodes/weight (Sec. 2.1, eq. 12).

    "legendre": Gauss-Legendre with the Jacobian r folded into the weight,
    r_i = c (1 + x_i)/2, weight (c/2) w_i r_i.  "jacobi": the Gauss-Jacobi rule
    for the weight (1 + x) on [-1, 1] (the rule the paper names), which has the
    Jacobian as its weight function: r_i = c (1 + x_i)/2, weight (c/2)^2 w_i.
    scipy's Gauss-Jacobi routine serves as the rule."""
    _, c = split_constants(p)
    if p.radial == "jacobi":
        from scipy.special import roots_jacobi
        x, w = roots_jacobi(p.n_r, 0.0, 1.0)
        r = 0.5 * c * (1.0 + x)
        w_r = 0.25 * c * c * w
    else:
        x, w = np.polynomial.legendre.leggauss(p.n_r)
        r = 0.5 * c * (1.0 + x)
        w_r = 0.5 * c * w * r
    theta = 2.0 * np.pi * np.arange(p.n_theta) / p.n_theta
    w_t = 2.0 * np.pi / p.n_theta
    return r, w_r, theta, w_t


def polar_rule(p: SplitParams):
    """Polar nodes k_j and the I2 weights q_j (Sec. 2.1, eqs. 11-12).

    Radial Gauss-Legendre on [0, c]: r_i = c (1 + x_i)/2 with weight
    (c/2) w_i r_i (the Jacobian r of eq. 11 folded in); azimuthal trapezoid
    theta_j = 2 pi j / N_theta with weight 2 pi / N_theta.  The I2 weight is
        q_ij = -omega_i omega_j cos^2(theta_j) p(k_ij)      ("xx")
    (sin^2 for "yy", cos sin for "xy": the multiplier on the unit circle).
    "coulomb": the multiplier 1/r cancels the Jacobian r, so
        q_ij = (omega_i / r_i) omega_j p(r_i)
    with p the Gaussian or erfc(r/sigma) (see SplitParams).  Returns flattened
    arrays kx, ky, q of length N_r N_theta in (radial-major, angle-minor) order."""
    partition = p.partition_kind           # validates the partition for the component
    sigma, _ = split_constants(p)
    r, w_r, theta, w_t = polar_nodes_weights(p)
    rr, tt = np.meshgrid(r, theta, indexing="ij")
    kx = rr * np.cos(tt)
    ky = rr * np.sin(tt)
    if p.component == "coulomb":
        if p.radial == "jacobi":
            # the rule's weight is the Jacobian, which 1/r cancels: the integrand
            # p(r) is smooth, and p(r)/r against the weight (1 + x) is not
            raise ValueError("the Coulomb multiplier cancels the Jacobian: use the Gauss-Legendre radial rule")
        if partition == "erfc":
            from scipy.special import erfc
            part = erfc(rr / sigma)
        else:
            part = np.exp(-(rr ** 2) / sigma ** 2)
        q = (w_r[:, None] / rr * w_t) * part
        return kx.ravel(), ky.ravel(), q.ravel()
    ang = {"xx": np.cos(tt) ** 2, "yy": np.sin(tt) ** 2, "xy": np.cos(tt) * np.sin(tt)}[p.component]
    q = -(w_r[:, None] * w_t) * ang * np.exp(-(rr ** 2) / sigma ** 2)
    return kx.ravel(), ky.ravel(), q.ravel()


def type2_direct(rho: np.ndarray, h: float, xs: np.ndarray, kx: np.ndarray,
                 ky: np.ndarray) -> np.ndarray:
    """rho_hat(k_j) = h^2 sum_{n1,n2} rho[n2][n1] e^{-2 pi i (kx_j x_n1 + ky_j y_n2)}.

    The trapezoidal rule applied to eq. 5 on the grid, at nonuniform k_j: the
    type-2 sum of Sec. 2.2, eq. 16, evaluated directly (separably)."""
    ex = np.exp(-2j * np.pi * np.outer(kx, xs))      # [j][n1]
    ey = np.exp(-2j * np.pi * np.outer(ky, xs))      # [j][n2]
    partial = ex @ rho.T                              # [j][n2] = sum_n1 ex rho[n2][n1]
    return h * h * np.einsum("jn,jn->j", partial, ey)


def type1_direct(coef: np.ndarray, xs: np.ndarray, kx: np.ndarray,
                 ky: np.ndarray) -> np.ndarray:
    """f[n2][n1] = sum_j coef_j e^{+2 pi i (kx_j x_n1 + ky_j y_n2)} (complex).

    The type-1 sum of Sec. 2.2, eq. 15, evaluated directly (separably)."""
    ex = np.exp(2j * np.pi * np.outer(kx, xs))       # [j][n1]
    ey = np.exp(2j * np.pi * np.outer(ky, xs))       # [j][n2]
    return (ey.T * coef[None, :]) @ ex                # [n2][n1]


def i2_direct(rho: np.ndarray, p: SplitParams, return_imag: bool = False):
    """I2 on the grid: eq. 12 with rho_hat from the direct type-2 sum."""
    kx, ky, q = polar_rule(p)
    xs = grid_points(p)
    rho_hat = type2_direct(rho, p.h, xs, kx, ky)
    field = type1_direct(q * rho_hat, xs, kx, ky)
    if return_imag:
        return field.real.copy(), field.imag.copy()
    return field.real.copy()


def phi_parts(rho: np.ndarray, p: SplitParams) -> dict:
    """I1, I2, Phi = I1 + I2 (Sec. 2.1, eq. 8) and max |Im I2| as a diagnostic."""
    rho = np.asarray(rho, dtype=np.float64)
    if rho.shape != (p.n, p.n):
        raise ValueError(f"rho must be {p.n}x{p.n}, got {rho.shape}")
    i1 = i1_padded_fft(rho, p)
    i2, i2_imag = i2_direct(rho, p, return_imag=True)
    return {"i1": i1, "i2": i2, "phi": i1 + i2,
            "max_imag_i2": float(np.max(np.abs(i2_imag)))}


def phi(rho: np.ndarray, p: SplitParams) -> np.ndarray:
    """Phi on the grid, FP64."""
    return phi_parts(rho, p)["phi"]


def phi_transpose(g: np.ndarray, p: SplitParams) -> np.ndarray:
    """The literal transpose A^T g of the discrete operator A: rho -> Phi.

    Not assumed symmetric: every factor is transposed and the order reversed.
      A1 = crop . F^-1 . diag(g1) . F . pad  ->  A1^T = crop . F . diag(g1) . F^-1 . pad
           (the 2-D DFT matrix F and F^-1 are symmetric; crop^T = pad).
      A2 = Re(E1 . diag(q) . E2), E2[j][n] = h^2 e^{-2 pi i k_j.x_n},
           E1[n][j] = e^{+2 pi i k_j.x_n}  ->  A2^T = Re(E2^T . diag(q) . E1^T).
    For a complex matrix C acting on real vectors, (Re C)^T = Re(C^T)."""
    g = np.asarray(g, dtype=np.float64)
    m_side = p.padded_side
    padded = np.zeros((m_side, m_side), dtype=np.float64)
    padded[: p.n, : p.n] = g
    g1 = padded_multiplier(p)
    a1t = np.fft.fft2(g1 * np.fft.ifft2(padded))[: p.n, : p.n].real

    nkx, nky, q = polar_rule(p)
    xs = grid_points(p)
    e1t_x = np.exp(2j * np.pi * np.outer(nkx, xs))   # E1^T[j][n] factors
    e1t_y = np.exp(2j * np.pi * np.outer(nky, xs))
    s = np.einsum("jn,jn->j", e1t_x @ g.T, e1t_y)    # (E1^T g)_j
    e2t_x = np.exp(-2j * np.pi * np.outer(nkx, xs))  # E2^T[n][j] = h^2 e^{-...}
    e2t_y = np.exp(-2j * np.pi * np.outer(nky, xs))
    a2t = (p.h * p.h) * ((e2t_y.T * (q * s)[None, :]) @ e2t_x)
    return a1t + a2t.real
