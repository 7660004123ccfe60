"""Pins of the oracle's mixed component, multiplier -kx ky/|k|^2 (CPU only).

The Remark of Sec. 2.1 extends the split to other potentials given by their
Fourier multiplier.  -kx ky/|k|^2 is bounded, even and homogeneous of degree 0
like the DS multiplier, so only the multiplier's values change: g1 of I1 and
the angular factor cos(theta) sin(theta) of the I2 weights.  Pins:
  * two independent closed forms of its potential for a Gaussian density (a
    rotation of the DS closed form, and the 1-D integral from the Fourier
    derivative rule), which must agree, and the PDE the potential solves;
  * the split solve against the closed form, at the grid where the trapezoidal
    rule resolves the density (rounding level);
  * reflection and transposition symmetries of the discrete operator, and A = A^T;
  * the periodic solver against a brute-force DFT whose multiplier is the mean
    over the frequencies each bin stands for (on the Nyquist lines +k and -k,
    which gives 0 there: the reading both solvers take);
  * planted mistakes that the pins catch."""
import math

import numpy as np
import pytest

from oracle import closed_forms as C
from oracle import periodic as P
from oracle import split_solver as O
import workloads as W


def test_closed_forms_agree_and_vanish_on_the_axes():
    rng = np.random.default_rng(9)
    x = rng.uniform(-4, 4, 300)
    y = rng.uniform(-4, 4, 300)
    for alpha in (1.0, math.pi ** 2, 0.3):
        s = 1.0 / math.sqrt(alpha)
        iso = C.phi_xy_isotropic_gaussian(x, y, 1.0, alpha)
        axis = C.phi_axis_gaussian(x, y, s, s, "xy")
        assert np.max(np.abs(iso - axis)) < 1e-14 * max(1.0, np.max(np.abs(iso)))
    # odd in x and in y: zero on both axes and at the origin
    z = np.zeros(5)
    t = np.linspace(-2, 2, 5)
    assert np.max(np.abs(C.phi_axis_gaussian(t, z, 0.8, 1.3, "xy"))) == 0.0
    assert np.max(np.abs(C.phi_axis_gaussian(z, t, 0.8, 1.3, "xy"))) == 0.0
    assert C.phi_xy_isotropic_gaussian(np.array(0.0), np.array(0.0), 2.0, 1.0) == 0.0


def test_closed_form_solves_its_pde():
    # -Laplace(Phi_xy) = d_x d_y rho, checked by 4th-order finite differences on
    # the anisotropic closed form (rho = exp(-x^2/a^2 - y^2/b^2))
    a, b, d = 0.9, 1.4, 1e-2
    c = [-1 / 12, 4 / 3, -5 / 2, 4 / 3, -1 / 12]

    def phi(xv, yv):
        return float(C.phi_axis_gaussian(np.array([xv]), np.array([yv]), a, b, "xy")[0])

    for xv, yv in [(0.3, 0.7), (-1.1, 0.4), (1.5, -0.9), (-0.6, -1.7)]:
        lap = sum(c[i] * (phi(xv + (i - 2) * d, yv) + phi(xv, yv + (i - 2) * d)) for i in range(5)) / d ** 2
        rho = math.exp(-(xv / a) ** 2 - (yv / b) ** 2)
        dxy = (2 * xv / a ** 2) * (2 * yv / b ** 2) * rho
        assert abs(-lap - dxy) < 2e-6


def example1(n, half, comp):
    h = 2 * half / n
    x, y, _ = W.grid_2d(n, half)
    rho = W.paper_gaussian_density(n, half)
    got = O.phi(rho, O.SplitParams(n=n, h=h, n_r=64, n_theta=128, component=comp))
    return got, C.phi_xy_isotropic_gaussian(x, y, math.pi, math.pi ** 2)


def test_split_solve_matches_closed_form():
    got, ex = example1(256, 8.0, "xy")
    assert np.max(np.abs(got - ex)) < 1e-13 * np.max(np.abs(ex))


def test_mixture_against_exact_potential():
    n, half = 256, 12.0                  # h = 3/32 resolves the narrowest product term
    spec = W.draw_mixture(4, 8, 4.0, (0.6, 1.5))
    rho = W.mixture_density(n, half, spec)
    ph = O.phi(rho, O.SplitParams(n=n, h=2 * half / n, n_r=64, n_theta=128, component="xy"))
    x, y, _ = W.grid_2d(n, half)
    terms = C.mixture_terms(spec.cx, spec.cy, spec.wx, spec.wy, spec.phase)
    idx = np.random.default_rng(8).integers(0, n, size=(48, 2))
    ex = C.phi_mixture(terms, x[idx[:, 0], idx[:, 1]], y[idx[:, 0], idx[:, 1]], "xy")
    assert np.max(np.abs(ph[idx[:, 0], idx[:, 1]] - ex)) < 1e-13 * np.max(np.abs(ph))


@pytest.fixture(scope="module")
def mixed_case():
    n, half = 64, 6.0
    spec = W.draw_mixture(12, 6, 2.5, (0.5, 1.2))
    rho = W.mixture_density(n, half, spec)
    return rho, O.SplitParams(n=n, h=2 * half / n, n_r=48, n_theta=96, component="xy")


def test_reflection_flips_and_transposition_keeps(mixed_case):
    rho, p = mixed_case
    n = p.n
    rho = rho.copy()
    rho[:, 0] = 0.0                      # column x = -L has no mirror image on the grid
    idx = (-np.arange(n)) % n
    a = O.phi(rho[:, idx], p)[:, 1:]
    b = O.phi(rho, p)[:, idx][:, 1:]
    assert np.max(np.abs(a + b)) < 1e-13 * np.max(np.abs(b))
    t = O.phi(np.ascontiguousarray(rho.T), p)
    assert np.max(np.abs(t - O.phi(rho, p).T)) < 1e-13 * np.max(np.abs(t))


def test_operator_is_symmetric(mixed_case):
    rho, p = mixed_case
    g = np.random.default_rng(6).standard_normal(rho.shape)
    a = O.phi(g, p)
    assert np.max(np.abs(O.phi_transpose(g, p) - a)) < 1e-13 * np.max(np.abs(a))
    lhs = float(np.vdot(O.phi(rho, p), g))
    rhs = float(np.vdot(rho, O.phi_transpose(g, p)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_periodic_brute_force_over_representatives():
    # Every DFT bin stands for the frequencies congruent to it; on a Nyquist line
    # (index n/2) those are +k and -k.  The multiplier is taken as its mean over
    # the representatives of the bin -- for the mixed one 0 on both lines and at
    # the corner -- and the sum is done by brute force with explicit exponentials.
    n, h = 8, 0.5
    rho = np.random.default_rng(4).standard_normal((n, n))
    step = 1.0 / (n * h)

    def reps(m):
        k = (m if m < n // 2 else m - n) * step
        return (k, -k) if m == n // 2 else (k,)

    ref = np.zeros((n, n))
    xs = np.arange(n)
    for my in range(n):
        for mx in range(n):
            vals = [-kx * ky / (kx * kx + ky * ky) for kx in reps(mx) for ky in reps(my) if kx or ky]
            if not vals:
                continue
            mult = sum(vals) / len(vals)
            c = np.sum(rho * np.exp(-2j * np.pi * (mx * xs[None, :] + my * xs[:, None]) / n))
            ref += (mult * c * np.exp(2j * np.pi * (mx * xs[None, :] + my * xs[:, None]) / n)).real
    ref /= n * n
    assert np.max(np.abs(P.phi_periodic(rho, h, "xy") - ref)) < 1e-12


def test_periodic_error_falls_with_the_box():
    errs = []
    for half in (16.0, 32.0):
        h = 1 / 8
        n = int(2 * half / h)
        x, y, _ = W.grid_2d(n, half)
        ex = C.phi_xy_isotropic_gaussian(x, y, math.pi, math.pi ** 2)
        got = P.phi_periodic(W.paper_gaussian_density(n, half), h, "xy")
        errs.append(np.max(np.abs(got - ex)) / np.max(np.abs(ex)))
    # truncation to the periodic box: the error falls as 1/L^2
    assert 3.5 < errs[0] / errs[1] < 4.5


# ---- planted mistakes ------------------------------------------------------------

def _pins_hold():
    try:
        got, ex = example1(128, 8.0, "xy")
        assert np.max(np.abs(got - ex)) < 1e-7 * np.max(np.abs(ex))
        return True
    except AssertionError:
        return False


def _sign_of_i1(monkeypatch):
    orig = O.highfreq_multiplier
    monkeypatch.setattr(O, "highfreq_multiplier",
                        lambda kx, ky, s, component="xx", partition="gauss":
                        -orig(kx, ky, s, component, partition) if component == "xy"
                        else orig(kx, ky, s, component, partition))


def _abs_of_i1(monkeypatch):
    orig = O.highfreq_multiplier
    monkeypatch.setattr(O, "highfreq_multiplier",
                        lambda kx, ky, s, component="xx", partition="gauss":
                        -np.abs(orig(kx, ky, s, component, partition)) if component == "xy"
                        else orig(kx, ky, s, component, partition))


def _squared_angle_in_i2(monkeypatch):
    orig = O.polar_rule

    def rule(p):
        kx, ky, q = orig(p)
        r2 = kx * kx + ky * ky
        with np.errstate(invalid="ignore", divide="ignore"):
            fix = np.where(r2 > 0, (ky * ky) / np.where(r2 > 0, kx * ky, 1.0), 0.0)
        return kx, ky, q * fix
    monkeypatch.setattr(O, "polar_rule", rule)


def test_unmodified_oracle_passes_the_mixed_pins():
    assert _pins_hold()


@pytest.mark.parametrize("mutation", [_sign_of_i1, _abs_of_i1, _squared_angle_in_i2])
def test_planted_mixed_mistake_is_caught(monkeypatch, mutation):
    mutation(monkeypatch)
    assert not _pins_hold()
