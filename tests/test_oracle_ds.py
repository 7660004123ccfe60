"""Pins of the oracle stepper (CPU only): the linear substep against the exact
evolution of a Gaussian, the nonlinear substep against the closed-form
potential of an isotropic Gaussian, mass conservation, second-order
convergence of the symmetric composition, and the reverse-mode gradient
against central finite differences."""
import math

import numpy as np
import pytest

from oracle import closed_forms as C
from oracle import ds_stepper as D
import workloads as W


def gaussian_free_flow(x, y, t, s1, s2, alpha):
    """Exact solution of i v_t = -v_xx + alpha v_yy from exp(-x^2/s1 - y^2/s2) on
    the whole plane: v_t = i v_xx + (-i alpha) v_yy is a heat equation with
    complex diffusivities D_x = i, D_y = -i alpha, whose Gaussian solution is
    sqrt(s / (s + 4 D t)) exp(-x^2 / (s + 4 D t)) in each variable."""
    ax = s1 + 4j * t
    ay = s2 - 4j * alpha * t
    return np.sqrt(s1 / ax) * np.exp(-x ** 2 / ax) * np.sqrt(s2 / ay) * np.exp(-y ** 2 / ay)


@pytest.mark.parametrize("alpha", [1.0, -1.0])
def test_linear_flow_matches_exact_gaussian_evolution(alpha):
    n, half = 128, 16.0
    p = D.DSParams(n=n, h=2 * half / n, alpha=alpha)
    x, y, _ = W.grid_2d(n, half)
    u0 = np.exp(-x ** 2 / 1.0 - y ** 2 / 2.0).astype(np.complex128)
    t = 0.3
    got = D.linear_flow(u0, p, t)
    ref = gaussian_free_flow(x, y, t, 1.0, 2.0, alpha)
    assert np.max(np.abs(got - ref)) < 1e-12
    # the flow backwards in time undoes it
    assert np.max(np.abs(D.linear_flow(got, p, -t) - u0)) < 1e-13


def test_nonlinear_phase_uses_the_potential_of_the_density():
    """v = exp(-r^2 / 2) has rho = exp(-r^2), whose Phi is known in closed form
    (Sec. 3.1 Example 1 family); the phase is t (2 beta rho + 4 beta Phi)."""
    n, half = 64, 8.0
    p = D.DSParams(n=n, h=2 * half / n, beta=0.7, n_r=32, n_theta=64)
    x, y, _ = W.grid_2d(n, half)
    v = np.exp(-(x ** 2 + y ** 2) / 2.0).astype(np.complex128)
    t = 0.05
    w = D.nonlinear_flow(v, p, t)
    rho = np.exp(-(x ** 2 + y ** 2))
    expect = v * np.exp(1j * t * (2 * 0.7 * rho + 4 * 0.7 * C.phi_isotropic_gaussian(x, y)))
    assert np.max(np.abs(w - expect)) < 1e-12
    assert np.max(np.abs(np.abs(w) - np.abs(v))) < 1e-15


def test_steps_conserve_mass():
    n, half = 32, 4.0
    p = D.DSParams(n=n, h=2 * half / n, tau=1e-2, n_r=16, n_theta=32)
    x, y, _ = W.grid_2d(n, half)
    u = np.exp(-(x ** 2 + 2 * y ** 2)).astype(np.complex128) * np.exp(0.3j * x)
    m0 = np.sum(np.abs(u) ** 2)
    for _ in range(5):
        u = D.strang_step(u, p)
        assert abs(np.sum(np.abs(u) ** 2) - m0) < 1e-13 * m0


def test_symmetric_composition_is_second_order():
    n, half = 32, 4.0
    x, y, _ = W.grid_2d(n, half)
    u0 = (np.exp(-(x ** 2 + 2 * y ** 2)) * np.exp(0.5j * x)).astype(np.complex128)
    base = dict(n=n, h=2 * half / n, alpha=1.0, beta=2.0, n_r=16, n_theta=32)
    t_end = 0.08
    ref = D.evolve(u0, D.DSParams(tau=t_end / 64, **base), 64)
    errs = [np.max(np.abs(D.evolve(u0, D.DSParams(tau=t_end / m, **base), m) - ref)) for m in (4, 8)]
    ratio = errs[0] / errs[1]
    assert 3.5 < ratio < 4.5, (errs, ratio)


def test_reverse_mode_gradient_matches_central_differences():
    n, half = 16, 4.0
    p = D.DSParams(n=n, h=2 * half / n, alpha=1.0, beta=1.5, tau=2e-2, n_r=12, n_theta=24)
    x, y, _ = W.grid_2d(n, half)
    u0 = (np.exp(-(x ** 2 + 2 * y ** 2)) * np.exp(0.4j * y)).astype(np.complex128)
    steps = 3
    loss, g = D.loss_l4_gradient(u0, p, steps)
    assert abs(loss - D.loss_l4(D.evolve(u0, p, steps), p)) < 1e-14 * loss
    rng = np.random.default_rng(7)
    eps = 1e-5
    for _ in range(4):
        d = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        fd = (D.loss_l4(D.evolve(u0 + eps * d, p, steps), p)
              - D.loss_l4(D.evolve(u0 - eps * d, p, steps), p)) / (2 * eps)
        dot = float(np.sum(np.real(np.conj(g) * d)))
        assert abs(fd - dot) <= 1e-7 * abs(dot), (fd, dot)


def test_linear_part_of_a_step_is_the_exact_flow():
    """With beta = 0 the nonlinear substep is the identity and `steps` Strang
    steps must reproduce the exact linear evolution over steps * tau."""
    n, half = 64, 8.0
    p = D.DSParams(n=n, h=2 * half / n, alpha=1.0, beta=0.0, tau=0.05, n_r=16, n_theta=32)
    x, y, _ = W.grid_2d(n, half)
    u0 = np.exp(-x ** 2 - y ** 2 / 1.5).astype(np.complex128)
    got = D.evolve(u0, p, 4)
    assert np.max(np.abs(got - gaussian_free_flow(x, y, 0.2, 1.0, 1.5, 1.0))) < 1e-12


def lump(x, y, t):
    """Arkadiev's exact solution of the H-E DS system (alpha = 1, beta = -1),
    Sec. 3.2 Example 3 case I."""
    return 2.0 * np.exp(1j * (2.0 * y + 4.0 * t)) / ((x + 1.0) ** 2 + (y + 4.0 * t) ** 2 + 1.0)


@pytest.mark.parametrize("scheme", ["strang", "yoshida4"])
@pytest.mark.parametrize("pot", ["split", "periodic"])
def test_short_time_evolution_of_the_exact_lump(scheme, pot):
    """On [-8, 8)^2 at h = 1/2 the lump's algebraic tails are cut by the box, so
    the error is about 1e-2 after T = 0.05; a sign error in alpha or beta or in
    the coupling gives 0.1 or more."""
    n, half = 32, 8.0
    x, y, h = W.grid_2d(n, half)
    p = D.DSParams(n=n, h=h, alpha=1.0, beta=-1.0, tau=0.005, n_r=32, n_theta=64, scheme=scheme, potential=pot)
    u = D.evolve(lump(x, y, 0.0), p, 10)
    ex = lump(x, y, 0.05)
    assert np.linalg.norm(u - ex) / np.linalg.norm(ex) < 0.02


def test_coefficients_default_to_the_ds_system():
    """c_local = 2 beta and c_potential = 4 beta reproduce eq. 1's nonlinear
    substep; setting them apart changes only that substep's phase."""
    n, half = 16, 4.0
    x, y, _ = W.grid_2d(n, half)
    v = (np.exp(-(x ** 2 + y ** 2) / 2) * np.exp(0.2j * x)).astype(np.complex128)
    base = dict(n=n, h=2 * half / n, beta=0.7, n_r=12, n_theta=24)
    a = D.nonlinear_flow(v, D.DSParams(**base), 0.1)
    b = D.nonlinear_flow(v, D.DSParams(c_local=1.4, c_potential=2.8, **base), 0.1)
    assert np.array_equal(a, b)
    c = D.nonlinear_flow(v, D.DSParams(c_local=1.4, c_potential=0.0, **base), 0.1)
    assert np.max(np.abs(c - v * np.exp(0.1j * 1.4 * np.abs(v) ** 2))) < 1e-15


def test_yoshida_composition_is_fourth_order():
    """A smooth field on a coarse grid keeps the step in the asymptotic regime:
    halving tau divides the error by 16 (the symmetric composition: by 4)."""
    n, half = 16, 4.0
    x, y, _ = W.grid_2d(n, half)
    u0 = (np.exp(-(x ** 2 + 2 * y ** 2) / 2) * np.exp(0.3j * x)).astype(np.complex128)
    base = dict(n=n, h=2 * half / n, alpha=1.0, beta=2.0, n_r=12, n_theta=24, scheme="yoshida4")
    t_end = 0.1
    ref = D.evolve(u0, D.DSParams(tau=t_end / 128, **base), 128)
    errs = [np.max(np.abs(D.evolve(u0, D.DSParams(tau=t_end / m, **base), m) - ref)) for m in (4, 8, 16)]
    for a, b in zip(errs, errs[1:]):
        assert 14.0 < a / b < 18.5, errs


def test_yoshida_linear_part_is_the_exact_flow():
    n, half = 64, 8.0
    p = D.DSParams(n=n, h=2 * half / n, alpha=-1.0, beta=0.0, tau=0.05, n_r=16, n_theta=32, scheme="yoshida4")
    x, y, _ = W.grid_2d(n, half)
    got = D.evolve(np.exp(-x ** 2 - y ** 2 / 1.5).astype(np.complex128), p, 4)
    assert np.max(np.abs(got - gaussian_free_flow(x, y, 0.2, 1.0, 1.5, -1.0))) < 1e-12


@pytest.mark.parametrize("scheme,pot,coef", [("yoshida4", "split", None), ("strang", "periodic", None),
                                            ("yoshida4", "periodic", None), ("strang", "split", (1.0, -1.0))])
def test_gradient_of_other_schemes_matches_central_differences(scheme, pot, coef):
    n, half = 16, 4.0
    cl, cp = coef if coef else (None, None)
    p = D.DSParams(n=n, h=2 * half / n, alpha=-1.0, beta=1.5, tau=2e-2, n_r=12, n_theta=24, scheme=scheme,
                   potential=pot, c_local=cl, c_potential=cp)
    x, y, _ = W.grid_2d(n, half)
    u0 = (np.exp(-(x ** 2 + 2 * y ** 2)) * np.exp(0.4j * y)).astype(np.complex128)
    steps = 2
    loss, g = D.loss_l4_gradient(u0, p, steps)
    assert abs(loss - D.loss_l4(D.evolve(u0, p, steps), p)) < 1e-14 * loss
    rng = np.random.default_rng(11)
    eps = 1e-5
    for _ in range(3):
        d = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        fd = (D.loss_l4(D.evolve(u0 + eps * d, p, steps), p)
              - D.loss_l4(D.evolve(u0 - eps * d, p, steps), p)) / (2 * eps)
        dot = float(np.sum(np.real(np.conj(g) * d)))
        assert abs(fd - dot) <= 1e-7 * abs(dot), (fd, dot)


# ---- the pins above must catch plausible mistakes in the stepper -------------

def _ds_pins_hold():
    checks = []
    for fn in (lambda: test_linear_flow_matches_exact_gaussian_evolution(1.0),
               lambda: test_linear_flow_matches_exact_gaussian_evolution(-1.0),
               test_nonlinear_phase_uses_the_potential_of_the_density,
               test_symmetric_composition_is_second_order,
               test_linear_part_of_a_step_is_the_exact_flow,
               test_reverse_mode_gradient_matches_central_differences,
               test_yoshida_composition_is_fourth_order,
               lambda: test_short_time_evolution_of_the_exact_lump("yoshida4", "split"),
               lambda: test_gradient_of_other_schemes_matches_central_differences("yoshida4", "split", None)):
        try:
            fn()
            checks.append(True)
        except AssertionError:
            checks.append(False)
    return all(checks)


def _alpha_sign(monkeypatch):
    orig = D.linear_flow
    monkeypatch.setattr(D, "linear_flow", lambda u, p, t: orig(u, D.DSParams(**{**p.__dict__, "alpha": -p.alpha}), t))


def _no_two_pi(monkeypatch):
    def flow(u, p, t):
        k = np.fft.fftfreq(p.n, d=p.h)
        mult = np.exp(-1j * ((k ** 2)[None, :] - p.alpha * (k ** 2)[:, None]) * t)
        return np.fft.ifft2(np.fft.fft2(u) * mult)
    monkeypatch.setattr(D, "linear_flow", flow)


def _half_local_term(monkeypatch):
    orig = D.nonlinear_phase
    monkeypatch.setattr(D, "nonlinear_phase",
                        lambda v, p, t: orig(v, p, t) - t * p.beta * np.abs(v) ** 2)


def _lie_composition(monkeypatch):
    monkeypatch.setattr(D, "strang_step", lambda u, p: D.nonlinear_flow(D.linear_flow(u, p, p.tau), p, p.tau))


def _full_linear_substeps(monkeypatch):
    monkeypatch.setattr(D, "strang_step", lambda u, p: D.linear_flow(
        D.nonlinear_flow(D.linear_flow(u, p, p.tau), p, p.tau), p, p.tau))


def _adj_local_only(g, v, p, t):
    """The adjoint of the nonlinear substep with the potential's A^T term dropped."""
    ph = D.nonlinear_phase(v, p, t)
    w = v * np.exp(1j * ph)
    s = -np.imag(np.conj(g) * w)
    return g * np.exp(-1j * ph) + 2.0 * (t * p.coefficients()[0] * s) * v


def _adjoint_without_potential_term(monkeypatch):
    monkeypatch.setattr(D, "nonlinear_flow_adjoint", _adj_local_only)


def _strang_weights_in_yoshida(monkeypatch):
    orig = D.composition
    monkeypatch.setattr(D, "composition", lambda scheme: orig("strang") if scheme == "yoshida4" else orig(scheme))


def _yoshida_middle_sign(monkeypatch):
    orig = D.composition

    def comp(scheme):
        lin, nonlin = orig(scheme)
        if scheme == "yoshida4":
            nonlin = [nonlin[0], -nonlin[1], nonlin[2]]
        return lin, nonlin
    monkeypatch.setattr(D, "composition", comp)


def _beta_sign(monkeypatch):
    orig = D.nonlinear_phase
    monkeypatch.setattr(D, "nonlinear_phase", lambda v, p, t: -orig(v, p, t))


def test_unmodified_stepper_passes_the_pins():
    assert _ds_pins_hold()


@pytest.mark.parametrize("mutation", [_alpha_sign, _no_two_pi, _half_local_term, _lie_composition,
                                      _full_linear_substeps, _adjoint_without_potential_term,
                                      _strang_weights_in_yoshida, _yoshida_middle_sign, _beta_sign])
def test_planted_stepper_mistake_is_caught(monkeypatch, mutation):
    mutation(monkeypatch)
    assert not _ds_pins_hold()
