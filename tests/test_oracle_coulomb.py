"""Pins of the oracle's 2-D Coulomb solve (multiplier 1/|k|; Sec. 2.1, Remark:
the split applies to any potential whose Fourier transform is known).

What fixes the answer independently of the oracle:
  * the closed form of an isotropic Gaussian, pi^{3/2}/sqrt(a) e^{-a r^2/2}
    I_0(a r^2/2), itself checked against a brute-force 2-D quadrature of
    int rho(y)/|x - y| dy and against the one-dimensional integral for
    axis-aligned Gaussians (two independent derivations);
  * the exact potential of a Gaussian-mixture density by superposition;
  * the closed-form sum of the polar weights, sum_j q_j = 2 pi int_0^c p(r) dr
    (the Jacobian r cancels 1/r, so a dropped or doubled factor r fails);
  * the dot-product identity with the literal transpose;
  * planted mistakes, each of which must break a pin.

Readings (listed in the design notes): the paper's partition p = e^{-|k|^2/sigma^2}
leaves a cone |k|/sigma^2 in the I1 integrand at k = 0; its error falls like
1/L at the default sigma and like 1/(sigma^2 (kappa L)^3) at fixed sigma (the
trapezoidal rule's error at a cone), and is pinned here.  The partition
erfc(|k|/sigma) keeps both integrands smooth (erf(r)/r is even and entire) and
reaches rounding."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import erf, erfc

import oracle as O
from oracle import closed_forms as C
import workloads as W


def _grid_gaussian(half, h, a=1.0):
    n = int(round(2 * half / h))
    x, y, _ = W.grid_2d(n, half)
    return n, x, y, np.exp(-a * (x * x + y * y))


def rel_linf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# --------------------------------------------------------------------------
# the closed forms themselves
# --------------------------------------------------------------------------

def test_isotropic_closed_form_against_brute_force_quadrature():
    """int e^{-a|y|^2} / |x - y| dy in polar coordinates around x (the integrand
    is bounded there: the Jacobian s cancels 1/s), adaptive quadrature."""
    for (px, py, a) in [(0.0, 0.0, 1.0), (0.7, -0.4, 1.0), (2.5, 1.0, 0.6), (0.3, 3.0, 2.0)]:
        f = lambda s, t: math.exp(-a * ((px + s * math.cos(t)) ** 2 + (py + s * math.sin(t)) ** 2))
        val, _ = integrate.dblquad(f, 0.0, 2 * math.pi, 0.0, 40.0, epsabs=1e-13, epsrel=1e-13)
        ref = C.coulomb_isotropic_gaussian(np.array([px]), np.array([py]), 1.0, a)[0]
        assert abs(val - ref) <= 1e-11 * abs(ref)
    # r = 0: pi^{3/2}/sqrt(a)
    assert abs(C.coulomb_isotropic_gaussian(np.zeros(1), np.zeros(1), 2.0, 4.0)[0] - math.pi ** 1.5) < 1e-14


def test_axis_gaussian_integral_against_isotropic_and_brute_force():
    rng = np.random.default_rng(3)
    x, y = rng.uniform(-5, 5, 40), rng.uniform(-5, 5, 40)
    for w in (0.6, 1.0, 1.7):
        assert rel_linf(C.coulomb_axis_gaussian(x, y, w, w), C.coulomb_isotropic_gaussian(x, y, 1.0, 1.0 / w ** 2)) \
            < 1e-14
    px, py, a, b = 0.9, -0.2, 0.7, 1.8
    f = lambda s, t: math.exp(-((px + s * math.cos(t)) / a) ** 2 - ((py + s * math.sin(t)) / b) ** 2)
    val, _ = integrate.dblquad(f, 0.0, 2 * math.pi, 0.0, 40.0, epsabs=1e-13, epsrel=1e-13)
    assert abs(val - C.coulomb_axis_gaussian(np.array([px]), np.array([py]), a, b)[0]) <= 1e-11 * val


# --------------------------------------------------------------------------
# the split with the erfc partition reaches rounding
# --------------------------------------------------------------------------

@pytest.mark.parametrize("half,h", [(8.0, 0.25), (8.0, 0.125), (16.0, 0.25)])
def test_erfc_partition_matches_closed_form(half, h):
    n, x, y, rho = _grid_gaussian(half, h)
    p = O.SplitParams(n=n, h=h, n_r=64, n_theta=128, component="coulomb", partition="erfc")
    err = rel_linf(O.phi(rho, p), C.coulomb_isotropic_gaussian(x, y))
    assert err < 2e-15


def test_erfc_partition_matches_mixture_closed_form():
    """C2-shaped density scaled to [-8, 8)^2: an 8-Gaussian mixture wave, rho =
    |u|^2, against the superposition of exact axis-Gaussian potentials."""
    half, n = 8.0, 128
    h = 2 * half / n
    spec = W.draw_mixture(11, 8, 3.0, (0.5, 1.5))
    rho = W.mixture_density(n, half, spec)
    p = O.SplitParams(n=n, h=h, n_r=64, n_theta=128, component="coulomb", partition="erfc")
    got = O.phi(rho, p)
    terms = C.mixture_terms(spec.cx, spec.cy, spec.wx, spec.wy, spec.phase)
    xs = O.grid_points(p)
    idx = np.random.default_rng(5).integers(0, n, size=(120, 2))
    ref = C.coulomb_mixture(terms, xs[idx[:, 1]], xs[idx[:, 0]])
    assert np.max(np.abs(got[idx[:, 0], idx[:, 1]] - ref)) <= 1e-12 * np.max(np.abs(got))


# --------------------------------------------------------------------------
# the paper's Gaussian partition: a cone-limited error, pinned as a reading
# --------------------------------------------------------------------------

def test_gauss_partition_error_falls_like_one_over_l():
    errs = []
    for half in (8.0, 16.0, 32.0):
        n, x, y, rho = _grid_gaussian(half, 0.25)
        p = O.SplitParams(n=n, h=0.25, n_r=64, n_theta=128, component="coulomb", partition="gauss")
        errs.append(rel_linf(O.phi(rho, p), C.coulomb_isotropic_gaussian(x, y)))
    assert 2.5e-4 < errs[0] < 4e-4                    # measured 3.14e-4 at L = 8
    for e0, e1 in zip(errs, errs[1:]):
        assert 1.8 < e0 / e1 < 2.2                      # halves as L doubles


def test_gauss_partition_error_at_fixed_sigma_falls_like_kappa_cubed():
    """With sigma held fixed the error is the trapezoidal rule's at the cone
    |k|/sigma^2: O(dk^3 / sigma^2), dk = 1/(kappa 2L) -- doubling kappa divides
    it by about 8, doubling sigma by about 4."""
    n, x, y, rho = _grid_gaussian(8.0, 0.25)
    ref = C.coulomb_isotropic_gaussian(x, y)
    s0, c0 = O.split_constants(O.SplitParams(n=n, h=0.25, n_r=8, n_theta=8))

    def err(kappa, fac):
        p = O.SplitParams(n=n, h=0.25, n_r=64, n_theta=128, component="coulomb", partition="gauss",
                          kappa=kappa, sigma=s0 * fac, cutoff=c0 * fac)
        return rel_linf(O.phi(rho, p), ref)
    e22, e42, e24 = err(2, 1), err(4, 1), err(2, 2)
    assert 7.0 < e22 / e42 < 10.0
    assert 3.5 < e22 / e24 < 4.5


def test_partitions_agree_to_the_cone_error():
    n, x, y, rho = _grid_gaussian(8.0, 0.25)
    pe = O.SplitParams(n=n, h=0.25, n_r=64, n_theta=128, component="coulomb", partition="erfc")
    pg = O.SplitParams(n=n, h=0.25, n_r=64, n_theta=128, component="coulomb", partition="gauss")
    a, b = O.phi(rho, pe), O.phi(rho, pg)
    assert rel_linf(b, a) < 4e-4


# --------------------------------------------------------------------------
# weights, transpose, invariants
# --------------------------------------------------------------------------

@pytest.mark.parametrize("partition", ["gauss", "erfc"])
def test_polar_weights_sum_to_the_disk_integral(partition):
    """sum_j q_j = int_{|k|<=c} p(k)/|k| dk = 2 pi int_0^c p(r) dr, closed form:
    gauss: pi^{3/2} sigma erf(c/sigma);  erfc: 2 pi sigma [z erfc z - e^{-z^2}/sqrt(pi) + 1/sqrt(pi)],
    z = c/sigma."""
    p = O.SplitParams(n=64, h=0.25, n_r=64, n_theta=16, component="coulomb", partition=partition)
    sigma, c = O.split_constants(p)
    _, _, q = O.polar_rule(p)
    z = c / sigma
    if partition == "gauss":
        ref = math.pi ** 1.5 * sigma * erf(z)
    else:
        ref = 2 * math.pi * sigma * (z * erfc(z) - math.exp(-z * z) / math.sqrt(math.pi) + 1 / math.sqrt(math.pi))
    assert abs(q.sum() - ref) <= 1e-12 * ref


@pytest.mark.parametrize("partition", ["gauss", "erfc"])
def test_transpose_dot_product_identity(partition):
    n, h = 16, 0.5
    rng = np.random.default_rng(21)
    p = O.SplitParams(n=n, h=h, n_r=24, n_theta=32, component="coulomb", partition=partition)
    for _ in range(3):
        u, v = rng.standard_normal((n, n)), rng.standard_normal((n, n))
        lhs = float(np.sum(O.phi(u, p) * v))
        rhs = float(np.sum(u * O.phi_transpose(v, p)))
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_coulomb_is_symmetric_under_the_grid_symmetries():
    """1/|k| is isotropic: transposing the density transposes the potential
    (N_theta a multiple of 4 maps the node set onto itself)."""
    n, h = 32, 0.5
    rho = np.random.default_rng(8).random((n, n))
    rho[0, :] = 0.0
    rho[:, 0] = 0.0
    p = O.SplitParams(n=n, h=h, n_r=32, n_theta=64, component="coulomb", partition="erfc")
    a = O.phi(rho, p)
    b = O.phi(rho.T.copy(), p)
    assert np.max(np.abs(a.T - b)) <= 1e-13 * np.max(np.abs(a))


def test_erfc_partition_refused_for_the_quadratic_multipliers():
    with pytest.raises(ValueError):
        O.polar_rule(O.SplitParams(n=16, h=0.5, n_r=4, n_theta=8, component="xx", partition="erfc"))


def test_jacobi_rule_refused_for_coulomb():
    """Gauss-Jacobi(0, 1) carries the Jacobian r as its weight; with 1/|k| the
    radial integrand is p(r) alone, and p(r)/r against (1 + x) converges slowly
    (1.6e-3 at 64 nodes), so the Coulomb rule is Gauss-Legendre."""
    with pytest.raises(ValueError):
        O.polar_rule(O.SplitParams(n=16, h=0.5, n_r=4, n_theta=8, component="coulomb", radial="jacobi"))


# --------------------------------------------------------------------------
# planted mistakes
# --------------------------------------------------------------------------

def _pins_hold():
    n, x, y, rho = _grid_gaussian(8.0, 0.25)
    p = O.SplitParams(n=n, h=0.25, n_r=64, n_theta=128, component="coulomb", partition="erfc")
    return rel_linf(O.phi(rho, p), C.coulomb_isotropic_gaussian(x, y)) < 2e-15


def _jacobian_not_cancelled(monkeypatch):
    orig = O.split_solver.polar_rule

    def rule(p):
        kx, ky, q = orig(p)
        return kx, ky, q * np.hypot(kx, ky)
    monkeypatch.setattr(O.split_solver, "polar_rule", rule)


def _mismatched_partition(monkeypatch):
    orig = O.split_solver.highfreq_multiplier
    monkeypatch.setattr(O.split_solver, "highfreq_multiplier",
                        lambda kx, ky, s, component="xx", partition="gauss": orig(kx, ky, s, component, "gauss"))


def _zero_mode_dropped(monkeypatch):
    orig = O.split_solver.highfreq_multiplier

    def g1(kx, ky, s, component="xx", partition="gauss"):
        out = orig(kx, ky, s, component, partition)
        out[(kx == 0) & (ky == 0)] = 0.0
        return out
    monkeypatch.setattr(O.split_solver, "highfreq_multiplier", g1)


def _squared_distance_kernel(monkeypatch):
    orig = O.split_solver.highfreq_multiplier

    def g1(kx, ky, s, component="xx", partition="gauss"):
        k = np.hypot(kx, ky)
        out = orig(kx, ky, s, component, partition)
        return np.where(k > 0, out / np.where(k > 0, k, 1.0), out)
    monkeypatch.setattr(O.split_solver, "highfreq_multiplier", g1)


@pytest.mark.parametrize("plant", [_jacobian_not_cancelled, _mismatched_partition, _zero_mode_dropped,
                                   _squared_distance_kernel])
def test_planted_coulomb_mistake_is_caught(monkeypatch, plant):
    assert _pins_hold()
    plant(monkeypatch)
    assert not _pins_hold()
