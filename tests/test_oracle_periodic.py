"""Pins of the oracle of the standard periodic FFT potential solver (CPU only):
the errors printed in Tables 1 and 4 of Sec. 3.1, the exact invariant
Phi_xx + Phi_yy = -(rho - mean rho), brute-force DFT sums on a tiny grid, and
planted mistakes that at least one pin must catch."""
import math

import numpy as np
import pytest

from oracle import closed_forms as C
from oracle import periodic as P
import workloads as W


def rel_linf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def table_error(kind, half, h):
    n = int(round(2 * half / h))
    x, y, _ = W.grid_2d(n, half)
    if kind == "gaussian":
        rho = W.paper_gaussian_density(n, half)
        exact = C.phi_isotropic_gaussian(x, y, math.pi, math.pi ** 2)
    else:
        rho = W.arkadiev_density(n, half)
        exact = C.phi_arkadiev(x, y)
    return rel_linf(P.phi_periodic(rho, h), exact)


def printed_close(err, printed):
    # three printed digits: half a unit of the last one, plus a little
    return abs(err - printed) <= 0.006 * printed


def test_table1_gaussian_errors(golden):
    for half, h, printed in golden("table1_gaussian_periodic_fft.txt"):
        if 2 * half / h > 2048:
            continue        # the L = 128 row needs a 4096^2 grid; its neighbours pin the 1/L^2 law
        err = table_error("gaussian", half, h)
        assert printed_close(err, printed), (half, h, err, printed)


def test_table4_arkadiev_errors(golden):
    for half, h, printed in golden("table4_arkadiev_periodic_fft.txt"):
        if 2 * half / h > 1024:
            continue
        err = table_error("arkadiev", half, h)
        assert printed_close(err, printed), (half, h, err, printed)


def test_components_sum_to_minus_the_fluctuation():
    rho = W.mixture_density(64, 8.0, W.draw_mixture(4, 4, 3.0, (0.6, 1.4)))
    s = P.phi_periodic(rho, 0.25, "xx") + P.phi_periodic(rho, 0.25, "yy")
    assert np.max(np.abs(s + (rho - rho.mean()))) < 1e-14 * rho.max()


def test_brute_force_dft_on_a_tiny_grid():
    n, h = 8, 0.7
    rng = np.random.default_rng(3)
    rho = rng.standard_normal((n, n))
    got = P.phi_periodic(rho, h)
    ref = np.zeros((n, n))
    for a in range(n):                 # y index of the output point
        for b in range(n):             # x index
            acc = 0.0
            for my in range(n):
                for mx in range(n):
                    kx = (mx if mx < n // 2 else mx - n) / (n * h)
                    ky = (my if my < n // 2 else my - n) / (n * h)
                    if kx == 0 and ky == 0:
                        continue
                    c = 0.0j
                    for yy in range(n):
                        for xx in range(n):
                            c += rho[yy, xx] * np.exp(-2j * np.pi * (mx * xx + my * yy) / n)
                    acc += (-kx * kx / (kx * kx + ky * ky)) * c * np.exp(2j * np.pi * (mx * b + my * a) / n)
            ref[a, b] = (acc / (n * n)).real
    assert np.max(np.abs(got - ref)) < 1e-12


# ---- planted mistakes ------------------------------------------------------------

def _pins_hold():
    try:
        assert printed_close(table_error("gaussian", 8, 0.25), 2.38e-3)
        assert printed_close(table_error("arkadiev", 16, 0.25), 6.24e-3)
        assert printed_close(table_error("arkadiev", 8, 0.5), 2.51e-2)
        test_components_sum_to_minus_the_fluctuation()
        return True
    except AssertionError:
        return False


def _swapped_axes(monkeypatch):
    orig = P.periodic_multiplier
    monkeypatch.setattr(P, "periodic_multiplier", lambda n, h, component="xx": orig(n, h, "yy" if component == "xx" else "xx"))


def _wrong_sign(monkeypatch):
    orig = P.periodic_multiplier
    monkeypatch.setattr(P, "periodic_multiplier", lambda n, h, component="xx": -orig(n, h, component))


def _zero_mode_kept(monkeypatch):
    orig = P.periodic_multiplier

    def mult(n, h, component="xx"):
        m = orig(n, h, component)
        m[0, 0] = -0.5
        return m
    monkeypatch.setattr(P, "periodic_multiplier", mult)


def _first_power(monkeypatch):
    def mult(n, h, component="xx"):
        k = np.fft.fftfreq(n, d=h)
        kx, ky = np.abs(k)[None, :], np.abs(k)[:, None]
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.where(kx + ky > 0, -(kx if component == "xx" else ky) / (kx + ky), 0.0)
    monkeypatch.setattr(P, "periodic_multiplier", mult)


def test_unmodified_periodic_oracle_passes_the_pins():
    assert _pins_hold()


@pytest.mark.parametrize("mutation", [_swapped_axes, _wrong_sign, _zero_mode_kept, _first_power])
def test_planted_periodic_mistake_is_caught(monkeypatch, mutation):
    mutation(monkeypatch)
    assert not _pins_hold()
